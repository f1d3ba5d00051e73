"""hpt_pauli_weights (the per-site non-identity Pauli weight n(r, t) of Sec.
"Operator Spreading and Lightcone Saturation" and the spreading measures of
Sec. "Spatial operator spreading") against the oracle, layer by layer from
the same t = 0 state: the FP64 form at 1e-9, the FP32 form at 2e-5 (its
gauge BP stops at 1e-6, its cutoff is 1e-7 and its site tensors are
float32; the FP32 C(t) bound on these layers is 5e-5), the t = 0 state
exactly, and the C4 symmetry of n on a 5x5 grid (centre (2, 2)) at every
layer, truncated ones included."""

import numpy as np
import pytest

from tests.gpu_util import load_hpt

pytestmark = pytest.mark.gpu


def _oracle_weights(cfg, n):
    from oracle.network import Config, OperatorNetwork, spreading_stats
    from oracle.run import layer
    net = OperatorNetwork(Config(**cfg))
    out = [(net.pauli_weights(), spreading_stats(net.pauli_weights(), net.lat, net.centre))]
    for _ in range(n):
        layer(net)
        w = net.pauli_weights()
        out.append((w, spreading_stats(w, net.lat, net.centre)))
    return out


@pytest.mark.parametrize("geom,chi,n,precision,tol", [((3, 3), 8, 6, "fp64", 1e-9), ((4, 4), 20, 6, "fp64", 1e-9),
                                                      ((5, 1), 16, 6, "fp64", 1e-9), ((4, 4), 20, 6, "fp32", 2e-5)])
def test_weights_match_oracle(geom, chi, n, precision, tol):
    hpt = load_hpt()
    cfg = dict(Lx=geom[0], Ly=geom[1], chi_max=chi, dt=0.1, J=1.0, h=0.8, bp_tol=1e-11)
    ref = _oracle_weights(cfg, n)
    extra = dict(precision=precision)
    if precision == "fp32":
        extra.update(bp_tol=1e-6)
    sim = hpt.Simulator(**{**cfg, **extra})
    for k in range(n + 1):
        if k:
            sim.step(1)
        w, st = sim.pauli_weights()
        if k == 0:
            assert np.array_equal(w, ref[0][0])
        assert np.max(np.abs(w - ref[k][0])) <= tol, (k, w, ref[k][0])
        assert np.max(np.abs(np.array(st) - np.array(ref[k][1]))) <= 10 * tol
    sim.close()


def test_c4_symmetry_on_5x5():
    hpt = load_hpt()
    sim = hpt.Simulator(Lx=5, Ly=5, chi_max=24, dt=0.1, J=1.0, h=1.0, bp_tol=1e-11)
    rot = [(4 - v // 5) + 5 * (v % 5) for v in range(25)]   # 90 degrees about (2, 2): (x, y) -> (4 - y, x)
    assert sorted(rot) == list(range(25)) and rot[12] == 12
    for k in range(8):
        sim.step(1)
        w, (r1, r2, sf) = sim.pauli_weights()
        assert np.max(np.abs(w - w[rot])) <= 1e-6 * np.max(w), (k, w)
        assert 0.0 < sf <= 1.0 and 0.0 < r1 <= 4.0 and r1 <= r2 * np.sqrt(2.0) + 1e-12
    sim.close()
