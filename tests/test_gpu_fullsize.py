"""Parity at the full per-bond size of the 10x10 chi = 100 workload: one
interior-interior bond update on a seeded saturated state (every bond at the
two sites has chi = 100, so both site tensors hold 4 * 100^4 entries and the
QR blocks are 10^6 x 400).  The oracle computes the same update; the test
compares the full Vidal spectrum, the bond dimension and sampled entries of
both new site tensors."""

import numpy as np
import pytest

from paper_2606_30985_amd import inputs
from tests.gpu_util import load_hpt, max_rel

pytestmark = pytest.mark.gpu


def _state(cfg, chi, seed):
    from oracle.network import Config, OperatorNetwork
    net = OperatorNetwork(Config(**cfg))
    lat = net.lat
    b0 = [b for b, (v1, v2, _) in enumerate(lat.bonds) if (v1, v2) == (5, 6)][0]
    big = {b for b, (v1, v2, _) in enumerate(lat.bonds) if {v1, v2} & {5, 6}}
    net.chi = [chi if b in big else 1 for b in range(lat.n_bonds)]
    for v in range(lat.n_sites):
        net.psi[v] = np.array(inputs.site_tensor(seed + v, net.site_dims(v)))
    for b in range(lat.n_bonds):
        c = net.chi[b]
        net.M[b] = [inputs.env_message(7 * seed + 2 * b, c), inputs.env_message(7 * seed + 2 * b + 1, c)]
    return net, b0


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-9), ("fp32", 2e-4)])
def test_interior_bond_update_chi100(precision, tol):
    hpt = load_hpt()
    cfg = dict(Lx=4, Ly=4, chi_max=100, dt=0.05, J=1.0, h=1.0)
    net, b = _state(cfg, 100, 3)
    sim = hpt.Simulator(precision=precision, **cfg)
    for v in range(net.lat.n_sites):
        sim.set_site(v, net.psi[v])
    for bb in range(net.lat.n_bonds):
        for d in range(2):
            sim.set_message(bb, d, net.M[bb][d])
    v1, v2, _ = net.lat.bonds[b]
    r = net.gate_update(b)
    sim.apply_bond(b)
    assert sim.chi(b) == r["chi_new"] == 100
    assert max_rel(sim.spectrum(b), r["lam"]) < tol
    rng = np.random.default_rng(0)
    for v in (v1, v2):
        got = sim.get_site(v).ravel(order="F")
        ref = net.psi[v].ravel(order="F")
        idx = rng.integers(0, ref.size, 20000)
        assert max_rel(got[idx], ref[idx]) < tol * 10
        assert abs(np.linalg.norm(got) / np.linalg.norm(ref) - 1) < tol * 10
    sim.close()
