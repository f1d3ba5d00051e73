"""Row-by-row GPU parity against the CPU oracle on the same seeded inputs,
through the C ABI: field half-step (a1), one bond update (a2-a7), gauge BP
(a8), measurement BP + Bethe (a9), and the device permutation."""

import itertools

import numpy as np
import pytest

from paper_2606_30985_amd import inputs
from tests.gpu_util import load_hpt, copy_state, max_rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hpt():
    return load_hpt()


def _oracle_net(cfg, layers):
    from oracle.network import Config, OperatorNetwork
    from oracle.run import layer
    net = OperatorNetwork(Config(**cfg))
    for _ in range(layers):
        layer(net)
    return net


def _synthetic_net(cfg, chi, seed):
    """Saturated synthetic state: every bond at chi, Gaussian site tensors,
    PSD environment messages with a decaying spectrum."""
    from oracle.network import Config, OperatorNetwork
    net = OperatorNetwork(Config(**cfg))
    lat = net.lat
    net.chi = [chi] * lat.n_bonds
    for v in range(lat.n_sites):
        net.psi[v] = np.array(inputs.site_tensor(seed + v, net.site_dims(v)))
    for b in range(lat.n_bonds):
        net.M[b] = [inputs.env_message(1000 * seed + 2 * b, chi), inputs.env_message(1000 * seed + 2 * b + 1, chi)]
    return net


# ---------------------------------------------------------------------------
@pytest.mark.parametrize("dtype", ["float64", "float32"])
def test_permute_bit_exact(hpt, dtype):
    import torch
    rng = np.random.default_rng(0)
    cases = [((7, 5, 3, 4), None), ((1, 9, 6, 4), None), ((33, 70, 5, 4), None), ((100, 3, 17, 2, 4), None),
             ((5, 6), None), ((2, 3, 4, 5, 6), None), ((64, 65, 4), None), ((1, 130, 129, 4), None)]
    for dims, _ in cases:
        nd = len(dims)
        for perm in itertools.permutations(range(nd)):
            if nd == 5 and rng.random() < 0.8:
                continue
            x = rng.standard_normal(int(np.prod(dims))).astype(dtype)
            src = torch.from_numpy(x).cuda()
            dst = torch.empty_like(src)
            # column-major dims: the flat buffer is the Fortran order of `dims`
            hpt.permute(src.view(*dims[::-1]).permute(*range(nd - 1, -1, -1)), dst, perm)
            torch.cuda.synchronize()
            ref = np.transpose(x.reshape(dims, order="F"), perm).ravel(order="F")
            got = dst.cpu().numpy()
            assert np.array_equal(got.view(np.uint8), ref.view(np.uint8)), (dims, perm)


def test_field_half_step(hpt):
    cfg = dict(Lx=3, Ly=2, chi_max=6, dt=0.13, J=0.7, h=1.3)
    net = _synthetic_net(cfg, 3, 5)
    sim = hpt.Simulator(**cfg)
    copy_state(net, sim)
    net.apply_field()
    sim.apply_field()
    for v in range(net.lat.n_sites):
        assert max_rel(sim.get_site(v), net.psi[v]) < 1e-15
    sim.close()


@pytest.mark.parametrize("geom,chi,qr", [((3, 3), 4, "adaptive"), ((3, 3), 6, "adaptive"), ((4, 3), 5, "householder"),
                                          ((2, 2), 3, "adaptive"), ((5, 1), 4, "adaptive"), ((3, 3), 8, "adaptive")])
def test_bond_update_synthetic(hpt, geom, chi, qr):
    Lx, Ly = geom
    cfg = dict(Lx=Lx, Ly=Ly, chi_max=chi + 1, dt=0.11, J=1.1, h=0.9)
    net = _synthetic_net(cfg, chi, 17)
    sim = hpt.Simulator(qr_mode=qr, **cfg)
    copy_state(net, sim)
    for b in range(net.lat.n_bonds):
        v1, v2, _ = net.lat.bonds[b]
        r = net.gate_update(b)
        sim.apply_bond(b)
        assert sim.chi(b) == r["chi_new"]
        assert max_rel(sim.spectrum(b), r["lam"]) < 1e-12
        for v in (v1, v2):
            assert max_rel(sim.get_site(v), net.psi[v]) < 1e-10, (b, v)
        for d in range(2):
            assert max_rel(sim.get_message(b, d), net.M[b][d]) < 1e-12
    sim.close()


def test_bond_update_physical_state(hpt):
    cfg = dict(Lx=3, Ly=3, chi_max=6, dt=0.1)
    net = _oracle_net(cfg, 4)
    sim = hpt.Simulator(**cfg)
    copy_state(net, sim)
    for c in range(4):
        for b in net.lat.bonds_of_colour(c):
            r = net.gate_update(b)
            sim.apply_bond(b)
            assert sim.chi(b) == r["chi_new"]
            v1, v2, _ = net.lat.bonds[b]
            for v in (v1, v2):
                assert max_rel(sim.get_site(v), net.psi[v]) < 1e-10
    sim.close()


@pytest.mark.parametrize("geom,chi", [((3, 3), 4), ((4, 2), 3), ((6, 1), 5)])
def test_gauge_bp_matches_oracle(hpt, geom, chi):
    cfg = dict(Lx=geom[0], Ly=geom[1], chi_max=chi, dt=0.1, bp_tol=1e-11)
    net = _synthetic_net(cfg, chi, 29)
    sim = hpt.Simulator(**cfg)
    copy_state(net, sim)
    sw_o, de_o = net.gauge_bp()
    sw_g, de_g = sim.gauge_bp()
    assert sw_g == sw_o
    for b in range(net.lat.n_bonds):
        for d in range(2):
            assert max_rel(sim.get_message(b, d), net.M[b][d]) < 1e-9
    sim.close()


@pytest.mark.parametrize("geom,chi", [((3, 3), 4), ((2, 3), 3), ((5, 1), 6)])
def test_measurement_matches_oracle(hpt, geom, chi):
    cfg = dict(Lx=geom[0], Ly=geom[1], chi_max=chi, dt=0.1, bp_tol=1e-12)
    net = _oracle_net(cfg, 3)
    sim = hpt.Simulator(**cfg)
    copy_state(net, sim)
    r = net.measure()
    m = sim.measure()
    assert abs(m["C"] - r["C"]) <= 1e-12 * max(1.0, abs(r["C"]))
    assert m["meas_sweeps"] == r["meas_sweeps"]
    for b in range(net.lat.n_bonds):
        for d in range(2):
            assert max_rel(sim.get_meas_message(b, d), net.meas_messages[b][d]) < 1e-10
    sim.close()
