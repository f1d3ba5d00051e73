"""Failure handling through the C ABI (every condition forced from the host;
every kernel still runs to its normal end): non-finite host data refused,
BP budgets exhausted (flags, outputs still written), the R-core SVD sweep cap
reached (flag), and the Householder fallback of a rank-deficient CholeskyQR2
block (flag, result equal to the oracle's Householder route)."""

import numpy as np
import pytest

from paper_2606_30985_amd import inputs
from tests.gpu_util import load_hpt, copy_state, max_rel

pytestmark = pytest.mark.gpu


def test_non_finite_host_data_is_refused():
    hpt = load_hpt()
    sim = hpt.Simulator(Lx=3, Ly=3, chi_max=8)
    sim.step(2)
    before = sim.get_site(4)
    bad = before.copy()
    bad.flat[3] = np.nan
    with pytest.raises(hpt.HptError) as e:
        sim.set_site(4, bad)
    assert e.value.code == -4
    assert np.array_equal(sim.get_site(4), before)
    M = sim.get_message(1, 0)
    Mb = M.copy()
    Mb[0, 0] = np.inf
    with pytest.raises(hpt.HptError) as e:
        sim.set_message(1, 0, Mb)
    assert e.value.code == -4
    assert np.array_equal(sim.get_message(1, 0), M)
    sim.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_bp_budget_exhausted_sets_flags(precision):
    hpt = load_hpt()
    sim = hpt.Simulator(Lx=3, Ly=3, chi_max=8, bp_max_sweeps=1, meas_max_sweeps=1, precision=precision)
    sim.step(3)
    m = sim.measure()
    assert m["flags"] & hpt.FLAGS["BP_NOT_CONVERGED_GAUGE"]
    assert m["flags"] & hpt.FLAGS["BP_NOT_CONVERGED_MEAS"]
    assert m["gauge_sweeps"] == 1 and m["meas_sweeps"] == 1
    assert np.isfinite(m["C"])
    sim.close()


def test_svd_sweep_cap_sets_flag():
    hpt = load_hpt()
    flag = hpt.FLAGS["SVD_NOT_CONVERGED"]
    capped = hpt.Simulator(Lx=4, Ly=4, chi_max=20, svd_max_sweeps=1)
    free = hpt.Simulator(Lx=4, Ly=4, chi_max=20)
    hit = []
    for _ in range(14):
        capped.step(1)
        free.step(1)
        mc, mf = capped.measure(), free.measure()
        hit.append(bool(mc["flags"] & flag))
        assert not mf["flags"] & flag
        assert np.isfinite(mc["C"])
    assert any(hit)
    capped.close()
    free.close()


def test_rank_deficient_block_falls_back_to_householder():
    # 3x3, every bond at chi 4: the centre's blocks are 64 x 16 (CholeskyQR2
    # route).  Two Pauli columns of the centre made equal for cut index 0 make
    # every block of that site rank-deficient, whatever the environment.
    hpt = load_hpt()
    from oracle.network import Config, OperatorNetwork
    cfg = dict(Lx=3, Ly=3, chi_max=5, dt=0.1, J=0.9, h=1.2)
    net = OperatorNetwork(Config(**cfg))
    net.chi = [4] * net.lat.n_bonds
    for v in range(net.lat.n_sites):
        net.psi[v] = np.array(inputs.site_tensor(300 + v, net.site_dims(v)))
    T = net.psi[4]
    T[..., 2] = T[..., 1]
    for b in range(net.lat.n_bonds):
        net.M[b] = [inputs.env_message(700 + 2 * b, 4), inputs.env_message(701 + 2 * b, 4)]
    sim = hpt.Simulator(**cfg)
    copy_state(net, sim)
    b = [k for k, (v1, v2, _) in enumerate(net.lat.bonds) if (v1, v2) == (3, 4)][0]
    r = net.gate_update(b)
    sim.apply_bond(b)
    m = sim.measure()
    assert m["flags"] & hpt.FLAGS["QR_FALLBACK"]
    assert sim.chi(b) == r["chi_new"]
    assert max_rel(sim.spectrum(b), r["lam"]) < 1e-12
    for v in (3, 4):
        assert max_rel(sim.get_site(v), net.psi[v]) < 1e-10, v
    sim.close()


def test_arena_too_small_is_refused_before_any_launch():
    hpt = load_hpt()
    import ctypes
    cfg = hpt.make_config(Lx=3, Ly=3, chi_max=8)
    need = hpt.required_bytes(cfg)
    import torch
    buf = torch.empty(need, dtype=torch.uint8, device="cuda")
    h = ctypes.c_void_p()
    assert hpt.lib.hpt_create(ctypes.byref(cfg), ctypes.c_void_p(buf.data_ptr()), need - 256, None,
                              ctypes.byref(h)) == -2
    assert not h.value
