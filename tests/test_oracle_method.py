"""Pins for the oracle's implementation of the method (paper Secs. "Pauli
Basis Tensor Network", "Gate Update", "Correlation Function via Belief
Propagation"; Algorithm "Gate update"; Eqs. bp, damping, bethe_raw, ze, bethe).

Each test fixes the oracle against something other than itself: the dense
2^N route, exact contraction, a closed form, a textbook property, or a value
printed in the paper.
"""

import math

import numpy as np
import pytest

from oracle import dense, contract
from oracle.lattice import Lattice
from oracle.network import Config, OperatorNetwork, pseudo_sqrt, mode_product, bethe_log_sign
from oracle.run import layer, run, measurement_record


def _run_net(cfg, nsteps):
    net = OperatorNetwork(cfg)
    out = []
    for _ in range(nsteps):
        layer(net)
        out.append(measurement_record(net))
    return net, out


@pytest.mark.parametrize("Lx,Ly,n", [(2, 2, 3), (4, 1, 4), (3, 2, 2), (3, 3, 2)])
def test_untruncated_network_equals_dense_operator(Lx, Ly, n):
    # while nothing is truncated the network represents the Trotter-evolved
    # operator exactly: every Pauli coefficient matches the dense route
    cfg = Config(Lx=Lx, Ly=Ly, chi_max=256, dt=0.13, J=0.8, h=1.1, bp_tol=1e-9)
    net = OperatorNetwork(cfg)
    ops = dense.trotter_operators(net.lat, cfg.J, cfg.h, cfg.dt, n)
    for k in range(1, n + 1):
        layer(net)
        assert net.layer_gate_err < 1e-20
        a_net = contract.all_coefficients(net)
        a_dense = dense.pauli_coefficients(ops[k], net.lat.n_sites)
        assert np.max(np.abs(a_net - a_dense)) < 1e-12
        assert abs(np.sum(a_net ** 2) - 1.0) < 1e-12          # Tr[O^2]/2^N = 1


def test_chain_bethe_is_exact_and_gauge_norm_is_one():
    # on a tree BP is exact (Sec. "Pauli Basis Tensor Network": "On a tree
    # this gauge is exact"), so the method reproduces the dense C(t)
    lat = Lattice(5, 1)
    Cd, _ = dense.trotter_trajectory(lat, 1.0, 1.0, 0.05, 12)
    net, recs = _run_net(Config(Lx=5, Ly=1, chi_max=64, dt=0.05), 12)
    C = np.array([r["C"] for r in recs])
    assert np.max(np.abs(C - Cd[1:])) < 1e-12
    assert all(abs(r["bethe_norm"] - 1.0) < 1e-9 for r in recs)


def test_first_step_is_a_star_so_bethe_is_exact():
    # after one layer only the bonds at the centre have chi > 1: the
    # non-trivial part of the network is a tree and Bethe is exact
    for L in (3, 4):
        lat = Lattice(L, L)
        Cd, _ = dense.trotter_trajectory(lat, 1.0, 1.0, 0.1, 1) if L == 3 else (None, None)
        net, recs = _run_net(Config(Lx=L, Ly=L, chi_max=32, dt=0.1), 1)
        exact = contract.pinned_contraction(net)
        assert abs(recs[0]["C"] - exact) < 1e-12
        if Cd is not None:
            assert abs(recs[0]["C"] - Cd[1]) < 1e-12
        big = [b for b in range(lat.n_bonds) if net.chi[b] > 1]
        c = lat.centre()
        for b in big:
            assert c in lat.bonds[b][:2]


def test_single_loop_bethe_equals_dominant_eigenvalue():
    # 2x2 is one loop: BP converges to the dominant eigenvector of the loop
    # transfer matrix and the Bethe value is its eigenvalue, while the exact
    # contraction is the trace (Weiss 2000, loopy belief propagation)
    net, recs = _run_net(Config(Lx=2, Ly=2, chi_max=64, dt=0.2, J=1.0, h=1.0, bp_tol=1e-13,
                                 meas_max_sweeps=5000), 4)
    lat = net.lat
    T = net.pinned()
    # loop 0 -(b0)- 1 -(b3)- 3 -(b1)- 2 -(b2)- 0 ; build transfer matrices
    # site 0 legs (D=b2, R=b0); site 1 (D=b3, L=b0); site 3 (U=b3, L=b1); site 2 (U=b2, R=b1)
    A0 = T[0].T          # site 0 axes (D=b2, R=b0) -> [b0, b2]
    A1 = T[1].T          # site 1 axes (D=b3, L=b0) -> [b0, b3]
    A3 = T[3]            # site 3 axes (U=b3, L=b1) -> [b3, b1]
    A2 = T[2].T          # site 2 axes (U=b2, R=b1) -> [b1, b2]
    Mloop = (A0.T @ A1 @ A3 @ A2).T   # transfer b2 -> b0 -> b3 -> b1 -> b2
    ev = np.linalg.eigvals(Mloop)
    dom = ev[np.argmax(np.abs(ev))]
    assert abs(dom.imag) < 1e-12
    assert abs(np.sum(ev).real - contract.pinned_contraction(net)) < 1e-12
    assert abs(recs[-1]["C"] - dom.real) < 1e-9


def test_truncated_gate_is_eckart_young():
    # with truncation, the QR -> bond matrix -> SVD route finds the singular
    # values of the whole gated two-site block (environment absorbed)
    cfg = Config(Lx=3, Ly=2, chi_max=3, dt=0.3, J=1.0, h=0.7)
    net = OperatorNetwork(cfg)
    for _ in range(2):
        layer(net)
    lat = net.lat
    b = lat.bonds_of_colour(0)[0]
    v1, v2, _ = lat.bonds[b]
    cvs = []
    for v in (v1, v2):
        T = net.psi[v]
        for pos, (_, u, be) in enumerate(lat.legs[v]):
            if be != b:
                S, _, _ = pseudo_sqrt(net.incoming(be, v), cfg.eps_pinv)
                T = mode_product(T, S, pos)
        cvs.append((T, lat.leg_position(v, b)))
    (T1, c1), (T2, c2) = cvs
    # full block: contract the cut, apply the gate, flatten (env1, p1) x (env2, p2)
    T1m = np.moveaxis(T1, c1, -1)          # [env1.., p1, cut]
    T2m = np.moveaxis(T2, c2, -1)
    blk = np.tensordot(T1m, T2m, axes=([-1], [-1]))   # [env1.., p1, env2.., p2]
    n1 = T1m.ndim - 1
    blk = np.moveaxis(blk, n1 - 1, -1)                 # [env1.., env2.., p2, p1]
    blk = np.moveaxis(blk, -2, -1)                     # [env1.., env2.., p1, p2]
    G4 = net.G2.reshape(4, 4, 4, 4)
    blk = np.tensordot(blk, G4, axes=([-2, -1], [2, 3]))   # [env1.., env2.., e1, e2]
    nenv1 = n1 - 1
    blk = np.moveaxis(blk, -2, nenv1)                   # [env1.., e1, env2.., e2]
    m1 = int(np.prod(blk.shape[:nenv1 + 1]))
    s_full = np.linalg.svd(blk.reshape(m1, -1), compute_uv=False)
    r = net.gate_update(b)
    k = len(r["s"])
    assert np.allclose(r["s"], s_full[:k], rtol=1e-12, atol=1e-14 * s_full[0])
    kept = r["chi_new"]
    assert abs(r["gate_err"] - np.sum(s_full[kept:] ** 2) / np.sum(s_full ** 2)) < 1e-13


def test_gauge_transform_on_a_bond_leaves_C_unchanged():
    cfg = Config(Lx=3, Ly=3, chi_max=6, dt=0.1)
    net, recs = _run_net(cfg, 5)
    C0 = recs[-1]["C"]
    lat = net.lat
    b = 5
    v1, v2, _ = lat.bonds[b]
    chi = net.chi[b]
    rng = np.random.default_rng(3)
    G, _ = np.linalg.qr(rng.standard_normal((chi, chi)))
    p1, p2 = lat.leg_position(v1, b), lat.leg_position(v2, b)
    net.psi[v1] = mode_product(net.psi[v1], G, p1)
    net.psi[v2] = mode_product(net.psi[v2], G, p2)
    assert abs(net.measure()["C"] - C0) < 1e-10


def test_lightcone():
    # each layer spreads the support by at most one site: X components of
    # the centre commute with later XX gates only beyond distance n
    cfg = Config(Lx=5, Ly=5, chi_max=8, dt=0.1)
    net = OperatorNetwork(cfg)
    lat = net.lat
    c = lat.centre()
    for n in range(1, 4):
        layer(net)
        for v in range(lat.n_sites):
            if lat.manhattan(v, c) > n:
                assert net.psi[v].shape == (1,) * lat.degree(v) + (4,)
                e = net.psi[v].reshape(4)
                assert abs(abs(e[0]) - 1.0) < 1e-14 and np.max(np.abs(e[1:])) < 1e-14
        for b, (v1, v2, _) in enumerate(lat.bonds):
            if min(lat.manhattan(v1, c), lat.manhattan(v2, c)) >= n:
                assert net.chi[b] == 1


def test_method_sign_invariance_under_truncation():
    base, _ = run(Config(Lx=3, Ly=3, chi_max=4, dt=0.1, bp_tol=1e-12), 8)
    for J, h in [(-1.0, 1.0), (1.0, -1.0)]:
        other, _ = run(Config(Lx=3, Ly=3, chi_max=4, dt=0.1, J=J, h=h, bp_tol=1e-12), 8)
        for a, bb in zip(base, other):
            assert abs(a["C"] - bb["C"]) < 1e-9


def test_bethe_log_sign_matches_direct_product():
    rng = np.random.default_rng(11)
    vs = list(rng.standard_normal(9) * 3)
    ze = list(rng.standard_normal(12))
    C, la, s, f = bethe_log_sign(vs, ze)
    direct = np.prod(vs) / np.prod(ze)
    assert abs(C - direct) <= 1e-14 * abs(direct)
    assert bethe_log_sign([0.0, 1.0], [1.0])[0] == 0.0


def test_paper_printed_universal_value_5x5():
    # Table "C(t) at selected Trotter layers for n x n grids": C(0.9) = 0.140
    # on every grid from 5x5 upwards (h = J = -1, dt = 0.1).  Fixture:
    # tests/golden/paper_ct_grids.txt
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "paper_ct_grids.txt")
    rows = [l.split() for l in open(path) if l.strip() and not l.startswith("#")]
    target = {(int(r[0]), float(r[1])): float(r[2]) for r in rows}[(5, 0.9)]
    net, recs = _run_net(Config(Lx=5, Ly=5, chi_max=8, dt=0.1, J=-1.0, h=-1.0,
                                 bp_tol=1e-6, bp_max_sweeps=100), 9)
    assert abs(recs[-1]["C"] - target) <= 5e-4 + 2e-4


def test_trap_rule_on_records():
    # the remediation rule (paper, trap remediation steps 1-3) on plain records
    from oracle.network import Config, FLAG_TRAP_CANDIDATE
    from oracle.run import trap_verified, retry_alpha
    prev = dict(C=0.0622, gate_err=0.0054, flags=0)
    trapped = dict(C=0.0066, gate_err=0.0067, flags=FLAG_TRAP_CANDIDATE)
    assert trap_verified(trapped, prev)
    assert not trap_verified(dict(trapped, flags=0), prev)               # not a candidate
    assert not trap_verified(dict(trapped, C=0.04), prev)                # drop of less than half
    assert not trap_verified(dict(trapped, gate_err=0.02), prev)         # gate error grew in proportion
    assert not trap_verified(trapped, None)
    assert retry_alpha(Config(bp_alpha=0.5)) == 0.8
    assert retry_alpha(Config(bp_alpha=1.0)) == 0.5
    assert retry_alpha(Config(bp_alpha=0.5, trap_alpha=0.7)) == 0.7


def test_trap_retry_golden_continues_the_smooth_sequence():
    # the oracle run with the remediation (written by tests/golden/make_golden.py):
    # layers 1..39 equal the run without it, and the retried layer 40 lies on
    # the quadratic continuation of layers 37..39 (the trapped value does not)
    import json, os
    here = os.path.join(os.path.dirname(__file__), "golden")
    a = json.load(open(os.path.join(here, "oracle_4x4_chi20.json")))["records"]
    b = json.load(open(os.path.join(here, "oracle_4x4_chi20_trap_retry.json")))["records"]
    for k in range(40):
        assert abs(a[k]["C"] - b[k]["C"]) <= 1e-13
    c37, c38, c39 = (b[k]["C"] for k in (37, 38, 39))
    extrap = 3 * c39 - 3 * c38 + c37
    assert abs(b[40]["C"] - extrap) < 2e-3
    assert abs(a[40]["C"] - extrap) > 0.05
    assert b[40]["flags"] & (1 << 9)
