"""Parity at the full per-bond size of the 10x10 chi = 100 workload: one
interior-interior bond update on the seeded saturated state of
tests/fullsize_case.py (both site tensors hold 4 * 100^4 entries, the QR blocks
are 10^6 x 400).  The expected values were written by the CPU oracle
(tests/golden/make_golden.py oracle_bond_4x4_chi100, several minutes of CPU):
the full Vidal spectrum, the bond dimension, the gate error, the per-leg
marginals (sum of squares over all other indices, every leg) and sampled
entries and norms of both new site tensors."""

import json
import os
import sys
import time

import numpy as np
import pytest

from tests import fullsize_case as fc
from tests.gpu_util import load_hpt, max_rel

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "oracle_bond_4x4_chi100.json")


@pytest.fixture(scope="module")
def case():
    with open(GOLDEN) as f:
        ref = json.load(f)
    assert ref["config"] == fc.CFG and ref["seed"] == fc.SEED
    t0 = time.perf_counter()
    net, b = fc.state()
    print(f"\n# seeded chi=100 state generated in {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    assert b == ref["bond"]
    return net, b, ref


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-9), ("fp32", 2e-4)])
def test_interior_bond_update_chi100(precision, tol, case):
    hpt = load_hpt()
    net, b, ref = case
    sim = hpt.Simulator(precision=precision, **fc.CFG)
    for v in range(net.lat.n_sites):
        sim.set_site(v, net.psi[v])
    for bb in range(net.lat.n_bonds):
        for d in range(2):
            sim.set_message(bb, d, net.M[bb][d])
    t0 = time.perf_counter()
    sim.apply_bond(b)
    print(f"# {precision} bond update done ({time.perf_counter() - t0:.2f} s with sync)", file=sys.stderr, flush=True)
    assert sim.chi(b) == ref["chi_new"] == 100
    assert max_rel(sim.spectrum(b), ref["lam"]) < tol
    for v, site in ref["sites"].items():
        got = sim.get_site(int(v))
        assert list(got.shape) == site["dims"]
        flat = got.ravel(order="F")
        assert max_rel(flat[np.asarray(site["idx"])], site["val"]) < tol * 10
        assert abs(np.linalg.norm(flat) / site["norm"] - 1) < tol * 10
        # whole-tensor check: per-leg marginals (sum of squares over all other
        # indices) of every leg, 100 values per bond leg and 4 for the Pauli leg
        sq = got * got
        for l, ref_m in enumerate(site["marginals"]):
            m = sq.sum(axis=tuple(a for a in range(got.ndim) if a != l))
            assert max_rel(m, ref_m) < tol, (v, l, max_rel(m, ref_m))
    sim.close()


BP_GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "oracle_bp_4x4_chi100.json")


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("fp32", 2e-5)])
def test_bp_sweeps_chi100(precision, tol, case):
    """The a8 / a9 kernels at chi = 100 (leg Grams of 10^6-entry slices, the
    last-leg measurement kernel over 10^6-row slices) against the oracle on the
    same seeded state: one gauge-BP sweep from the seeded messages and three
    measurement-BP sweeps from the uniform start
    (tests/golden/make_golden.py oracle_bp_4x4_chi100).  The float32 form
    stores the site tensors in float32 (relative rounding 6e-8 of every
    entry), so its messages are held to 2e-5 of their largest entry."""
    if not os.path.exists(BP_GOLDEN):
        pytest.skip("oracle_bp_4x4_chi100.json not generated")
    with open(BP_GOLDEN) as f:
        ref = json.load(f)
    assert ref["config"] == fc.CFG and ref["seed"] == fc.SEED
    hpt = load_hpt()
    net, _, _ = case
    sim = hpt.Simulator(precision=precision, bp_max_sweeps=1, bp_init="warm", meas_max_sweeps=3, meas_tol=1e-300,
                        **fc.CFG)
    for v in range(net.lat.n_sites):
        sim.set_site(v, net.psi[v])
    for bb in range(net.lat.n_bonds):
        for d in range(2):
            sim.set_message(bb, d, net.M[bb][d])
    t0 = time.perf_counter()
    sweeps, delta = sim.gauge_bp(hpt.HPT_BP_WARM)
    print(f"# {precision} gauge sweep {time.perf_counter() - t0:.2f} s, delta {delta:.3e} "
          f"(oracle {ref['gauge_delta']:.3e})", file=sys.stderr, flush=True)
    assert sweeps == 1
    assert abs(delta - ref["gauge_delta"]) <= tol * max(1.0, abs(ref["gauge_delta"]))
    worst = 0.0
    for g in ref["gauge"]:
        M = sim.get_message(g["bond"], g["dir"])
        scale = max(abs(x) for x in g["diag"])
        worst = max(worst, max(abs(a - b) for a, b in zip(np.diag(M), g["diag"])) / scale,
                    max(abs(M[i, j] - v) for i, j, v in zip(g["i"], g["j"], g["val"])) / scale,
                    abs(np.linalg.norm(M) / g["fro"] - 1))
    print(f"# {precision} gauge messages: worst relative difference {worst:.2e}", file=sys.stderr, flush=True)
    assert worst <= tol
    t0 = time.perf_counter()
    r = sim.measure()
    print(f"# {precision} measurement {time.perf_counter() - t0:.2f} s, {r['meas_sweeps']} sweeps, "
          f"C {r['C']:.12e} (oracle {ref['C']:.12e})", file=sys.stderr, flush=True)
    assert r["meas_sweeps"] == ref["meas_sweeps"] == 3
    worst = 0.0
    for mm in ref["meas"]:
        got = sim.get_meas_message(mm["bond"], mm["dir"])
        exp = np.asarray(mm["m"])
        assert got.shape == exp.shape
        worst = max(worst, float(np.max(np.abs(got - exp))) / float(np.max(np.abs(exp))))
    print(f"# {precision} measurement messages: worst relative difference {worst:.2e}", file=sys.stderr, flush=True)
    assert worst <= tol
    assert abs(r["C"] - ref["C"]) <= tol * max(1.0, abs(ref["C"]))
