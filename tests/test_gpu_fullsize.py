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
