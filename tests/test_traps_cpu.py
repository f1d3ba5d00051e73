"""The trap scan on the oracle's own trajectories (no GPU): the 4x4 chi 20
run collapses at layer 40 (C 0.0622 -> 0.0066 after 93 converged sweeps, the
gate error growing 1.24x), the same run with the remediation retried that
layer and kept C = 0.0604; plus hand-made records for each branch of the
rule."""

import json
import os

import pytest

traps = pytest.importorskip("paper_2606_30985_amd.traps")
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _records(name):
    return json.load(open(os.path.join(GOLDEN, name + ".json")))["records"]


def test_layer40_trap_of_the_4x4_chi20_run():
    recs = _records("oracle_4x4_chi20")
    r = traps.detect_traps(recs, tol=1e-10)
    assert r["type1"] == 1 and r["type2"] == 0
    (e,) = r["events"]
    assert e["layer"] == 40 and e["type"] == 1 and not e["remediated"]
    # at tol 1e-10 nearly every layer is a runtime candidate: the collapse test
    # is what separates the trap
    assert r["candidates"] >= 30


def test_remediated_run_has_no_trap_left():
    recs = _records("oracle_4x4_chi20_trap_retry")
    r = traps.detect_traps(recs, tol=1e-10)
    assert r["type1"] == 0 and r["type2"] == 0
    (e,) = r["events"]
    assert e["layer"] == 40 and e["remediated"] and e["type"] == 0


def _rec(C, g, sweeps, delta, flags=0):
    return dict(C=C, gate_err=g, meas_sweeps=sweeps, meas_delta=delta, flags=flags)


def test_rule_branches():
    tol = 1e-5
    prev = _rec(0.06, 1e-3, 15, 1e-6)
    assert traps.classify(_rec(0.006, 1.2e-3, 40, 1e-6), prev, tol) == 1      # converged collapse
    assert traps.classify(_rec(0.006, 1.2e-3, 20, 1e-6), prev, tol) == 0      # too few sweeps
    assert traps.classify(_rec(0.006, 3e-3, 40, 1e-6), prev, tol) == 0        # explained by truncation
    assert traps.classify(_rec(0.05, 1.2e-3, 40, 1e-6), prev, tol) == 0       # candidate without collapse
    assert traps.classify(_rec(0.06, 1.2e-3, 100, 2e-5), prev, tol) == 2      # non-convergence
    assert traps.classify(_rec(0.006, 0.0, 40, 1e-6), _rec(0.06, 0.0, 15, 1e-6), tol) == 1
