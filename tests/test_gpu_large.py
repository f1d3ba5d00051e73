"""The FP32-MFMA form against the FP64 form on the 10x10 chi = 100
workload (dt = 0.05, the benchmark's BP settings, the FP32 form's
truncation cutoff in both): |dC(t)| per layer.  The runs take about three
minutes of GPU time and 110 + 217 GB of HBM (one after the other).  Layers where
either measurement BP did not converge are reported, not compared (the
method's own non-convergence, flagged by the library)."""

import json
import os
import sys
import time

import numpy as np
import pytest

from tests.gpu_util import load_hpt

pytestmark = pytest.mark.gpu

CFG = dict(Lx=10, Ly=10, chi_max=100, dt=0.05, J=1.0, h=1.0, bp_tol=1e-5, bp_max_sweeps=100,
           bp_init="warm", meas_tol=1e-10, meas_max_sweeps=400)


def _run(hpt, precision, steps, **extra):
    import torch
    sim = hpt.Simulator(precision=precision, **CFG, **extra)
    out = []
    for _ in range(steps):
        t0 = time.perf_counter()
        sim.step(1)
        m = sim.measure()
        m["seconds"] = time.perf_counter() - t0
        out.append(m)
        print(f"# {precision} step {m['step']} C={m['C']:.12f} meas_sweeps={m['meas_sweeps']} "
              f"gauge_sweeps={m['gauge_sweeps']} flags={m['flags']} {m['seconds']:.2f}s", file=sys.stderr, flush=True)
    sim.close()
    del sim
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    return out


def test_10x10_chi100_fp32_form_against_fp64():
    # both float32 forms: plain float32 products, and six bf16 products of
    # split operands (precision "bf16x6"), against one float64 run
    hpt = load_hpt()
    steps = int(os.environ.get("HPT_LARGE_STEPS", "30"))
    r32 = _run(hpt, "fp32", steps)
    rbs = _run(hpt, "bf16x6", steps)
    # the FP64 reference: same truncation cutoff as the FP32 form (1e-7 s_0),
    # so the comparison isolates the arithmetic; dependent QR columns are
    # deflated below 1e-15 of the largest Gram pivot (singular values below
    # 3e-8 of the largest) instead of sending the 10^6 x 400 blocks to the
    # single-workgroup Householder
    r64 = _run(hpt, "fp64", steps, qr_rank_tol=1e-15, eps_cut=1e-7)
    bad = hpt.FLAGS["BP_NOT_CONVERGED_MEAS"]
    for name, rf in (("fp32", r32), ("bf16x6", rbs)):
        rows = []
        for a, b in zip(rf, r64):
            ok = not (a["flags"] & bad) and not (b["flags"] & bad)
            rows.append(dict(step=a["step"], t=a["t"], C32=a["C"], C64=b["C"], dC=abs(a["C"] - b["C"]), compared=ok,
                             meas_sweeps=[a["meas_sweeps"], b["meas_sweeps"]], seconds=[a["seconds"], b["seconds"]]))
        print(f"# {name}-vs-fp64 " + json.dumps(rows), file=sys.stderr, flush=True)
        cmp = [r for r in rows if r["compared"]]
        assert cmp, "no layer with both measurement BPs converged"
        early = [r for r in cmp if r["t"] <= 1.0 + 1e-12]
        if name == "fp32":
            # the target of the float32 form, on every layer: |dC| <= 1e-6
            # (measured 6.2e-7 at most, 4.1e-7 on layers 29-30)
            assert max(r["dC"] for r in cmp) <= 1e-6, name
        else:
            # the split-bf16 products: C(t) drifts one-signed from the FP64
            # run (measured: -7.1e-6 at t = 1, -1.04e-5 at t = 1.5) because
            # the bf16 MFMA truncates the low bits of the smaller products of
            # each group of eight toward zero (test_gpu_bsplit_rounding.py);
            # the bound records that drift, not the FP32 form's 1e-6 level
            assert max(r["dC"] for r in early) <= 2e-5, name
        assert max(r["dC"] for r in cmp) <= 5e-5, name


def test_10x10_chi30_fp64_against_oracle():
    # the benchmark lattice at a bond dimension the CPU oracle can follow:
    # 12 layers of the FP64 form against the oracle's trajectory
    # (tests/golden/oracle_10x10_chi30.json), within 1e-10
    import json
    hpt = load_hpt()
    path = os.path.join(os.path.dirname(__file__), "golden", "oracle_10x10_chi30.json")
    g = json.load(open(path))
    sim = hpt.Simulator(precision="fp64", **g["config"])
    got = [sim.measure()]
    for _ in range(g["nsteps"]):
        sim.step(1)
        got.append(sim.measure())
        print(f"# fp64 10x10 chi30 step {got[-1]['step']} C={got[-1]['C']:.12f}", file=sys.stderr, flush=True)
    sim.close()
    for k, rec in enumerate(g["records"]):
        assert abs(got[k]["C"] - rec["C"]) <= 1e-10, (k, got[k]["C"], rec["C"])
        assert got[k]["chi_live_max"] == rec["chi_live_max"]


def _c4_pairs(L):
    """(b, b') for every bond b and its image b' under the 90-degree rotation
    about the centre of an odd L x L grid."""
    from oracle.lattice import Lattice
    lat = Lattice(L, L)
    c = (L - 1) // 2
    pos = {frozenset([(v1 % L, v1 // L), (v2 % L, v2 // L)]): b for b, (v1, v2, _) in enumerate(lat.bonds)}

    def rot(p):
        return (c - (p[1] - c), c + (p[0] - c))

    return [(b, pos[frozenset(rot(p) for p in key)]) for key, b in pos.items()]


def _c4_worst(sim, pairs, cut):
    """Largest difference between the descending spectra of C4-related bonds.
    Values within a few orders of the truncation cutoff (cut x lambda_0) carry
    relative rounding of order eps / cut, so two related bonds may keep a
    different number of them: the longer spectrum's extra values must lie
    below 1e3 x cut, and only the common leading part is compared."""
    worst = 0.0
    for b, b2 in pairs:
        l1, l2 = np.sort(sim.spectrum(b))[::-1], np.sort(sim.spectrum(b2))[::-1]
        n = min(len(l1), len(l2))
        for extra in (l1[n:], l2[n:]):
            if len(extra) and float(np.max(extra)) > 1e3 * cut * l1[0]:
                return float("inf")
        worst = max(worst, float(np.max(np.abs(l1[:n] - l2[:n]))))
    return worst


def test_11x11_chi30_fp64_against_oracle():
    # the odd lattice with the centre site (5, 5), C4-symmetric placement:
    # 10 layers of the FP64 form against the oracle's trajectory
    # (tests/golden/oracle_11x11_chi30.json) within 1e-10.  The untruncated
    # layer is C4-invariant (the ZZ gates commute), so bonds related by the
    # 90-degree rotation about the centre carry equal spectra: 1e-12 on the
    # first 4 layers.  From layer 5 on some of the values that the 1e-11 cutoff
    # discards lie within rounding of it, two related bonds can keep different
    # sets, and the environment inversions of the next gates carry that
    # difference into the kept spectra (1e-8 measured, with Householder QR as
    # with the adaptive QR); those layers are reported, not asserted.
    hpt = load_hpt()
    path = os.path.join(os.path.dirname(__file__), "golden", "oracle_11x11_chi30.json")
    if not os.path.exists(path):
        pytest.skip("oracle_11x11_chi30.json not generated")
    g = json.load(open(path))
    pairs = _c4_pairs(11)
    sim = hpt.Simulator(precision="fp64", **g["config"])
    got = [sim.measure()]
    for k in range(g["nsteps"]):
        sim.step(1)
        got.append(sim.measure())
        w = _c4_worst(sim, pairs, 1e-11)
        print(f"# fp64 11x11 chi30 step {got[-1]['step']} C={got[-1]['C']:.12f} C4 spectra {w:.1e}", file=sys.stderr,
              flush=True)
        if k + 1 <= 4:
            assert w <= 1e-12, (k + 1, w)
    sim.close()
    for k, rec in enumerate(g["records"]):
        assert abs(got[k]["C"] - rec["C"]) <= 1e-10, (k, got[k]["C"], rec["C"])
        assert got[k]["chi_live_max"] == rec["chi_live_max"]


def test_11x11_chi100_fp32_form():
    # the benchmark's second lattice, 11x11 at chi_max = 100 in the FP32 form
    # (139 GB arena; FP64 at chi 100 does not fit one GPU): the first 6 layers,
    # untruncated at chi 30 already, against the oracle's 11x11 chi 30
    # trajectory within 1e-6, and C4-related bonds with equal spectra to 1e-5
    # (float32 storage of the site tensors)
    import torch
    hpt = load_hpt()
    path = os.path.join(os.path.dirname(__file__), "golden", "oracle_11x11_chi30.json")
    if not os.path.exists(path):
        pytest.skip("oracle_11x11_chi30.json not generated")
    g = json.load(open(path))
    cfg = dict(g["config"])
    cfg["chi_max"] = 100
    pairs = _c4_pairs(11)
    sim = hpt.Simulator(precision="fp32", **cfg)
    done = 0
    for k in range(1, 7):
        ref = g["records"][k]
        if ref["gate_err"] >= 1e-20:
            break   # the chi 30 oracle truncates from here on
        sim.step(1)
        m = sim.measure()
        w = _c4_worst(sim, pairs, 1e-7)
        print(f"# fp32 11x11 chi100 step {k} C={m['C']:.12f} (oracle chi30 {ref['C']:.12f}) C4 spectra {w:.1e}",
              file=sys.stderr, flush=True)
        assert abs(m["C"] - ref["C"]) <= 1e-6
        assert w <= 1e-5
        done += 1
    assert done >= 4
    sim.close()
    del sim
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
