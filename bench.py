"""Benchmark: Trotter layers per second of the Heisenberg-picture TFIM network.

Workload (default): 10 x 10 open lattice, J = h = 1, dt = 0.05, chi_max = 100,
observable Z at (4, 4), float32 site tensors with MFMA contractions and float64
Cholesky / SVD / eigensolver / BP normalisation / Bethe sum.  A "step" is one
whole pass of the hot path: field half-step, 4-colour gate sweep, field
half-step, gauge BP, measurement BP and the log-space Bethe sum of C(t).

Default: the 30-layer run, layers 1..28 untimed (warm-up, the bond dimension
saturates at chi_max on the central bonds), layers 29 and 30 timed.

Prints one JSON line.  `roofline` reports the dominant MFMA contraction kernel
(largest summed duration), timed with HIP events on its launch stream over the
timed region; `cpu_baseline` times the CPU oracle on one bond update sample and
scales it to the workload.
"""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_TFLOPS = {"fp32": 157.3, "fp64": 78.6, "bf16": 2500.0}
FORM_NAMES = {"fp32": "FP32-MFMA form", "bf16x6": "FP32 form with split-bf16 (x6) GEMMs", "fp64": "FP64 plain form"}
KERNEL_NAMES = {"gemm": "tile_gemm_kernel<float> / gemm_pipe_kernel (tiled MFMA GEMM)",
                "gram64": "gram64_kernel (float64-accumulated Gram, MFMA f64)",
                "mode": "mode_product_kernel (MFMA mode product, factor in LDS)",
                "leggram": "leg_gram_kernel (MFMA leg Gram of the gauge BP, with its partial sum)",
                "bsplit": "tile_gemm_kernel<split> (six bf16 MFMA products of split float32 operands)"}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=28)
    ap.add_argument("--precision", default="fp32", choices=["fp32", "bf16x6", "fp64"])
    ap.add_argument("--L", type=int, default=10)
    ap.add_argument("--chi", type=int, default=100)
    ap.add_argument("--dt", type=float, default=0.05)
    ap.add_argument("--bp-tol", type=float, default=1e-5)
    ap.add_argument("--bp-max-sweeps", type=int, default=100)
    ap.add_argument("--meas-tol", type=float, default=1e-10)
    ap.add_argument("--meas-max-sweeps", type=int, default=400)
    ap.add_argument("--bp-init", default="warm", choices=["warm", "uniform"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--trace", default="", help="append per-step records (JSON lines) to this file")
    ap.add_argument("--profile-all", action="store_true",
                    help="kernel event profile over every layer (warm-up included), for counter comparisons")
    ap.add_argument("--workload", default="large", choices=["large", "batched"],
                    help="large: the 10x10 chi=100 run (default); batched: the independent-runs set")
    ap.add_argument("--batch-runs", type=int, default=64)
    ap.add_argument("--batch-chi", type=int, default=40)
    ap.add_argument("--calibrate-copy", type=int, default=0,
                    help="first copy this many bytes with the library's plain copy kernel (counter calibration)")
    return ap.parse_args()


def cpu_baseline(chi, L, dt, sample_chi=70):
    """CPU oracle on one interior-interior bond update (synthetic saturated
    inputs) at sample_chi, extrapolated to the workload's chi by the chi^5
    cost of the update and scaled to layers/s by the layer's bond count."""
    import numpy as np
    from oracle.network import Config, OperatorNetwork
    from paper_2606_30985_amd import inputs
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        threads = os.cpu_count() or 1
    c = sample_chi
    cfg = Config(Lx=4, Ly=4, chi_max=c, dt=dt)
    net = OperatorNetwork(cfg)
    lat = net.lat
    b0 = [b for b, (v1, v2, _) in enumerate(lat.bonds) if (v1, v2) == (5, 6)][0]
    big = {b for b, (v1, v2, _) in enumerate(lat.bonds) if {v1, v2} & {5, 6}}
    net.chi = [c if b in big else 1 for b in range(lat.n_bonds)]
    for v in range(lat.n_sites):
        net.psi[v] = np.array(inputs.site_tensor(100 + v, net.site_dims(v)))
    for b in range(lat.n_bonds):
        cb = net.chi[b]
        net.M[b] = [inputs.env_message(900 + 2 * b, cb), inputs.env_message(901 + 2 * b, cb)]
    t0 = time.perf_counter()
    net.gate_update(b0)
    sec = time.perf_counter() - t0
    print(f"# cpu baseline: oracle bond update at chi={c}: {sec:.2f} s", file=sys.stderr, flush=True)
    scale = (chi / c) ** 5
    n_bonds = (L - 1) * L * 2
    est = sec * scale
    return {"value": 1.0 / (est * n_bonds), "unit": "layers/s", "cores": int(threads), "kind": "oracle",
            "sample": f"one interior-interior bond update at chi={c} ({c ** 3} x {4 * c} QR blocks, synthetic "
                      f"saturated inputs) took {sec:.2f} s; extrapolated by (chi/{c})^5 = {scale:.1f} to "
                      f"chi={chi} ({est:.0f} s per bond) and by the {n_bonds} bond updates of one {L}x{L} "
                      f"layer; gauge BP and measurement not counted (an upper bound on the CPU rate)",
            "bond_updates_per_s_extrapolated": 1.0 / est}


def roofline_peak(kind, precision):
    """MFMA peak (TFLOP/s of algorithmic flops) for a contraction kind: float64
    products (the Gram of float32 data, or every product of the float64 form)
    run on the FP64 MFMA; the split-bf16 products on the bf16 MFMA, six bf16
    flops per algorithmic flop; the rest on the FP32 MFMA."""
    if kind == "gram64" or precision == "fp64":
        return PEAK_TFLOPS["fp64"]
    if kind == "bsplit":
        return PEAK_TFLOPS["bf16"] / 6.0
    return PEAK_TFLOPS["fp32"]


def traffic_ratio(kernel_key):
    """HBM bytes per algorithmic byte of a kernel family, from the committed
    PMC summary; None when the kernel source has changed since it was taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "mode_product_kernel_10x10_chi100_pmc.md")
    if not os.path.exists(path):
        return None
    names = {"mode": "mode_product_kernel", "gram64": "gram64", "leggram": "leggram", "gemm": "gemm"}
    ratio = sha = src = None
    for line in open(path):
        f = line.split()
        if len(f) == 3 and f[0] == "traffic_ratio" and f[1] == names.get(kernel_key):
            ratio = float(f[2])
        if len(f) == 3 and f[0] == "kernel_source_sha256":
            src, sha = f[1], f[2]
    if ratio is None or sha is None:
        return None
    with open(os.path.join(ROOT, src), "rb") as fh:
        if hashlib.sha256(fh.read()).hexdigest() != sha:
            return None
    return ratio


def batched(args):
    """The batched form: independent runs (grid 3x3..6x6, h ~ U[0.5, 3], dt in
    {0.025, 0.05, 0.1, 0.2}, total time 2, chi_max 40, FP32 form), measured
    after every layer.  Timed twice on the same handles: one run after
    another, then all at once through hpt_run_batch; the trajectories must
    agree exactly.  Batched first (fresh handles), then one after another."""
    import torch
    from paper_2606_30985_amd import hpt, inputs
    runs = inputs.batched_runs()[: args.batch_runs]
    sims = [hpt.Simulator(Lx=r["Lx"], Ly=r["Ly"], J=r["J"], h=r["h"], dt=r["dt"], chi_max=args.batch_chi,
                          precision="fp32", bp_tol=args.bp_tol, bp_max_sweeps=args.bp_max_sweeps, bp_alpha=0.5,
                          bp_init=args.bp_init, meas_tol=args.meas_tol, meas_max_sweeps=args.meas_max_sweeps,
                          stream=torch.cuda.Stream())
            for r in runs]
    nsteps = [r["nsteps"] for r in runs]
    total = sum(nsteps)
    os.environ["HPT_BATCH_PROGRESS"] = "1"   # one line per finished run
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = hpt.run_batch(sims, nsteps)
    torch.cuda.synchronize()
    t_bat = time.perf_counter() - t0
    print(f"# batched: {t_bat:.2f} s", file=sys.stderr, flush=True)
    for s in sims:
        s.reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    seq = []
    for i, (s, n) in enumerate(zip(sims, nsteps)):
        traj = []
        for _ in range(n):
            s.step(1)
            traj.append(s.measure()["C"])
        seq.append(traj)
        print(f"# sequential run {i}: {runs[i]['Lx']}x{runs[i]['Ly']} dt={runs[i]['dt']} {n} layers "
              f"C(2)={traj[-1]:.8f} {time.perf_counter() - t0:.1f}s", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t0
    print(f"# sequential: {t_seq:.2f} s (batched {t_bat:.2f} s)", file=sys.stderr, flush=True)
    dmax = max(abs(a - b["C"]) for traj, rr in zip(seq, res) for a, b in zip(traj, rr))
    for s in sims:
        s.close()
    out = {"metric": "Trotter layers/sec, batched form (independent runs, MPF step-size set)",
           "value": total / t_bat, "unit": "layers/s", "n_gpus": 1, "steps": total, "warmup": 0,
           "ms_per_step": 1e3 * t_bat / total, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic (seeded run parameters, deterministic initial operators)",
           "config": {"workload": f"{len(runs)} independent runs, grids 3x3..6x6, h ~ U[0.5,3], dt in "
                                  f"{{0.025,0.05,0.1,0.2}}, t = 2, chi_max={args.batch_chi}, FP32 form",
                      "layers": total, "sequential_layers_per_s": total / t_seq, "speedup_vs_sequential": t_seq / t_bat,
                      "max_abs_dC_batched_vs_sequential": dmax}}
    print(json.dumps(out), flush=True)


def main():
    args = parse()
    if args.workload == "batched":
        if args.gpus != 1:
            print(json.dumps({"error": "this library runs on one GPU; run with --gpus 1"}))
            sys.exit(2)
        return batched(args)
    if args.gpus != 1:
        print(json.dumps({"error": "this library runs on one GPU; multi-GPU sharding is a design note only, "
                                   "run with --gpus 1"}))
        sys.exit(2)
    import torch
    from paper_2606_30985_amd import hpt

    if args.calibrate_copy:
        # one plain copy of known size through permute_generic (identity permutation)
        nel = args.calibrate_copy // 4
        src = torch.rand(nel, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        hpt.permute(src, dst, [0])
        torch.cuda.synchronize()
        del src, dst
        print(f"# calibration copy: {nel * 4} bytes read, {nel * 4} bytes written", file=sys.stderr, flush=True)

    L, chi = args.L, args.chi
    sim = hpt.Simulator(Lx=L, Ly=L, chi_max=chi, dt=args.dt, J=1.0, h=1.0, precision=args.precision,
                        bp_tol=args.bp_tol, bp_max_sweeps=args.bp_max_sweeps, bp_alpha=0.5,
                        meas_tol=args.meas_tol, meas_max_sweeps=args.meas_max_sweeps, bp_init=args.bp_init)
    trace = open(args.trace, "a") if args.trace else None

    def one(timed):
        t0 = time.perf_counter()
        sim.step(1)
        m = sim.measure()
        rec = dict(m, seconds=time.perf_counter() - t0, timed=timed)
        print(f"# step {m['step']} t={m['t']:.3f} C={m['C']:.10f} chi={m['chi_live_max']} "
              f"gauge_sweeps={m['gauge_sweeps']} meas_sweeps={m['meas_sweeps']} "
              f"gate_err={m['gate_err']:.2e} {rec['seconds']:.2f}s", file=sys.stderr, flush=True)
        if trace:
            trace.write(json.dumps(rec) + "\n")
            trace.flush()
        return rec

    if args.profile_all:
        hpt.profile_gemm(True)
    for _ in range(args.warmup):
        one(False)
    torch.cuda.synchronize()
    if not args.profile_all:
        hpt.profile_gemm(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    recs = [one(True) for _ in range(args.steps)]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    kinds = {k: hpt.profile_gemm_read(k) for k in hpt.PROF_KINDS}
    hpt.profile_gemm(False)
    # the dominant contraction kernel (largest summed duration) carries the roofline
    dom = max(kinds, key=lambda k: kinds[k]["ms"])
    prof = kinds[dom]
    n_bonds = (L - 1) * L * 2
    value = args.steps / elapsed
    ratio = traffic_ratio(dom)
    achieved = prof["flops"] / (prof["ms"] * 1e-3) / 1e12 if prof["ms"] > 0 else 0.0
    peak = roofline_peak(dom, args.precision)
    out = {
        "metric": "Trotter layers/sec at 10x10 chi=100 (|dC(t)| vs FP64 oracle); bond updates/sec",
        "value": value,
        "unit": "layers/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32", "bf16x6": "f32 (bf16x6 split products)"}[args.precision],
        "data": "synthetic (deterministic initial operator Z_c, no dataset)",
        "config": {"workload": f"{L}x{L} TFIM Heisenberg Z_c(t), chi_max={chi}, dt={args.dt}, J=h=1, "
                               f"{FORM_NAMES[args.precision]}, "
                               f"gauge BP tol {args.bp_tol} max {args.bp_max_sweeps} sweeps, damping 0.5, "
                               f"{args.bp_init} init; measurement BP tol {args.meas_tol} max "
                               f"{args.meas_max_sweeps} sweeps; layers {args.warmup + 1}..{args.warmup + args.steps}",
                   "bond_updates_per_s": n_bonds * args.steps / elapsed,
                   "chi_live_max": recs[-1]["chi_live_max"],
                   "gauge_sweeps": [r["gauge_sweeps"] for r in recs],
                   "meas_sweeps": [r["meas_sweeps"] for r in recs],
                   "C": [r["C"] for r in recs]},
        "roofline": {"bound": "mfma", "kernel": KERNEL_NAMES[dom],
                     "achieved": achieved, "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak,
                     # HBM bytes per launch: PMC FETCH_SIZE + WRITE_SIZE (copy-calibrated) per
                     # algorithmic byte, times this run's algorithmic bytes per launch
                     "traffic": (None if ratio is None else ratio * prof["bytes"] / max(prof["launches"], 1)),
                     "traffic_unit": "bytes per launch",
                     "algorithmic_bytes_per_launch": prof["bytes"] / max(prof["launches"], 1),
                     "launches": prof["launches"], "kernel_ms": prof["ms"],
                     "avg_launch_ms": prof["ms"] / max(prof["launches"], 1),
                     "flop_per_launch": prof["flops"] / max(prof["launches"], 1),
                     "kernel_share_of_step": prof["ms"] * 1e-3 / elapsed,
                     "contractions": {KERNEL_NAMES[k]: {"launches": v["launches"], "ms": v["ms"],
                                                        "tflops": v["flops"] / (v["ms"] * 1e-3) / 1e12 if v["ms"] > 0 else 0.0,
                                                        "algorithmic_bytes": v["bytes"]}
                                      for k, v in kinds.items()}},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(chi, L, args.dt)
    sim.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
