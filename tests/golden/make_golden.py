"""Write oracle trajectories used as expected values by the GPU parity tests.

Calls only the CPU oracle (oracle/).  Usage: python tests/golden/make_golden.py NAME
Each output file records the configuration it was computed with.
"""

import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle.network import Config  # noqa: E402
from oracle.run import run  # noqa: E402

CASES = {
    # 4x4, centre (1,1), dt 0.05, 40 steps, chi_max 20, FP64, uniform-init BP, damping 0.5, tol 1e-10
    "oracle_4x4_chi20": (dict(Lx=4, Ly=4, J=1.0, h=1.0, dt=0.05, chi_max=20, bp_alpha=0.5, bp_tol=1e-10), 40),
    # chi_max 40 and 60: the first layers (the centre bonds reach chi_max by layer ~10 at 40 and
    # ~12 at 60; the full 40-layer runs take hours in the oracle)
    "oracle_4x4_chi40": (dict(Lx=4, Ly=4, J=1.0, h=1.0, dt=0.05, chi_max=40, bp_alpha=0.5, bp_tol=1e-10), 14),
    "oracle_4x4_chi60": (dict(Lx=4, Ly=4, J=1.0, h=1.0, dt=0.05, chi_max=60, bp_alpha=0.5, bp_tol=1e-10), 9),
    "oracle_3x3_chi8": (dict(Lx=3, Ly=3, J=1.0, h=1.0, dt=0.05, chi_max=8, bp_alpha=0.5, bp_tol=1e-10), 20),
    # 10x10 (the benchmark lattice) at chi_max 30, FP64 cutoff, the benchmark's BP settings, 12 layers
    "oracle_10x10_chi30": (dict(Lx=10, Ly=10, J=1.0, h=1.0, dt=0.05, chi_max=30, bp_alpha=0.5, bp_tol=1e-5,
                                bp_max_sweeps=100, bp_init="warm", meas_tol=1e-10, meas_max_sweeps=400), 12),
    # 11x11 (odd, centre (5,5): C4-symmetric placement) at chi_max 30, same settings, 10 layers
    "oracle_11x11_chi30": (dict(Lx=11, Ly=11, J=1.0, h=1.0, dt=0.05, chi_max=30, bp_alpha=0.5, bp_tol=1e-5,
                                bp_max_sweeps=100, bp_init="warm", meas_tol=1e-10, meas_max_sweeps=400), 10),
    # the 4x4 chi_max 20 run with the trap remediation (the layer-40 trap is retried)
    "oracle_4x4_chi20_trap_retry": (dict(Lx=4, Ly=4, J=1.0, h=1.0, dt=0.05, chi_max=20, bp_alpha=0.5, bp_tol=1e-10,
                                         trap_retry=True), 40),
}

BOND_CASES = ("oracle_bond_4x4_chi100",)
BP_CASES = ("oracle_bp_4x4_chi100",)
BP_SAMPLES = 64


def bp_case(name):
    """Belief propagation at chi = 100 on the seeded saturated state of
    tests/fullsize_case.py: one gauge-BP sweep (damping 0.5) from the seeded
    environment messages, and three measurement-BP sweeps from the uniform
    start (tolerance never met, so all three run).  For every chi = 100 bond
    and direction: the diagonal, sampled off-diagonal entries and the
    Frobenius norm of the new gauge message; every measurement message whole,
    and C at the messages of the third sweep."""
    import dataclasses
    import numpy as np
    from tests import fullsize_case as fc
    t0 = time.time()
    net, _ = fc.state()
    net.cfg = dataclasses.replace(net.cfg, bp_max_sweeps=1, bp_init="warm", meas_max_sweeps=3, meas_tol=1e-300)
    print(f"state {time.time() - t0:.1f}s", flush=True)
    sweeps, delta = net.gauge_bp()
    print(f"gauge sweep {time.time() - t0:.1f}s", flush=True)
    rng = np.random.default_rng(1)
    gauge = []
    for b in range(net.lat.n_bonds):
        if net.chi[b] != fc.CFG["chi_max"]:
            continue
        for d in range(2):
            M = net.M[b][d]
            c = M.shape[0]
            i = rng.integers(0, c, BP_SAMPLES)
            j = rng.integers(0, c, BP_SAMPLES)
            gauge.append(dict(bond=b, dir=d, diag=[float(x) for x in np.diag(M)], i=[int(x) for x in i],
                              j=[int(x) for x in j], val=[float(M[a, bb]) for a, bb in zip(i, j)],
                              fro=float(np.linalg.norm(M))))
    r = net.measure()
    print(f"measurement sweeps {time.time() - t0:.1f}s", flush=True)
    meas = [dict(bond=b, dir=d, m=[float(x) for x in net.meas_messages[b][d]])
            for b in range(net.lat.n_bonds) for d in range(2)]
    out = dict(config=fc.CFG, seed=fc.SEED, source="oracle/ (CPU FP64 restatement of the method)",
               gauge_delta=float(delta), gauge=gauge, meas=meas, meas_sweeps=int(r["meas_sweeps"]),
               meas_delta=float(r["meas_delta"]), C=float(r["C"]))
    with open(os.path.join(HERE, name + ".json"), "w") as f:
        json.dump(out, f)


def bond_case(name):
    """One interior-interior bond update at chi = 100 on the seeded saturated
    state of tests/fullsize_case.py: spectrum, bond dimension, gate error and
    sampled entries (with norms) of both new site tensors."""
    import numpy as np
    from tests import fullsize_case as fc
    t0 = time.time()
    net, b = fc.state()
    print(f"state {time.time() - t0:.1f}s", flush=True)
    r = net.gate_update(b)
    print(f"update {time.time() - t0:.1f}s", flush=True)
    v1, v2, _ = net.lat.bonds[b]
    sites = {}
    for v in (v1, v2):
        T = net.psi[v]
        flat = T.ravel(order="F")
        idx = fc.sample_index(flat.size)
        # per-leg marginals: for every leg, the sum of squares over all other indices
        sq = T * T
        marg = [[float(x) for x in sq.sum(axis=tuple(a for a in range(T.ndim) if a != l))] for l in range(T.ndim)]
        sites[str(v)] = dict(dims=list(T.shape), norm=float(np.linalg.norm(flat)),
                             idx=[int(i) for i in idx], val=[float(x) for x in flat[idx]], marginals=marg)
    out = dict(config=fc.CFG, seed=fc.SEED, bond=int(b), source="oracle/ (CPU FP64 restatement of the method)",
               chi_new=int(r["chi_new"]), lam=[float(x) for x in r["lam"]], gate_err=float(r["gate_err"]),
               sites=sites)
    with open(os.path.join(HERE, name + ".json"), "w") as f:
        json.dump(out, f)


def main(name):
    if name in BOND_CASES:
        return bond_case(name)
    if name in BP_CASES:
        return bp_case(name)
    cfg, n = CASES[name]
    t0 = time.time()

    def cb(net, rec):
        print(rec["step"], rec["C"], f"{time.time() - t0:.1f}s", flush=True)

    recs, _ = run(Config(**cfg), n, callback=cb)
    out = dict(config=cfg, nsteps=n, source="oracle/ (CPU FP64 restatement of the method)",
               records=[{k: (v if not isinstance(v, float) or v == v else None) for k, v in r.items()}
                        for r in recs])
    with open(os.path.join(HERE, name + ".json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main(sys.argv[1])
