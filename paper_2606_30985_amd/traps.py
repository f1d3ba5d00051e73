"""Trap scan over the per-layer measurement records of a run (Sec. "BP
Fixed-Point Multiplicity": the two failure modes and the runtime rule).

A record is a mapping with the keys the library's hpt_measure fills in:
C, gate_err, meas_sweeps, meas_delta, flags.  Host post-processing of logged
records; nothing here runs on the device or touches the simulation."""

from .flags import FLAGS

TRAP_REMEDIATED = FLAGS["TRAP_REMEDIATED"]
TRAP_UNRESOLVED = FLAGS["TRAP_UNRESOLVED"]


def classify(rec, prev, tol, trap_sweeps=30):
    """Failure type of one layer given the previous layer's record:
    2 -- non-convergence: the measurement BP ended with delta >= tol;
    1 -- verified metastable trap: converged after >= trap_sweeps sweeps
         (the runtime candidate rule) and C fell below half of the previous
         layer's C while the gate error grew less than twofold (a collapse the
         truncation does not explain);
    0 -- otherwise (a candidate that is not a collapse is not a trap)."""
    if not (rec["meas_delta"] < tol):
        return 2
    if prev is None or rec["meas_sweeps"] < trap_sweeps:
        return 0
    collapse = abs(rec["C"]) < 0.5 * abs(prev["C"])
    gate_ok = rec["gate_err"] < 2.0 * prev["gate_err"] or rec["gate_err"] == 0.0
    return 1 if collapse and gate_ok else 0


def detect_traps(records, tol, trap_sweeps=30):
    """Scan a trajectory (records[0] = layer 0): every layer of failure type
    1 or 2, with the layer's sweeps, delta, C, the previous C, and whether the
    library's remediation retried it (TRAP_REMEDIATED / TRAP_UNRESOLVED);
    and the counts per type and the runtime candidates (sweeps >= trap_sweeps
    with delta < tol, trapped or not)."""
    events = []
    candidates = 0
    for k, rec in enumerate(records):
        prev = records[k - 1] if k > 0 else None
        if rec["meas_sweeps"] >= trap_sweeps and rec["meas_delta"] < tol:
            candidates += 1
        t = classify(rec, prev, tol, trap_sweeps)
        flags = int(rec.get("flags", 0))
        if t or flags & (TRAP_REMEDIATED | TRAP_UNRESOLVED):
            events.append(dict(layer=k, type=t, sweeps=rec["meas_sweeps"], delta=rec["meas_delta"], C=rec["C"],
                               C_prev=None if prev is None else prev["C"],
                               remediated=bool(flags & TRAP_REMEDIATED), unresolved=bool(flags & TRAP_UNRESOLVED)))
    return dict(events=events, type1=sum(1 for e in events if e["type"] == 1),
                type2=sum(1 for e in events if e["type"] == 2), candidates=candidates, layers=len(records))
