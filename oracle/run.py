"""Time loop of the method (oracle; test infrastructure only).

Paper, implementation pipeline figure ("one time step"): field gate on all
sites, 4-colour sweep of two-site gates, field gate on all sites, belief
propagation, then the measurement of C(t) by the log-space Bethe sum.
C(0) is measured on the initial operator (Sec. "Numerical Experiments":
C(0) = 1 by normalisation).
"""

import math
import time

import numpy as np

from .network import (Config, OperatorNetwork, FLAG_BP_NOT_CONVERGED_GAUGE, FLAG_BP_NOT_CONVERGED_MEAS,
                      FLAG_TRAP_CANDIDATE, FLAG_NORM_EXPLODED, FLAG_TRAP_REMEDIATED,
                      FLAG_TRAP_UNRESOLVED)


def layer(net: OperatorNetwork):
    """One Trotter layer: a1 .. a8."""
    lat = net.lat
    net.apply_field()
    gate_err, flags = 0.0, 0
    s_frac = 0.0
    for c in range(4):
        for b in lat.bonds_of_colour(c):
            r = net.gate_update(b)
            gate_err += r["gate_err"]
            flags |= r["flags"]
    net.apply_field()
    gs, gd = (0, 0.0)
    if net.cfg.gauge_bp:
        gs, gd = net.gauge_bp()
        if gd >= net.cfg.bp_tol:
            flags |= FLAG_BP_NOT_CONVERGED_GAUGE
        if gs >= net.cfg.trap_sweeps and gd < net.cfg.bp_tol:
            flags |= FLAG_TRAP_CANDIDATE
    for b in range(lat.n_bonds):
        lam = net.lam[b]
        l2 = lam * lam
        S = -math.fsum([x * math.log(x) for x in l2 if x > 0])
        if net.cfg.chi_max > 1:
            s_frac = max(s_frac, S / math.log(net.cfg.chi_max))
    net.step_count += 1
    net.layer_gate_err = gate_err
    net.layer_flags = flags
    net.layer_sfrac = s_frac
    net.last_gauge = (gs, gd)


def measurement_record(net: OperatorNetwork):
    r = net.measure()
    gs, gd = net.last_gauge
    flags = r["flags"] | net.layer_flags
    bn = getattr(net, "bethe_norm", 1.0)
    if bn == bn and bn >= 2.0:
        flags |= FLAG_NORM_EXPLODED
    return dict(step=net.step_count, t=net.step_count * net.cfg.dt, C=r["C"],
                log_abs_C=r["log_abs_C"], sign=r["sign"], gate_err=net.layer_gate_err,
                bethe_norm=bn, max_S_over_logchi=getattr(net, "layer_sfrac", 0.0),
                gauge_sweeps=gs, meas_sweeps=r["meas_sweeps"], gauge_delta=gd,
                meas_delta=r["meas_delta"], chi_live_max=max(net.chi), flags=flags)


def trap_verified(rec, prev):
    """Paper, Sec. "BP Fixed-Point Multiplicity", trap remediation steps 1-2:
    a BP of this layer converged only after >= trap_sweeps sweeps (candidate)
    and C(t) fell below half of the previous layer's value while the gate
    error did not grow in proportion (reading: to less than twice the previous
    layer's gate error)."""
    if prev is None or not (rec["flags"] & FLAG_TRAP_CANDIDATE):
        return False
    if not (abs(rec["C"]) < 0.5 * abs(prev["C"])):
        return False
    return rec["gate_err"] < 2.0 * prev["gate_err"] or rec["gate_err"] == 0.0


def retry_alpha(cfg: Config):
    """Paper, trap remediation step 3: retry at 0.50 when the undamped update
    trapped, at 0.80 when 0.50 trapped (any other damping: 0.80)."""
    if cfg.trap_alpha is not None:
        return cfg.trap_alpha
    a = cfg.bp_alpha if cfg.meas_alpha is None else cfg.meas_alpha
    return 0.5 if a >= 1.0 else 0.8


def remediate_trap(net: OperatorNetwork, rec, prev):
    """Retry the measurement BP (fresh uniform start) with the other damping
    when a trap is verified.  The retry is accepted when it converges and its
    C(t) is no longer a drop below half of the previous layer's value (flag
    TRAP_REMEDIATED); otherwise the first result stands with TRAP_UNRESOLVED
    (paper: step 4, the bond dimension is insufficient).  Returns the record
    to keep."""
    if not trap_verified(rec, prev):
        return rec
    r = net.measure(alpha=retry_alpha(net.cfg))
    tol = net.cfg.bp_tol if net.cfg.meas_tol is None else net.cfg.meas_tol
    out = dict(rec)
    if r["meas_delta"] < tol and abs(r["C"]) >= 0.5 * abs(prev["C"]):
        out.update(C=r["C"], log_abs_C=r["log_abs_C"], sign=r["sign"], meas_sweeps=r["meas_sweeps"],
                   meas_delta=r["meas_delta"])
        out["flags"] = (rec["flags"] & ~FLAG_BP_NOT_CONVERGED_MEAS) | FLAG_TRAP_REMEDIATED
    else:
        out["flags"] = rec["flags"] | FLAG_TRAP_UNRESOLVED
    return out


def run(cfg: Config, nsteps: int, callback=None):
    """Trajectory C(n dt), n = 0..nsteps, with per-step diagnostics."""
    net = OperatorNetwork(cfg)
    recs = [measurement_record(net)]
    for _ in range(nsteps):
        t0 = time.perf_counter()
        layer(net)
        rec = measurement_record(net)
        if cfg.trap_retry:
            rec = remediate_trap(net, rec, recs[-1])
        rec["seconds"] = time.perf_counter() - t0
        recs.append(rec)
        if callback:
            callback(net, rec)
    return recs, net


def trajectory(cfg: Config, nsteps: int):
    recs, _ = run(cfg, nsteps)
    return np.array([r["C"] for r in recs])
