"""Bits of hpt_measurement.flags (the HPT_FLAG_* values of include/hpt.h).

Kept apart from the ctypes binding so that host post-processing (the trap
scan) can use them without loading the library."""

FLAGS = {
    "BP_NOT_CONVERGED_GAUGE": 1 << 0,
    "BP_NOT_CONVERGED_MEAS": 1 << 1,
    "TRAP_CANDIDATE": 1 << 2,
    "NORM_EXPLODED": 1 << 3,
    "DEGENERATE_CUT": 1 << 4,
    "PINV_CUT": 1 << 5,
    "BETHE_ZERO": 1 << 6,
    "QR_FALLBACK": 1 << 7,
    "QR_RANK_DEFICIENT": 1 << 8,
    "TRAP_REMEDIATED": 1 << 9,
    "TRAP_UNRESOLVED": 1 << 10,
    "SVD_NOT_CONVERGED": 1 << 11,
}
