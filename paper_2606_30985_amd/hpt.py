"""ctypes binding of libhpt (include/hpt.h).

Argument marshalling only: every step of the method runs inside libhpt's
HIP kernels.  PyTorch supplies the device arena (one uint8 tensor) and the
stream.  Importing this module loads libhpt.so and fails loudly if it is not
built.
"""

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhpt.so")

HPT_FP64 = 0
HPT_FP32_MFMA = 1
HPT_FP32_BF16X6 = 2
HPT_QR_ADAPTIVE = 0
HPT_QR_HOUSEHOLDER = 1
HPT_BP_UNIFORM = 0
HPT_BP_WARM = 1
HPT_BP_LEARNED = 2
LEARN_FEATURES = 16
LEARN_HIDDEN = 128
LEARN_PARAMS = LEARN_HIDDEN * LEARN_FEATURES + 2 * LEARN_HIDDEN + 1

from .flags import FLAGS  # noqa: E402  (the measurement flag bits)
HPT_AXES_PAPER = 0
HPT_AXES_ZZX = 1


class HptConfig(ctypes.Structure):
    _fields_ = [
        ("Lx", ctypes.c_int32), ("Ly", ctypes.c_int32),
        ("J", ctypes.c_double), ("h", ctypes.c_double), ("dt", ctypes.c_double),
        ("chi_max", ctypes.c_int32), ("cx", ctypes.c_int32), ("cy", ctypes.c_int32),
        ("precision", ctypes.c_int32), ("qr_mode", ctypes.c_int32),
        ("chol_min_ratio", ctypes.c_int32), ("chol_min_cols", ctypes.c_int32),
        ("eps_cut", ctypes.c_double), ("eps_pinv", ctypes.c_double),
        ("bp_alpha", ctypes.c_double), ("bp_tol", ctypes.c_double),
        ("bp_max_sweeps", ctypes.c_int32), ("bp_init", ctypes.c_int32),
        ("meas_alpha", ctypes.c_double), ("meas_tol", ctypes.c_double),
        ("meas_max_sweeps", ctypes.c_int32), ("gauge_bp", ctypes.c_int32),
        ("trap_sweeps", ctypes.c_int32), ("qr_rank_tol", ctypes.c_double),
        ("trap_retry", ctypes.c_int32), ("reserved0", ctypes.c_int32), ("trap_alpha", ctypes.c_double),
        ("model_axes", ctypes.c_int32), ("svd_max_sweeps", ctypes.c_int32),
        ("meas_init", ctypes.c_int32), ("meas_graph", ctypes.c_int32),
    ]


class HptMeasurement(ctypes.Structure):
    _fields_ = [
        ("step", ctypes.c_int32), ("t", ctypes.c_double), ("C", ctypes.c_double),
        ("log_abs_C", ctypes.c_double), ("sign", ctypes.c_int32),
        ("gate_err", ctypes.c_double), ("bethe_norm", ctypes.c_double),
        ("max_S_over_logchi", ctypes.c_double),
        ("gauge_sweeps", ctypes.c_int32), ("meas_sweeps", ctypes.c_int32),
        ("gauge_delta", ctypes.c_double), ("meas_delta", ctypes.c_double),
        ("chi_live_max", ctypes.c_int32), ("flags", ctypes.c_uint32),
    ]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libhpt.so is not built ({LIB_PATH}); run __graft_entry__.build() "
                          "or python paper_2606_30985_amd/build.py")
    # torch first: its HIP runtime is then the one libhpt.so binds to (two
    # copies of the runtime in one process do not share the device)
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    i32, u64, dbl = ctypes.c_int32, ctypes.c_uint64, ctypes.c_double
    cfgp = ctypes.POINTER(HptConfig)
    sig = {
        "hpt_config_default": [cfgp],
        "hpt_required_bytes": [cfgp, ctypes.POINTER(u64)],
        "hpt_state_bytes": [cfgp, ctypes.POINTER(u64)],
        "hpt_create": [cfgp, P, u64, P, ctypes.POINTER(P)],
        "hpt_reset": [P],
        "hpt_step": [P, i32],
        "hpt_apply_field": [P],
        "hpt_apply_bond": [P, i32],
        "hpt_gauge_bp": [P, i32, ctypes.POINTER(i32), ctypes.POINTER(dbl)],
        "hpt_measure": [P, ctypes.POINTER(HptMeasurement)],
        "hpt_get_chi": [P, i32, ctypes.POINTER(i32)],
        "hpt_get_bond_spectrum": [P, i32, ctypes.POINTER(dbl), i32, ctypes.POINTER(i32)],
        "hpt_get_site_tensor": [P, i32, ctypes.POINTER(dbl), u64, ctypes.POINTER(i32)],
        "hpt_set_site_tensor": [P, i32, ctypes.POINTER(dbl), ctypes.POINTER(i32)],
        "hpt_get_messages": [P, i32, i32, ctypes.POINTER(dbl), i32],
        "hpt_set_messages": [P, i32, i32, ctypes.POINTER(dbl), i32],
        "hpt_get_meas_messages": [P, i32, i32, ctypes.POINTER(dbl), i32],
        "hpt_destroy": [P],
        "hpt_permute": [P, P, i32, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(i32), i32, P],
        "hpt_profile_gemm": [i32],
        "hpt_profile_gemm_read": [ctypes.POINTER(dbl)],
        "hpt_profile_read": [i32, ctypes.POINTER(dbl)],
        "hpt_run_batch": [ctypes.POINTER(ctypes.c_void_p), i32, ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_void_p)],
        "hpt_checkpoint_bytes": [P, ctypes.POINTER(u64)],
        "hpt_checkpoint_save": [P, P, u64, i32],
        "hpt_checkpoint_load": [P, P, u64, i32],
        "hpt_phase_timing": [P, i32],
        "hpt_phase_read": [P, ctypes.POINTER(dbl)],
        "hpt_gram64_workspace_bytes": [ctypes.c_int64, i32, ctypes.POINTER(u64)],
        "hpt_gram64": [P, ctypes.c_int64, i32, ctypes.c_int64, P, ctypes.c_int64, P, u64, P],
        "hpt_gram64_noalloc": [P, ctypes.c_int64, i32, ctypes.c_int64, P, ctypes.c_int64, P],
        "hpt_meas_learn_rows": [P, ctypes.POINTER(ctypes.c_int64)],
        "hpt_meas_features": [P, P, P, ctypes.c_int64],
        "hpt_meas_targets": [P, P, P, ctypes.c_int64],
        "hpt_set_meas_model": [P, P],
        "hpt_learn_forward": [P, P, ctypes.c_int64, P, P],
        "hpt_learn_backward": [P, P, P, P, ctypes.c_int64, P, P],
        "hpt_learn_adam": [P, P, P, P, i32, ctypes.c_float, P],
        "hpt_bf16_mfma_sum": [P, ctypes.c_float, P, P],
        "hpt_mode_product_f32": [P, P, P, i32, ctypes.c_int64, ctypes.c_int64, P],
        "hpt_autotune": [i32],
        "hpt_pauli_weights": [P, ctypes.POINTER(dbl), i32, ctypes.POINTER(dbl)],
        "hpt_autotune_report": [ctypes.c_char_p, u64, ctypes.POINTER(u64)],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    lib.hpt_strerror.argtypes = [ctypes.c_int]
    lib.hpt_strerror.restype = ctypes.c_char_p
    lib.hpt_last_hip_error.argtypes = []
    lib.hpt_last_hip_error.restype = ctypes.c_char_p
    return lib


lib = _load()

EXPORTED = ["hpt_config_default", "hpt_required_bytes", "hpt_state_bytes", "hpt_create",
            "hpt_reset", "hpt_step", "hpt_apply_field", "hpt_apply_bond", "hpt_gauge_bp",
            "hpt_measure", "hpt_get_chi", "hpt_get_bond_spectrum", "hpt_get_site_tensor",
            "hpt_set_site_tensor", "hpt_get_messages", "hpt_set_messages",
            "hpt_get_meas_messages", "hpt_destroy", "hpt_strerror", "hpt_last_hip_error",
            "hpt_permute", "hpt_profile_gemm", "hpt_profile_gemm_read", "hpt_profile_read", "hpt_run_batch",
            "hpt_checkpoint_bytes", "hpt_checkpoint_save", "hpt_checkpoint_load", "hpt_phase_timing",
            "hpt_phase_read", "hpt_gram64_workspace_bytes", "hpt_gram64", "hpt_gram64_noalloc",
            "hpt_meas_learn_rows", "hpt_meas_features", "hpt_meas_targets", "hpt_set_meas_model",
            "hpt_learn_forward", "hpt_learn_backward", "hpt_learn_adam", "hpt_bf16_mfma_sum",
            "hpt_mode_product_f32", "hpt_autotune", "hpt_autotune_report", "hpt_pauli_weights"]

HPT_MEM_HOST = 0
HPT_MEM_DEVICE = 1


def profile_gemm(enable=True):
    check(lib.hpt_profile_gemm(1 if enable else 0), "hpt_profile_gemm")


PROF_KINDS = {"gemm": 0, "gram64": 1, "mode": 2, "leggram": 3, "bsplit": 4}


def profile_gemm_read(kind=None):
    """Counters of one contraction kind ("gemm", "gram64", "mode", "leggram") or of all."""
    out = (ctypes.c_double * 4)()
    k = -1 if kind is None else PROF_KINDS[kind]
    check(lib.hpt_profile_read(k, out), "hpt_profile_read")
    return dict(launches=int(out[0]), ms=out[1], flops=out[2], bytes=out[3])


def run_batch(sims, nsteps, measure=True):
    """Advance independent handles concurrently (hpt_run_batch): sims[i] by
    nsteps[i] layers; returns, per run, the measurement after every layer (or
    None when measure is False).  Give each handle its own stream."""
    n = len(sims)
    if len(nsteps) != n:
        raise ValueError("one step count per handle")
    arr = (ctypes.c_void_p * n)(*[s.h.value for s in sims])
    ns = (ctypes.c_int32 * n)(*[int(k) for k in nsteps])
    outs, bufs = None, []
    if measure:
        bufs = [(HptMeasurement * max(int(k), 1))() for k in nsteps]
        outs = (ctypes.c_void_p * n)(*[ctypes.cast(b, ctypes.c_void_p).value for b in bufs])
    check(lib.hpt_run_batch(arr, n, ns, outs), "hpt_run_batch")
    if not measure:
        return None
    return [[b[k].as_dict() for k in range(int(nsteps[i]))] for i, b in enumerate(bufs)]


class HptError(RuntimeError):
    def __init__(self, code, where):
        msg = lib.hpt_strerror(code).decode()
        hip = lib.hpt_last_hip_error().decode()
        super().__init__(f"{where}: {msg} ({code})" + (f" [{hip}]" if code == -3 and hip else ""))
        self.code = code


def check(code, where):
    if code != 0:
        raise HptError(code, where)


def make_config(**kw):
    cfg = HptConfig()
    check(lib.hpt_config_default(ctypes.byref(cfg)), "hpt_config_default")
    names = {n for n, _ in HptConfig._fields_}
    for k, v in kw.items():
        if k == "precision" and isinstance(v, str):
            v = {"fp64": HPT_FP64, "fp32": HPT_FP32_MFMA, "fp32_mfma": HPT_FP32_MFMA, "bf16x6": HPT_FP32_BF16X6}[v]
        if k == "qr_mode" and isinstance(v, str):
            v = {"adaptive": HPT_QR_ADAPTIVE, "householder": HPT_QR_HOUSEHOLDER}[v]
        if k == "model_axes" and isinstance(v, str):
            v = {"paper": HPT_AXES_PAPER, "zzx": HPT_AXES_ZZX}[v]
        if k == "meas_init" and isinstance(v, str):
            v = {"uniform": HPT_BP_UNIFORM, "learned": HPT_BP_LEARNED}[v]
        if k == "bp_init" and isinstance(v, str):
            v = {"uniform": HPT_BP_UNIFORM, "warm": HPT_BP_WARM}[v]
        if k not in names:
            raise KeyError(k)
        setattr(cfg, k, v)
    return cfg


def required_bytes(cfg):
    n = ctypes.c_uint64()
    check(lib.hpt_required_bytes(ctypes.byref(cfg), ctypes.byref(n)), "hpt_required_bytes")
    return n.value


def state_bytes(cfg):
    n = ctypes.c_uint64()
    check(lib.hpt_state_bytes(ctypes.byref(cfg), ctypes.byref(n)), "hpt_state_bytes")
    return n.value


class Simulator:
    """One handle of libhpt on a CUDA/HIP device via PyTorch memory and stream."""

    def __init__(self, cfg=None, device="cuda:0", torch_arena=True, stream=None, **kw):
        import torch
        self.torch = torch
        self.cfg = cfg if cfg is not None else make_config(**kw)
        self.device = torch.device(device)
        torch.cuda.set_device(self.device)
        self.nbytes = required_bytes(self.cfg)
        self.arena = None
        ptr = None
        if torch_arena:
            self.arena = torch.empty(self.nbytes + 256, dtype=torch.uint8, device=self.device)
            base = self.arena.data_ptr()
            ptr = (base + 255) // 256 * 256
        # the handle's stream: the caller's (e.g. one per run of a batch) or torch's current one
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        check(lib.hpt_create(ctypes.byref(self.cfg), ptr, self.nbytes if ptr else 0,
                             ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)), "hpt_create")
        self.h = h
        Lx, Ly = self.cfg.Lx, self.cfg.Ly
        self.n_sites = Lx * Ly
        self.n_bonds = (Lx - 1) * Ly + Lx * (Ly - 1)

    def close(self):
        if getattr(self, "h", None):
            lib.hpt_destroy(self.h)
            self.h = None
            self.arena = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def reset(self):
        check(lib.hpt_reset(self.h), "hpt_reset")

    def step(self, n=1):
        check(lib.hpt_step(self.h, n), "hpt_step")

    def apply_field(self):
        check(lib.hpt_apply_field(self.h), "hpt_apply_field")

    def apply_bond(self, b):
        check(lib.hpt_apply_bond(self.h, b), "hpt_apply_bond")

    def gauge_bp(self, init=HPT_BP_UNIFORM):
        sw, de = ctypes.c_int32(), ctypes.c_double()
        check(lib.hpt_gauge_bp(self.h, init, ctypes.byref(sw), ctypes.byref(de)), "hpt_gauge_bp")
        return sw.value, de.value

    def measure(self):
        m = HptMeasurement()
        check(lib.hpt_measure(self.h, ctypes.byref(m)), "hpt_measure")
        return m.as_dict()

    def pauli_weights(self):
        """(n, (R_L1, R_L2, S_frac)): per-site non-identity Pauli weight and the
        spreading measures (hpt_pauli_weights)."""
        N = self.cfg.Lx * self.cfg.Ly
        n = np.zeros(N)
        st = np.zeros(3)
        P = ctypes.POINTER(ctypes.c_double)
        check(lib.hpt_pauli_weights(self.h, n.ctypes.data_as(P), N, st.ctypes.data_as(P)), "hpt_pauli_weights")
        return n, tuple(st)

    def chi(self, b):
        c = ctypes.c_int32()
        check(lib.hpt_get_chi(self.h, b, ctypes.byref(c)), "hpt_get_chi")
        return c.value

    def spectrum(self, b):
        n = ctypes.c_int32()
        check(lib.hpt_get_bond_spectrum(self.h, b, None, 0, ctypes.byref(n)), "hpt_get_bond_spectrum")
        out = np.zeros(n.value)
        check(lib.hpt_get_bond_spectrum(self.h, b, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                        n.value, ctypes.byref(n)), "hpt_get_bond_spectrum")
        return out

    def get_site(self, v):
        """Site tensor as a numpy array with axes (present legs U,D,L,R..., Pauli)."""
        dims = (ctypes.c_int32 * 5)()
        check(lib.hpt_get_site_tensor(self.h, v, None, 0, dims), "hpt_get_site_tensor")
        deg = self._deg(v)
        shape = tuple(dims[i] for i in range(deg + 1))
        buf = np.zeros(int(np.prod(shape)))
        check(lib.hpt_get_site_tensor(self.h, v, buf.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                      buf.size, dims), "hpt_get_site_tensor")
        return buf.reshape(shape, order="F")

    def set_site(self, v, T):
        T = np.asarray(T, dtype=np.float64)
        dims = (ctypes.c_int32 * 5)(*T.shape)
        flat = np.ascontiguousarray(T.ravel(order="F"))
        check(lib.hpt_set_site_tensor(self.h, v, flat.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                      dims), "hpt_set_site_tensor")

    def get_message(self, b, d):
        c = self.chi(b)
        out = np.zeros(c * c)
        check(lib.hpt_get_messages(self.h, b, d, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                   c * c), "hpt_get_messages")
        return out.reshape((c, c), order="F")

    def set_message(self, b, d, M):
        M = np.asarray(M, dtype=np.float64)
        flat = np.ascontiguousarray(M.ravel(order="F"))
        check(lib.hpt_set_messages(self.h, b, d, flat.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                   M.shape[0]), "hpt_set_messages")

    def get_meas_message(self, b, d):
        c = self.chi(b)
        out = np.zeros(c)
        check(lib.hpt_get_meas_messages(self.h, b, d, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                        c), "hpt_get_meas_messages")
        return out

    def checkpoint_bytes(self):
        n = ctypes.c_uint64()
        check(lib.hpt_checkpoint_bytes(self.h, ctypes.byref(n)), "hpt_checkpoint_bytes")
        return n.value

    @staticmethod
    def _buffer(buf):
        # (pointer, bytes, where) of a torch uint8 tensor (device or host) or a numpy uint8 array
        if isinstance(buf, np.ndarray):
            if buf.dtype != np.uint8 or not buf.flags["C_CONTIGUOUS"]:
                raise ValueError("checkpoint buffer: contiguous uint8 array")
            return buf.ctypes.data, buf.nbytes, HPT_MEM_HOST
        if buf.dtype.itemsize != 1 or not buf.is_contiguous():
            raise ValueError("checkpoint buffer: contiguous uint8 tensor")
        return buf.data_ptr(), buf.numel(), HPT_MEM_DEVICE if buf.is_cuda else HPT_MEM_HOST

    def save_checkpoint(self, buf=None):
        """Write the state image into buf (torch uint8 tensor on the device or
        host, or numpy uint8 array); a new numpy array when buf is None."""
        if buf is None:
            buf = np.zeros(self.checkpoint_bytes(), dtype=np.uint8)
        ptr, n, where = self._buffer(buf)
        check(lib.hpt_checkpoint_save(self.h, ctypes.c_void_p(ptr), n, where), "hpt_checkpoint_save")
        return buf

    def load_checkpoint(self, buf):
        ptr, n, where = self._buffer(buf)
        check(lib.hpt_checkpoint_load(self.h, ctypes.c_void_p(ptr), n, where), "hpt_checkpoint_load")

    def phase_timing(self, enable=True):
        check(lib.hpt_phase_timing(self.h, 1 if enable else 0), "hpt_phase_timing")

    def phase_read(self):
        out = (ctypes.c_double * 7)()
        check(lib.hpt_phase_read(self.h, out), "hpt_phase_read")
        return dict(gate_ms=out[0], gauge_ms=out[1], meas_ms=out[2], layers=int(out[3]),
                    gauge_sweeps=int(out[4]), measurements=int(out[5]), meas_sweeps=int(out[6]))

    # -- learned warm start of the measurement BP ---------------------------
    def learn_rows(self):
        n = ctypes.c_int64()
        check(lib.hpt_meas_learn_rows(self.h, ctypes.byref(n)), "hpt_meas_learn_rows")
        return n.value

    def meas_features(self):
        """(X, base) device tensors of the current state (float32)."""
        import torch
        n = self.learn_rows()
        X = torch.empty((n, LEARN_FEATURES), dtype=torch.float32, device=self.device)
        base = torch.empty(n, dtype=torch.float32, device=self.device)
        check(lib.hpt_meas_features(self.h, ctypes.c_void_p(X.data_ptr()), ctypes.c_void_p(base.data_ptr()), n),
              "hpt_meas_features")
        return X, base

    def meas_targets(self, base):
        import torch
        n = base.numel()
        T = torch.empty(n, dtype=torch.float32, device=self.device)
        check(lib.hpt_meas_targets(self.h, ctypes.c_void_p(base.data_ptr()), ctypes.c_void_p(T.data_ptr()), n),
              "hpt_meas_targets")
        return T

    def set_meas_model(self, params):
        """params: float32 device tensor of LEARN_PARAMS entries (kept alive here)."""
        self._meas_model = params
        check(lib.hpt_set_meas_model(self.h, ctypes.c_void_p(params.data_ptr() if params is not None else 0)),
              "hpt_set_meas_model")

    def _deg(self, v):
        Lx, Ly = self.cfg.Lx, self.cfg.Ly
        x, y = v % Lx, v // Lx
        return (y > 0) + (y < Ly - 1) + (x > 0) + (x < Lx - 1)


def gram64_workspace_bytes(m, n):
    out = ctypes.c_uint64()
    check(lib.hpt_gram64_workspace_bytes(m, n, ctypes.byref(out)), "hpt_gram64_workspace_bytes")
    return out.value


def gram64(X, G, workspace=None, stream=None):
    """G (float64, n x n) = X^T X for a float32 device matrix X viewed
    column-major as X.shape = (n, ldx) row-major storage, i.e. X[j] is column
    j of length m = ldx (hpt_gram64).  workspace: uint8 device tensor of at
    least gram64_workspace_bytes(m, n) bytes; allocated here when None."""
    import torch
    n, m = X.shape
    if X.dtype != torch.float32 or G.dtype != torch.float64 or not X.is_contiguous() or not G.is_contiguous():
        raise ValueError("gram64: contiguous float32 X and float64 G")
    if workspace is None:
        workspace = torch.empty(max(gram64_workspace_bytes(m, n), 1), dtype=torch.uint8, device=X.device)
    st = stream if stream is not None else torch.cuda.current_stream(X.device).cuda_stream
    check(lib.hpt_gram64(ctypes.c_void_p(X.data_ptr()), m, n, m, ctypes.c_void_p(G.data_ptr()), G.shape[1],
                         ctypes.c_void_p(workspace.data_ptr()), workspace.numel(), ctypes.c_void_p(st)), "hpt_gram64")


def autotune(mode):
    """Launch-shape autotuner: 1 on (default), 0 off, 2 forget (hpt_autotune)."""
    check(lib.hpt_autotune(int(mode)), "hpt_autotune")


def autotune_report():
    """The autotuner's shape classes: a list of (site, (k0, k1, k2), [best ms or
    None per variant], choice) (hpt_autotune_report)."""
    need = ctypes.c_uint64()
    check(lib.hpt_autotune_report(None, 0, ctypes.byref(need)), "hpt_autotune_report")
    buf = ctypes.create_string_buffer(int(need.value))
    check(lib.hpt_autotune_report(buf, len(buf), ctypes.byref(need)), "hpt_autotune_report")
    out = []
    for line in buf.value.decode().splitlines():
        head, tail = line.split(":", 1)
        site, *key = head.split()
        times, choice = tail.split("->")
        out.append((site, tuple(int(k) for k in key),
                    [None if t == "-" else float(t) for t in times.split()], int(choice)))
    return out


def mode_product_f32(src, S, inner, outer, stream=None):
    """dst[a, j, b] = sum_k S[j, k] src[a, k, b] (hpt_mode_product_f32) for
    float32 device tensors: src holds inner * n * outer values in column-major
    order (a fastest), S is n x n column-major (S.T row-major); returns dst of
    src's shape."""
    import torch
    n = S.shape[0]
    if src.dtype != torch.float32 or S.dtype != torch.float32 or not src.is_contiguous() or not S.is_contiguous():
        raise ValueError("mode_product_f32: contiguous float32 tensors")
    if src.numel() != inner * n * outer or S.numel() != n * n:
        raise ValueError("mode_product_f32: src must hold inner * n * outer values and S n * n")
    dst = torch.empty_like(src)
    check(lib.hpt_mode_product_f32(ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()),
                                   ctypes.c_void_p(S.data_ptr()), n, inner, outer, _stream(src, stream)),
          "hpt_mode_product_f32")
    return dst


def _stream(t, stream):
    import torch
    return ctypes.c_void_p(stream if stream is not None else torch.cuda.current_stream(t.device).cuda_stream)


def learn_forward(params, X, stream=None):
    import torch
    y = torch.empty(X.shape[0], dtype=torch.float32, device=X.device)
    check(lib.hpt_learn_forward(ctypes.c_void_p(params.data_ptr()), ctypes.c_void_p(X.data_ptr()), X.shape[0],
                                ctypes.c_void_p(y.data_ptr()), _stream(X, stream)), "hpt_learn_forward")
    return y


def learn_backward(params, X, y, t, stream=None):
    """(grad [LEARN_PARAMS], loss tensor [1]) as device tensors."""
    import torch
    g = torch.empty(LEARN_PARAMS + 1, dtype=torch.float32, device=X.device)
    check(lib.hpt_learn_backward(ctypes.c_void_p(params.data_ptr()), ctypes.c_void_p(X.data_ptr()),
                                 ctypes.c_void_p(y.data_ptr()), ctypes.c_void_p(t.data_ptr()), X.shape[0],
                                 ctypes.c_void_p(g.data_ptr()), _stream(X, stream)), "hpt_learn_backward")
    return g[:LEARN_PARAMS], g[LEARN_PARAMS:]


def learn_adam(params, m, v, grad_full, step, lr, stream=None):
    check(lib.hpt_learn_adam(ctypes.c_void_p(params.data_ptr()), ctypes.c_void_p(m.data_ptr()),
                             ctypes.c_void_p(v.data_ptr()), ctypes.c_void_p(grad_full.data_ptr()), int(step),
                             float(lr), _stream(params, stream)), "hpt_learn_adam")


def permute(src, dst, perm, stream=None):
    """Device permutation of a column-major torch tensor (dims = src.shape[::-1]
    viewed column-major) into dst, through hpt_permute."""
    import torch
    dims = list(src.shape)
    nd = len(dims)
    d = (ctypes.c_int64 * nd)(*dims)
    p = (ctypes.c_int32 * nd)(*perm)
    st = stream if stream is not None else torch.cuda.current_stream(src.device).cuda_stream
    check(lib.hpt_permute(ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()), nd, d, p,
                          src.element_size(), ctypes.c_void_p(st)), "hpt_permute")
