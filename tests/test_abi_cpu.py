"""Host-only checks of the C ABI: the library loads, exports every symbol the
header declares, validates configs and evaluates its memory model without a GPU."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def hpt():
    from paper_2606_30985_amd import hpt as h
    return h


def test_every_declared_symbol_is_exported(hpt):
    hdr = open(os.path.join(ROOT, "include", "hpt.h")).read()
    declared = set(re.findall(r"\b(hpt_[a-z_0-9]+)\s*\(", hdr))
    assert len(declared) >= 20
    for name in declared:
        assert hasattr(hpt.lib, name), name
    assert declared == set(hpt.EXPORTED)


def test_config_defaults(hpt):
    c = hpt.make_config()
    assert (c.Lx, c.Ly, c.chi_max) == (3, 3, 8)
    assert c.eps_cut == -1.0 and c.bp_alpha == 0.5 and c.bp_tol == 1e-10
    assert c.cx == -1 and c.cy == -1 and c.trap_sweeps == 30
    assert c.trap_retry == 0 and c.trap_alpha == -1.0 and c.qr_rank_tol == -1.0


@pytest.mark.parametrize("kw", [dict(Lx=1, Ly=1), dict(Lx=0, Ly=3), dict(dt=0.0), dict(chi_max=0),
                                dict(cx=3, cy=0), dict(precision=7), dict(bp_alpha=0.0),
                                dict(bp_tol=-1.0), dict(chi_max=300), dict(trap_retry=2), dict(trap_alpha=1.5)])
def test_invalid_configs_rejected(hpt, kw):
    c = hpt.make_config(**kw)
    n = ctypes.c_uint64()
    assert hpt.lib.hpt_required_bytes(ctypes.byref(c), ctypes.byref(n)) == -1


def _paper_state_floats(k, l, chi):
    # paper, Sec. "Analytic Memory Model", Eq. mem_psi (in units of sizeof(float)):
    # (4 chi^2 + 2 (k + l - 4) chi^3 + (k - 2)(l - 2) chi^4) * D
    return (4 * chi ** 2 + 2 * (k + l - 4) * chi ** 3 + (k - 2) * (l - 2) * chi ** 4) * 4


@pytest.mark.parametrize("k,l,chi", [(3, 3, 8), (4, 4, 60), (10, 10, 100), (11, 11, 100), (5, 7, 13)])
def test_state_term_matches_paper_memory_model(hpt, k, l, chi):
    for prec, size in ((0, 8), (1, 4), (2, 4)):
        c = hpt.make_config(Lx=k, Ly=l, chi_max=chi, precision=prec)
        assert hpt.state_bytes(c) == _paper_state_floats(k, l, chi) * size


def test_required_bytes_fit_the_large_instance(hpt):
    # 10x10 at chi 100 in the float32 form fits well inside 288 GB of HBM,
    # and the float64 reference run fits as well
    c32 = hpt.make_config(Lx=10, Ly=10, chi_max=100, precision=1)
    c64 = hpt.make_config(Lx=10, Ly=10, chi_max=100, precision=0)
    b32, b64 = hpt.required_bytes(c32), hpt.required_bytes(c64)
    s32 = hpt.state_bytes(c32)
    assert s32 == pytest.approx(102.9e9, rel=0.01)
    assert b32 < 130e9
    assert b64 < 260e9
    assert b64 > hpt.state_bytes(c64)
    # the split-bf16 form keeps the float32 layout
    cs = hpt.make_config(Lx=10, Ly=10, chi_max=100, precision="bf16x6")
    assert hpt.required_bytes(cs) == b32


def test_strerror(hpt):
    assert hpt.lib.hpt_strerror(-2).decode() == "arena too small"
    assert hpt.lib.hpt_strerror(0).decode() == "ok"


def test_gram64_workspace_and_argument_checks_without_gpu(hpt):
    # 10^6 x 400 (an interior site at chi = 100): 32 row splits of 400^2 doubles
    assert hpt.gram64_workspace_bytes(10 ** 6, 400) == 32 * 400 * 400 * 8
    assert hpt.gram64_workspace_bytes(1000, 0) == 0
    assert hpt.gram64_workspace_bytes(10, 3) == 3 * 3 * 8
    assert hpt.gram64_workspace_bytes(10 ** 7, 2000) <= hpt_part_max()
    P = ctypes.c_void_p
    # every refusal happens before any launch
    assert hpt.lib.hpt_gram64(P(16), -1, 3, 4, P(16), 3, P(16), 1 << 20, None) == -1
    assert hpt.lib.hpt_gram64(P(16), 8, 3, 4, P(16), 3, P(16), 1 << 20, None) == -1
    assert hpt.lib.hpt_gram64(P(16), 8, 3, 8, P(16), 2, P(16), 1 << 20, None) == -1
    assert hpt.lib.hpt_gram64(None, 8, 3, 8, P(16), 3, P(16), 1 << 20, None) == -1
    assert hpt.lib.hpt_gram64(P(16), 8, 3, 8, P(16), 3, P(16), 8, None) == -2
    assert hpt.lib.hpt_gram64(P(16), 8, 0, 8, None, 0, None, 0, None) == 0


def hpt_part_max():
    hdr = open(os.path.join(ROOT, "include", "hpt.h")).read()
    m = re.search(r"#define HPT_GRAM64_PART_MAX \((\d+)ull << (\d+)\)", hdr)
    return int(m.group(1)) << int(m.group(2))


@pytest.mark.parametrize("kw", [dict(model_axes=2), dict(model_axes=-1), dict(svd_max_sweeps=-3)])
def test_invalid_axes_and_sweep_caps_rejected(hpt, kw):
    c = hpt.make_config(**kw)
    n = ctypes.c_uint64()
    assert hpt.lib.hpt_required_bytes(ctypes.byref(c), ctypes.byref(n)) == -1


def test_short_arena_refused_without_touching_the_device(hpt):
    # the arena is checked against the memory model before any HIP call, so a
    # fake device address is never dereferenced
    c = hpt.make_config(Lx=4, Ly=4, chi_max=12)
    need = hpt.required_bytes(c)
    h = ctypes.c_void_p()
    assert hpt.lib.hpt_create(ctypes.byref(c), ctypes.c_void_p(1 << 20), need - 1, None, ctypes.byref(h)) == -2
    assert not h.value
    assert hpt.make_config(model_axes="zzx").model_axes == 1


def test_flag_bits_match_the_header():
    # the flag table the host code uses without loading the library
    from paper_2606_30985_amd.flags import FLAGS
    hdr = open(os.path.join(ROOT, "include", "hpt.h")).read()
    defs = {m.group(1): 1 << int(m.group(2)) for m in re.finditer(r"#define HPT_FLAG_([A-Z_]+)\s+\(1u << (\d+)\)", hdr)}
    assert defs == FLAGS


def test_trap_scan_does_not_load_the_library():
    # importing the host post-processing must not load libhpt.so (the GPU
    # runtime it links would be loaded before torch's)
    import subprocess
    import sys
    code = ("import sys; sys.path.insert(0, %r); import paper_2606_30985_amd.traps; "
            "print('paper_2606_30985_amd.hpt' in sys.modules)" % ROOT)
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and r.stdout.strip() == "False", r.stdout + r.stderr
