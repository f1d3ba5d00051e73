"""Checkpoint/resume and per-phase timing through the C ABI.

A handle resumed from a checkpoint image continues bit for bit like the handle
that wrote it (FP64 form from a host image into a fresh handle, FP32 form from
a device image into the same handle after it ran on); images of another
configuration, truncated images and short buffers are refused."""

import numpy as np
import pytest

from tests.gpu_util import load_hpt

pytestmark = pytest.mark.gpu


def _layers(sim, n):
    out = []
    for _ in range(n):
        sim.step(1)
        out.append(sim.measure())
    return out


def _state(sim):
    sites = [sim.get_site(v) for v in range(sim.n_sites)]
    msgs = [sim.get_message(b, d) for b in range(sim.n_bonds) for d in range(2)]
    return sites, msgs


def test_fp64_resume_from_host_image_is_bit_identical():
    hpt = load_hpt()
    cfg = dict(Lx=3, Ly=3, chi_max=8, dt=0.05, precision="fp64", bp_init="warm", bp_tol=1e-10)
    a = hpt.Simulator(**cfg)
    _layers(a, 3)
    img = a.save_checkpoint()
    assert img.nbytes == a.checkpoint_bytes()
    ra = _layers(a, 4)
    sa = _state(a)
    b = hpt.Simulator(**cfg)
    b.load_checkpoint(img)
    rb = _layers(b, 4)
    sb = _state(b)
    for x, y in zip(ra, rb):
        assert x["step"] == y["step"]
        assert x["C"] == y["C"], (x["step"], x["C"], y["C"])
        assert x["gauge_sweeps"] == y["gauge_sweeps"] and x["meas_sweeps"] == y["meas_sweeps"]
    for x, y in zip(sa[0] + sa[1], sb[0] + sb[1]):
        assert np.array_equal(x, y)
    a.close()
    b.close()


def test_fp32_resume_from_device_image_is_bit_identical():
    hpt = load_hpt()
    import torch
    cfg = dict(Lx=4, Ly=4, chi_max=20, dt=0.05, precision="fp32", bp_init="warm", bp_tol=1e-5,
               meas_tol=1e-10, meas_max_sweeps=400)
    sim = hpt.Simulator(**cfg)
    _layers(sim, 10)
    buf = torch.empty(sim.checkpoint_bytes() + 1000, dtype=torch.uint8, device="cuda")
    sim.save_checkpoint(buf)
    first = _layers(sim, 3)
    s1 = _state(sim)
    sim.load_checkpoint(buf)
    assert sim.measure()["step"] == 10
    again = _layers(sim, 3)
    s2 = _state(sim)
    assert [r["C"] for r in first] == [r["C"] for r in again]
    for x, y in zip(s1[0] + s1[1], s2[0] + s2[1]):
        assert np.array_equal(x, y)
    sim.close()


def test_bad_images_are_refused():
    hpt = load_hpt()
    sim = hpt.Simulator(Lx=3, Ly=3, chi_max=8, precision="fp64")
    _layers(sim, 2)
    img = sim.save_checkpoint()
    short = np.zeros(img.nbytes - 8, dtype=np.uint8)
    with pytest.raises(hpt.HptError) as e:
        sim.save_checkpoint(short)
    assert e.value.code == -2
    with pytest.raises(hpt.HptError) as e:
        sim.load_checkpoint(img[: img.nbytes // 2].copy())
    assert e.value.code == -1
    bad = img.copy()
    bad[0] ^= 0xFF
    with pytest.raises(hpt.HptError) as e:
        sim.load_checkpoint(bad)
    assert e.value.code == -1
    other = hpt.Simulator(Lx=3, Ly=3, chi_max=6, precision="fp64")
    with pytest.raises(hpt.HptError) as e:
        other.load_checkpoint(img)
    assert e.value.code == -1
    f32 = hpt.Simulator(Lx=3, Ly=3, chi_max=8, precision="fp32")
    with pytest.raises(hpt.HptError) as e:
        f32.load_checkpoint(img)
    assert e.value.code == -1
    # a refused image leaves the handle as it was
    assert f32.measure()["step"] == 0 and other.measure()["step"] == 0
    for s in (sim, other, f32):
        s.close()


def test_phase_timing_counts_layers_and_sweeps():
    hpt = load_hpt()
    sim = hpt.Simulator(Lx=4, Ly=4, chi_max=12, precision="fp32", bp_tol=1e-8)
    sim.phase_timing(True)
    recs = _layers(sim, 3)
    p = sim.phase_read()
    assert p["layers"] == 3 and p["measurements"] == 3
    assert p["gauge_sweeps"] == sum(r["gauge_sweeps"] for r in recs)
    assert p["meas_sweeps"] == sum(r["meas_sweeps"] for r in recs)
    assert p["gate_ms"] > 0 and p["gauge_ms"] > 0 and p["meas_ms"] > 0
    sim.phase_timing(True)   # enabling again clears the totals
    assert sim.phase_read()["layers"] == 0
    sim.phase_timing(False)
    sim.step(1)
    assert sim.phase_read()["layers"] == 0
    sim.close()
