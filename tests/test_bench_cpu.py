"""Host-only checks of bench.py: the multi-GPU refusal, the counter-based
traffic lookup (reported only while the kernel source matches the hash
recorded with the counters), the roofline peaks, the lattice bookkeeping
behind the per-class rates and slice bytes, and the summaries of rocprofv3
kernel traces and counter runs (on small synthetic CSV files)."""

import os
import shutil
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stdout


def test_traffic_ratio_follows_the_kernel_source(tmp_path, monkeypatch):
    sys.path.insert(0, ROOT)
    import bench
    assert bench.traffic_ratio("unknown") is None
    r = bench.traffic_ratio("mode")
    if r is None:
        import pytest
        pytest.skip("the kernel source changed since the counters were taken")
    assert 1.0 <= r < 3.0
    # a copy of the tree whose kernel source differs: no traffic figure
    (tmp_path / "profiles").mkdir()
    (tmp_path / "paper_2606_30985_amd" / "csrc").mkdir(parents=True)
    shutil.copy(os.path.join(ROOT, "profiles", "mode_product_kernel_10x10_chi100_pmc.md"), tmp_path / "profiles")
    src = open(os.path.join(ROOT, "paper_2606_30985_amd", "csrc", "k_gemm.hip")).read()
    (tmp_path / "paper_2606_30985_amd" / "csrc" / "k_gemm.hip").write_text(src + "\n// changed\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.traffic_ratio("mode") is None


def test_roofline_peak_per_kind():
    sys.path.insert(0, ROOT)
    import bench
    assert bench.roofline_peak("mode", "fp32") == 157.3
    assert bench.roofline_peak("gemm", "bf16x6") == 157.3
    assert bench.roofline_peak("gram64", "fp32") == 78.6
    assert bench.roofline_peak("mode", "fp64") == 78.6
    assert abs(bench.roofline_peak("bsplit", "bf16x6") - 2500.0 / 6) < 1e-9



def test_bond_classes_of_the_10x10_lattice():
    sys.path.insert(0, ROOT)
    import bench
    cl = bench.bond_classes(10)
    assert {k: len(v) for k, v in cl.items()} == {"interior-interior": 112, "interior-edge": 32,
                                                  "edge-edge": 28, "corner": 8}
    assert sorted(sum(cl.values(), [])) == list(range(180))
    cb = bench.centre_bonds(10)
    assert len(cb) == 4
    # horizontal bonds ((3,4),(4,4)) and ((4,4),(5,4)); vertical ((4,3),(4,4)) and ((4,4),(4,5))
    assert cb == [4 * 9 + 3, 4 * 9 + 4, 90 + 3 * 10 + 4, 90 + 4 * 10 + 4]


def test_site_bonds_and_measurement_bytes():
    sys.path.insert(0, ROOT)
    import bench
    sb = bench.site_bonds(10)
    assert sorted(len(l) for l in sb).count(4) == 64 and sorted(len(l) for l in sb).count(2) == 4
    # every bond appears at its two end sites
    from collections import Counter
    cnt = Counter(b for l in sb for b in l)
    assert set(cnt.values()) == {2} and len(cnt) == 180
    # all bonds at chi: 64 chi^4 + 32 chi^3 + 4 chi^2 entries
    assert bench.meas_sweep_bytes([100] * 180, 10, 4) == 4 * (64 * 100 ** 4 + 32 * 100 ** 3 + 4 * 100 ** 2)


def test_site_bonds_follow_the_lattice_numbering():
    # the bench's per-site bond lists follow the lattice numbering of the
    # ABI (checked against the oracle's lattice), and one measurement sweep
    # reads every site's pinned slice (product of its bond dimensions) once
    sys.path.insert(0, ROOT)
    import bench
    from oracle.lattice import Lattice
    for L in (2, 3, 10):
        lat = Lattice(L, L)
        assert bench.site_bonds(L) == [[b for (_, _, b) in lat.legs[v]] for v in range(L * L)]
    chis = [100] * 180
    assert bench.meas_sweep_bytes(chis, 10, 4) == 4 * (64 * 100 ** 4 + 32 * 100 ** 3 + 4 * 100 ** 2)
    assert bench.meas_sweep_bytes([1] * 180, 10, 8) == 8 * 100


def _write_csv(path, header, rows):
    import csv
    path.parent.mkdir(parents=True, exist_ok=True)
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(header)
        w.writerows(rows)


def test_trace_summary_counts_only_the_window_between_the_markers(tmp_path, capsys):
    sys.path.insert(0, ROOT)
    import bench
    hdr = ["Kernel_Name", "Start_Timestamp", "End_Timestamp"]
    rows = [["hpt::(anonymous namespace)::mode_product_kernel<112, 25>", 0, 50],     # before the first marker
            ["void marker_kernel()", 100, 110],
            ["hpt::(anonymous namespace)::mode_product32_kernel<112, 25>", 200, 1200],
            ["hpt::(anonymous namespace)::mode_product_f64acc_kernel", 1300, 1400],
            ["hpt::(anonymous namespace)::gram64_kernel<true>", 1500, 3500],
            ["void marker_kernel()", 4000, 4010],
            ["hpt::(anonymous namespace)::gram64_kernel<true>", 5000, 9000]]          # after the second marker
    _write_csv(tmp_path / "run" / "x_kernel_trace.csv", hdr, rows)
    bench.summarize_trace(str(tmp_path))
    out = capsys.readouterr().out
    assert "window: 3 dispatches between the markers" in out
    assert "kernel busy 0.000 s" in out
    assert "mode: 1 dispatches, 0.00 ms, average 1.0 us" in out        # the f64acc kernel is its own family
    assert "mode_f64acc: 1 dispatches" in out
    assert "gram64: 1 dispatches, 0.00 ms, average 2.0 us" in out


def test_pmc_summary_sets_the_calibration_copy_apart(tmp_path, capsys):
    sys.path.insert(0, ROOT)
    import bench
    hdr = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]
    rows = [[1, "hpt::(anonymous namespace)::permute_generic_kernel(hpt::PermMeta)", "FETCH_SIZE", 1024],
            [2, "hpt::(anonymous namespace)::mode_product32_kernel<112, 25>(float const*)", "FETCH_SIZE", 10],
            [3, "hpt::(anonymous namespace)::mode_product_kernel<16, 4>(float const*)", "FETCH_SIZE", 5],
            [4, "hpt::(anonymous namespace)::mode_product_f64acc_kernel(double const*)", "FETCH_SIZE", 7],
            [5, "hpt::(anonymous namespace)::permute_generic_kernel(hpt::PermMeta)", "FETCH_SIZE", 3]]
    _write_csv(tmp_path / "p" / "y_counter_collection.csv", hdr, rows)
    bench.summarize_pmc(str(tmp_path))
    out = capsys.readouterr().out.splitlines()
    assert "FETCH_SIZE calibration_copy 1024" in out
    assert "FETCH_SIZE mode dispatches 2 sum 1.500000e+01" in out
    assert "FETCH_SIZE mode_f64acc dispatches 1 sum 7.000000e+00" in out
    assert "FETCH_SIZE permute dispatches 1 sum 3.000000e+00" in out
    assert "FETCH_SIZE kernel mode_product32_kernel<112, 25> dispatches 1 sum 1.000000e+01" in out
