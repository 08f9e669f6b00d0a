"""The benchmark's measurement bookkeeping on the CPU: algorithmic bytes, the
roofline of the dominant kernel and its per-kernel table, and the rocprofv3
summary (launch selection by grid, copy-calibrated traffic) on a synthetic
profiler output directory."""
import csv
import os

import pytest

import bench

HEAD = "heat3d_255_N64_lognormal"


def test_algorithmic_bytes_of_the_headline_kernels():
    dims = bench.level_dims(3, 255, 64, 1)
    n0, n1 = 255 ** 3, 127 ** 3
    kap = lambda b: 257 ** 3 * b  # noqa: E731  (one coefficient field on the nodes)
    # residual: u, p, F read in float64, r written in the storage type
    assert bench.algorithmic_bytes("k_resid_tile<a3>", 0, dims, 4) == 64 * n0 * (3 * 8 + 4) + kap(8)
    # down-sweep: fine b in, coarse b out, one field
    assert bench.algorithmic_bytes("k_mg_down_p3", 0, dims, 4) == 64 * (n0 + n1) * 4 + kap(4)
    # up-sweeps: b, e in and out stored, or b, e in and the float64 p read and written
    assert bench.algorithmic_bytes("k_mg_up_p3<store>", 0, dims, 4) == 64 * (2 * n0 + n1) * 4 + kap(4)
    assert bench.algorithmic_bytes("k_mg_up_p3<add64>", 0, dims, 2) == 64 * (n0 + n1) * 2 + 64 * n0 * 16 + kap(4)
    assert bench.algorithmic_bytes("k_time_fft2<a6,add64>", 0, dims, 4) == 64 * n0 * (4 + 16)
    assert bench.algorithmic_bytes("k_finalize", 0, dims, 4) is None


def test_roofline_takes_the_largest_summed_time_and_reports_every_kernel():
    dims = bench.level_dims(3, 255, 64, 1)
    rep = [dict(kernel="k_mg_down_p3", level=0, launches=12, avg_ms=2.0, total_ms=24.0),
           dict(kernel="k_resid_tile<a3>", level=0, launches=4, avg_ms=8.0, total_ms=32.0),
           dict(kernel="k_pair_norms<3, 1, 1>", level=0, launches=1, avg_ms=40.0, total_ms=40.0),
           dict(kernel="k_finalize", level=0, launches=4, avg_ms=0.2, total_ms=0.8)]
    roof, table = bench.roofline(rep, dims, 4, HEAD, "f32")
    # the residual-norm pass of the returned pair runs once per solve: never the dominant kernel
    assert roof["kernel"] == "k_resid_tile<a3>"
    b = bench.algorithmic_bytes("k_resid_tile<a3>", 0, dims, 4)
    assert roof["achieved"] == pytest.approx(b / 8e-3 / 1e9)
    assert roof["frac"] == pytest.approx(roof["achieved"] / bench.HBM_PEAK_GBS)
    assert [e["kernel"] for e in table] == ["k_resid_tile<a3>", "k_mg_down_p3", "k_finalize"]
    assert table[1]["frac"] == pytest.approx(bench.algorithmic_bytes("k_mg_down_p3", 0, dims, 4) / 2e-3 / 1e9 / 8000)
    assert "frac" not in table[2]
    # traffic only while the kernel sources hash to the recorded value
    sha_ok = bench.kernel_sources_sha256() == bench._SRC_SHA
    m = bench.MEASURED_TRAFFIC[(HEAD, "f32", "k_resid_tile<a3>", 0)]
    assert roof["traffic"] == (m["bytes"] if sha_ok else None)
    assert os.path.exists(os.path.join(bench.ROOT, m["profile"]))


def _write(path, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=list(rows[0]))
        w.writeheader()
        w.writerows(rows)


def _profile_dir(tmp_path):
    d = str(tmp_path / "prof")
    k = "void stp::k_resid_tile<3, float, 1, 1, 1>(stp::ResidJob const*, int)"
    # autotuner candidates (other grids) first, then the timed schedule
    launches = [(4096, 10_000), (8192, 9_000), (2048, 8_000), (2048, 8_200)]
    trace, p1, p2 = [], [], []
    for i, (g, ns) in enumerate(launches):
        trace.append(dict(Kernel_Name=k, Start_Timestamp=1000 * i, End_Timestamp=1000 * i + ns,
                          Grid_Size_X=g, Grid_Size_Y=1, Grid_Size_Z=1))
        p1.append(dict(Kernel_Name=k, Grid_Size=g, Counter_Name="FETCH_SIZE", Counter_Value=100.0 * (i + 1)))
        p2.append(dict(Kernel_Name=k, Grid_Size=g, Counter_Name="WRITE_SIZE", Counter_Value=10.0 * (i + 1)))
    _write(os.path.join(d, "trace", "run_kernel_trace.csv"), trace)
    _write(os.path.join(d, "trace", "run_kernel_stats.csv"),
           [dict(Name=k, Calls=4, AverageNs=8800, MinNs=8000, MaxNs=10000, Percentage=100.0)])
    _write(os.path.join(d, "p1", "run_counter_collection.csv"), p1)
    _write(os.path.join(d, "p2", "run_counter_collection.csv"), p2)
    # the calibration copy reads half its bytes per FETCH_SIZE KiB and all of them per WRITE_SIZE KiB
    cb = bench.COPY_ELEMS * 8 / 1024
    _write(os.path.join(d, "c1", "run_counter_collection.csv"),
           [dict(Kernel_Name="copyBuffer", Grid_Size=10 ** 6, Counter_Name="FETCH_SIZE", Counter_Value=cb / 2)])
    _write(os.path.join(d, "c2", "run_counter_collection.csv"),
           [dict(Kernel_Name="copyBuffer", Grid_Size=10 ** 6, Counter_Name="WRITE_SIZE", Counter_Value=cb)])
    return d


def test_profile_summary_selects_the_timed_schedule_and_scales_the_counters(tmp_path, capsys):
    d = _profile_dir(tmp_path)
    bench.summarize_profile(d, "k_resid_tile<3, float, 1", 1, final_grid=True)
    out = capsys.readouterr().out
    # only the two launches with the last launch's grid (2048): 8.0 and 8.2 us
    assert "| 2 | 8.1 | 8.0 | 8.2 |" in out
    # FETCH_SIZE 300 and 400 KiB -> 350 KiB x 1024 x 2; WRITE_SIZE 30 and 40 -> 35 KiB x 1024 x 1
    assert f"| HBM bytes read | {350 * 1024 * 2:,} |" in out
    assert f"| HBM bytes written | {35 * 1024:,} |" in out
    bench.summarize_profile(d, "k_resid_tile<3, float, 1", 1, final_grid=False)
    out = capsys.readouterr().out
    assert "| 4 | 8800.0 |" not in out and "| 4 | 8.8 | 8.0 | 10.0 |" in out
    assert f"| HBM bytes read | {250 * 1024 * 2:,} |" in out
