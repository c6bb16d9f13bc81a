"""Host logic of the measurement tools (no GPU): bench.py's byte accounting and
its one-GPU guard, the traffic summary it reads, and the rocprofv3 summaries."""
import os
import subprocess
import sys

import pytest

import bench
from paper_2601_18443_amd import prof_summary as PS

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_before_any_gpu_work():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_algorithmic_bytes_per_cell_update():
    # populations read + write, nu-tilde read + write, wall distance (FP64), flag byte
    assert bench.lup_bytes("f32", 0, 8) == 9 * 4 * 2 + 4 * 2 + 8 + 1 == 89
    assert bench.lup_bytes("f16", 3, 8) == 9 * 2 * 2 + 4 * 2 + 8 + 1 == 53
    assert bench.lup_bytes("f16s", 3, 8) == bench.lup_bytes("bf16", 3, 8) == 53
    assert bench.lup_bytes("f64", 0, 1) == 9 * 8 * 2 + 8 * 2 + 8 + 1 == 169
    # mixed storage: FP32 on the two finest levels only
    assert [bench.lup_bytes("mixeds", l, 5) for l in range(5)] == [53, 53, 53, 89, 89]
    # the kernel's own bytes: the wall distance in the arithmetic precision, plus the
    # stored rho, u (3 x CT written) and the stencil's u (2 x CT read)
    assert bench.lup_bytes("f32", 0, 8, bench.IMPL_BYTES) == 72 + 8 + 4 + 1 + 12 + 8 == 105
    assert bench.lup_bytes("f16s", 0, 8, bench.IMPL_BYTES) == 36 + 8 + 4 + 1 + 12 + 8 == 69

    class Sim:
        def level_info(self, l):
            return {"n_fluid": [100, 40, 7][l]}
    # every level l updates its cells 2^l times per coarse step
    assert bench.step_bytes("mixed", Sim(), 3, repeat=2) == 2 * (53 * 100 + 89 * 40 * 2 + 89 * 7 * 4)


def _write_traffic(path, sha, storage="f32", hbm=81000000):
    with open(path, "w") as fh:
        fh.write(f"# summary\nsource_sha256 = {sha}\nstorage = {storage}\nhbm_bytes_per_launch = {hbm}\n")


def test_traffic_is_read_only_for_the_sources_it_was_measured_on(tmp_path, monkeypatch):
    f = str(tmp_path / "traffic.txt")
    monkeypatch.setattr(bench, "TRAFFIC_FILE", f)
    assert bench.measured_traffic("f32") is None                  # no summary
    _write_traffic(f, "0000000000000000")
    assert bench.measured_traffic("f32") is None                  # other sources
    _write_traffic(f, bench.kernel_source_hash(), storage="f16")
    assert bench.measured_traffic("f32") is None                  # other storage
    _write_traffic(f, bench.kernel_source_hash())
    assert bench.measured_traffic("f32") == 81000000.0


def test_source_hash_ignores_comments_and_layout(tmp_path, monkeypatch):
    a, b, c = (str(tmp_path / n) for n in ("a.hip", "b.hip", "c.hip"))
    with open(a, "w") as fh:
        fh.write("int f(int x) {\n  return x + 1;  // one more\n}\n/* note */\n")
    with open(b, "w") as fh:
        fh.write("int f(int x)   { return x + 1; }\n")
    with open(c, "w") as fh:
        fh.write("int f(int x) { return x + 2; }\n")
    hashes = []
    for f in (a, b, c):
        monkeypatch.setattr(PS, "SOURCES", [f])
        hashes.append(PS.kernel_source_hash())
    assert hashes[0] == hashes[1] != hashes[2]


def test_stats_summary_averages_the_timed_dispatches(tmp_path):
    d = tmp_path / "ks"
    d.mkdir()
    with open(d / "run_kernel_stats.csv", "w") as fh:
        fh.write('"Name","Calls","TotalDurationNs","AverageNs","Percentage","MinNs","MaxNs"\n')
        fh.write('"void lbr::k_step_batch<float, float, 4>(x)",4,100000,25000,90.0,10000,40000\n')
        fh.write('"k_geometry(y)",1,11000,11000,10.0,11000,11000\n')
    with open(d / "run_kernel_trace.csv", "w") as fh:
        fh.write('"Kernel_Name","Start_Timestamp","End_Timestamp","Grid_Size_X"\n')
        for t0, dur in ((0, 10000), (100000, 40000), (200000, 20000), (300000, 30000)):
            fh.write(f'"void lbr::k_step_batch<float, float, 4>(x)",{t0},{t0 + dur},1024\n')
    out = PS.stats(str(d), "rocprofv3 ...", tail=3)
    assert "k_step_batch<float, float, 4>" in out
    assert "the last 3 dispatches" in out and "average 30.00 us" in out
    assert "1024" in out and "25.00" in out          # per launch size: 4 calls, 25 us on average


@pytest.mark.parametrize("name,short", [
    ("void lbr::(anonymous namespace)::k_step_batch<__half, float, 4>(lbr::StepArgs<__half, float> const*)",
     "k_step_batch<half, float, 4>"),
    ("void lbr::(anonymous namespace)::k_step_batch_mixed<8>(lbr::StepArgs<float, float> const*)",
     "k_step_batch_mixed<8>"),
    ("__amd_rocclr_copyBuffer", "__amd_rocclr_copyBuffer"),
])
def test_kernel_names_are_shortened(name, short):
    assert PS.short_name(name) == short


def test_gap_summary_of_a_dispatch_stream(tmp_path):
    """Two super steps of three launches: 10 us kernels, 2 us between the
    launches of a super step, 5 us between the super steps."""
    d = tmp_path / "tr"
    d.mkdir()
    with open(d / "run_kernel_trace.csv", "w") as fh:
        fh.write('"Kernel_Name","Start_Timestamp","End_Timestamp","Grid_Size_X"\n')
        t = 0
        for sup in range(2):
            for k in range(3):
                fh.write(f'"void lbr::k_step_batch<float, float, 4>(x)",{t},{t + 10000},1024\n')
                t += 10000 + (2000 if k < 2 else 5000)
        fh.write('"k_geometry(y)",0,1,64\n')

    class A:
        dir, cmd, kernel, skip, first, per_step = str(d), "rocprofv3 ...", "k_step_batch", 0, 6, 3
    out = PS.gaps(A())
    assert "span_us_per_super_step = 34.00" in out
    assert "kernel_us_per_super_step = 30.00" in out
    assert "gaps_inside_us_per_super_step = 4.00" in out
    assert "gap_between_super_steps_us = 5.00" in out
    assert "gaps_over_span = 0.1781" in out          # (2 x 4 + 5) / (2 x 34 + 5)


def test_default_line_runs_the_library_tiles_on_one_gpu():
    """With no flags the benchmark line is the 8-level airfoil in FP32 on one
    GPU, replayed from a graph, with the library's default tile height (the
    tuner only on request), the equal-Cf check, the three-element record and
    the CPU baseline; the sweep also times the persistent mode."""
    import bench
    a = bench.make_parser().parse_args([])
    assert (a.gpus, a.workload, a.storage, a.graph, a.tune, a.persistent) == (1, "airfoil", "f32", 1, 0, 1)
    assert a.equal_cf_steps > 0 and not a.no_three_element and not a.no_cpu_baseline
    assert bench.make_parser().parse_args(["--tune", "1"]).tune == 1
