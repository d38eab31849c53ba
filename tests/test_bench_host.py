"""Host-side logic of bench.py (no GPU): the one-GPU contract, the operation-count summary and
the rocprofv3 summary writers on small synthetic counter and trace files."""
import csv
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
import synth  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stdout + r.stderr


def test_operation_count_summary():
    w = synth.WORKLOADS["C3"]
    s = bench.flop_summary(w, [600] * 64, 0.8)
    assert s["setup_gflop"] > 0 and s["solve_gflop_per_rhs_mean"] > 0
    # the setup is shared by the batch: per-solve cost with it shared lies between the solve
    # alone and the solve plus a whole setup
    assert s["solve_gflop_per_rhs_mean"] < s["gflop_per_solve_setup_shared"] < s["gflop_per_solve_setup_per_rhs"]
    assert s["achieved_tflops"] == pytest.approx((s["setup_gflop"] + 64 * s["solve_gflop_per_rhs_mean"]) / 0.8 / 1e3)


def _write_csv(path, header, rows):
    with open(path, "w", newline="") as f:
        wr = csv.writer(f)
        wr.writerow(header)
        wr.writerows(rows)


def test_trace_summary(tmp_path):
    stats = tmp_path / "stats.csv"
    _write_csv(stats, ["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage"],
               [["void amamg::k_lag_update<20, 2>(double*)", 10, 3000000, 300000, 60.0],
                ["void amamg::k_gram<20, 2, true>(double*)", 10, 2000000, 200000, 40.0]])
    out = tmp_path / "summary.md"
    bench.trace_summary(str(stats), str(out), "CMD")
    text = out.read_text()
    assert "Total kernel time 5.0 ms over 20 dispatches" in text
    assert "| update (`k_lag_update<*`) | 10 | 300.00 | 3.00 |" in text


def test_traffic_summaries_scale_by_the_calibration_copy(tmp_path):
    # calibration: 1 GiB copy reads as 2^19 KiB of FETCH_SIZE (factor 0.5) and 2^20 KiB written
    cal = "void at::native::neg_kernel(...)"
    upd = "void amamg::k_lag_update<20, 2>(...)"
    fetch, write = tmp_path / "f.csv", tmp_path / "w.csv"
    hdr = ["Kernel_Name", "Counter_Name", "Counter_Value"]
    _write_csv(fetch, hdr, [[cal, "FETCH_SIZE", 2 ** 19], [upd, "FETCH_SIZE", 1000.0 * 0.5 * 1e6 / 1024]])
    _write_csv(write, hdr, [[cal, "WRITE_SIZE", 2 ** 20], [upd, "WRITE_SIZE", 200.0 * 1e6 / 1024]])
    out = tmp_path / "traffic.md"
    timer = json.dumps({"family": "update", "algorithmic_bytes_per_launch": 1200e6})
    bench.pmc_summary(str(fetch), str(write), str(out), "rocprofv3 --pmc COUNTER -- x", timer)
    text = out.read_text()
    assert "| update | 1 | 1000.0 | 200.0 | 1200.0 | 1.000 |" in text
    # both Gram-Schmidt families timed in one profiling pass: one marker each, and the roofline
    # finds the per-launch traffic of whichever family it reports
    dots = "void amamg::k_gram<20, 2, true>(...)"
    _write_csv(fetch, hdr, [[cal, "FETCH_SIZE", 2 ** 19], [upd, "FETCH_SIZE", 1000.0 * 0.5 * 1e6 / 1024],
                            [dots, "FETCH_SIZE", 1500.0 * 0.5 * 1e6 / 1024]])
    _write_csv(write, hdr, [[cal, "WRITE_SIZE", 2 ** 20], [upd, "WRITE_SIZE", 200.0 * 1e6 / 1024],
                            [dots, "WRITE_SIZE", 0.0]])
    timer = json.dumps({"profile_mixed": {}, "families": {
        "update": {"launches": 3, "avg_launch_us": 1.0, "algorithmic_bytes_per_launch": 1200e6},
        "dots": {"launches": 3, "avg_launch_us": 1.0, "algorithmic_bytes_per_launch": 1500e6}}})
    bench.pmc_summary(str(fetch), str(write), str(out), "rocprofv3 --pmc COUNTER -- x", timer)
    text = out.read_text()
    assert "| update | 1 | 1000.0 | 200.0 | 1200.0 | 1.000 |" in text
    assert "| dots | 1 | 1500.0 | 0.0 | 1500.0 | 1.000 |" in text
    saved = bench.TRAFFIC_MD
    try:
        bench.TRAFFIC_MD = str(out)
        assert bench.committed_traffic("update") == pytest.approx(1200e6)
        assert bench.committed_traffic("dots") == pytest.approx(1500e6)
        assert bench.committed_traffic("fine_gs") is None
    finally:
        bench.TRAFFIC_MD = saved
    # the stencil's summary on the same calibration, with a kernel trace for the duration
    st = "void amamg::k_wilson_apply<64, 1, double, HIP_vector_type<double, 2u>, HIP_vector_type<double, 2u> >(...)"
    alg = bench.STENCIL_BYTES_PER_SITE["fp64"] * bench.STENCIL_L ** 2
    _write_csv(fetch, hdr, [[cal, "FETCH_SIZE", 2 ** 19], [st, "FETCH_SIZE", alg * 0.5 / 1024]])
    _write_csv(write, hdr, [[cal, "WRITE_SIZE", 2 ** 20], [st, "WRITE_SIZE", 0.0]])
    stats = tmp_path / "stats.csv"
    _write_csv(stats, ["Name", "AverageNs"], [[st, 1e6]])
    bench.stencil_traffic_summary(str(fetch), str(write), str(stats), str(out), "CMD COUNTER", "TRACE")
    row = [ln for ln in out.read_text().splitlines() if "k_wilson_apply" in ln][0]
    assert "| fp64 | 1 |" in row and "| 1.000 |" in row and f"| {alg / 1e6:.0f} |" in row


def _leg_args(**kw):
    import argparse
    a = dict(groups=2, nrhs=64, workload="C3", serve_requests=0, serve_qps=None, tv_sweeps=None,
             aug_vectors=None)
    a.update(kw)
    return argparse.Namespace(**a)


def test_optional_leg_result_comes_back_from_its_child_process(tmp_path):
    """A leg run in a child process: its result line is picked out of the child's stdout, and
    the command carries the run's options."""
    script = tmp_path / "child.py"
    script.write_text("import json, sys\n"
                      "print('progress', file=sys.stderr)\n"
                      "print('not json')\n"
                      "print(json.dumps({'leg': sys.argv[2], 'result': {'argv': sys.argv[3:]}}))\n")
    out = bench.leg_child("agg", _leg_args(tv_sweeps=16), script=str(script))
    assert out["argv"][:2] == ["--groups", "2"] and "--tv-sweeps" in out["argv"]


def test_a_crashing_leg_costs_only_its_own_record(tmp_path):
    """A child that aborts (or prints no result) gives an error record instead of ending the
    benchmark."""
    script = tmp_path / "child.py"
    script.write_text("import os\nprint('partial output')\nos.abort()\n")
    out = bench.leg_child("multi", _leg_args(), script=str(script))
    assert "error" in out and "status" in out["error"]
    script.write_text("import sys\nsys.exit(0)\n")
    assert "error" in bench.leg_child("serving", _leg_args(), script=str(script))
