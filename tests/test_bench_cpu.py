"""Host-side behaviour of bench.py that needs no GPU."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout == ""


def test_counter_figures_follow_the_kernel_source():
    """The list kernel's counter-derived traffic and issue fractions are
    reported only for the source they were taken with."""
    sys.path.insert(0, ROOT)
    import bench
    flops, secs = 7.2503e13, 264.9e-3
    if bench.sources_hash(bench.TF_SOURCES) == bench.TF_COUNTERS["sources_sha256_16"]:
        c = bench.tf_counters(flops, secs)
        assert 0.3 < c["valu_issue_frac"] < 0.6 and 0.1 < c["mfma_busy_frac"] < 0.2
        assert 5e8 < bench.tf_traffic_bytes() < 6e8
    saved = dict(bench.TF_COUNTERS)
    try:
        bench.TF_COUNTERS["sources_sha256_16"] = "0" * 16
        assert bench.tf_counters(flops, secs) is None
        assert bench.tf_traffic_bytes() is None
    finally:
        bench.TF_COUNTERS.clear()
        bench.TF_COUNTERS.update(saved)
