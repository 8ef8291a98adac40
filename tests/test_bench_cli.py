"""The benchmark script's command line, without a GPU: it parses, lists its
modes, and refuses more than one GPU with a message."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_defines_every_mode():
    sys.path.insert(0, ROOT)
    import bench
    for name in ("main", "run_workload", "cpu_baseline", "oracle_step_seconds", "reuse_study", "loop_run",
                 "sort_ablation", "pmc_summary", "valu_summary", "trace_summary", "counter_summary"):
        assert callable(getattr(bench, name)), name


def test_help_and_gpu_count():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--help"], capture_output=True, text=True)
    assert r.returncode == 0 and "--sort-ablation" in r.stdout and "--loop" in r.stdout
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True)
    assert r.returncode == 2 and "one GPU" in r.stderr
