"""bench.py command-line contract checks that need no GPU."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_help_lists_the_measurement_modes():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--help"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 0
    for flag in ("--serving", "--matvec", "--complexity", "--variants", "--steps", "--warmup"):
        assert flag in r.stdout
    for flag in ("--shots", "--no-batching"):
        assert flag in r.stdout


def test_traffic_record_applies_only_to_its_workload_and_kernel_source():
    """The calibrated byte counts were taken on one workload with one kernel
    source; every other workload (and any edited source) reports none."""
    import hashlib
    import importlib.util
    import json
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    bench = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(bench)
    for other in ("constant_k20_129", "wedge_f40", "layered_f20"):
        assert bench.measured_traffic("cgs_update_norm", other) is None
    rec = json.load(open(bench.TRAFFIC_RECORD))
    src = hashlib.sha256(open(bench.KERNEL_SOURCE, "rb").read()).hexdigest()
    got = bench.measured_traffic("cgs_update_norm", bench.TRAFFIC_WORKLOAD)
    if rec["kernels_hip_sha256"] == src:
        assert got == rec["classes"]["cgs_update_norm"]["bytes_per_launch"]
    else:
        assert got is None
