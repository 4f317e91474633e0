"""CPU checks of the benchmark's command-line contract (no GPU work)."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench(*args, timeout=120):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          timeout=timeout, cwd=ROOT)


def test_more_than_one_gpu_is_refused_with_a_message():
    for mode in ([], ["--to-target"], ["--plbo"], ["--noisy", "0.5"], ["--peak"], ["--warmstart"]):
        r = _bench("--gpus", "2", *mode)
        assert r.returncode == 2, (mode, r.returncode, r.stderr)
        assert "one GPU" in r.stderr, (mode, r.stderr)


def test_defaults_are_one_gpu_and_a_short_run():
    sys.path.insert(0, ROOT)
    import bench
    old = sys.argv
    try:
        sys.argv = ["bench.py"]
        a = bench.parse()
    finally:
        sys.argv = old
    assert a.gpus == 1 and a.steps >= 1 and a.warmup >= 1
    assert a.workload == "gbs_n32_d16to8_chi128" and a.form == "fp32"


def test_host_record_has_the_cpu_model_and_blas():
    sys.path.insert(0, ROOT)
    import bench
    info = bench._host_info()
    assert info["nproc"] >= 1
    json.dumps(info)
