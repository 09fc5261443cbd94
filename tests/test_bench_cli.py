"""bench.py's command line on the CPU: one GPU only (a request for more
exits with a message before any GPU work), and its traffic record check
reads the committed counter summaries."""
import importlib.util
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=120)
    assert res.returncode != 0
    assert "one GPU" in res.stderr and res.stdout == ""


def test_traffic_records_match_the_kernel_sources():
    spec = importlib.util.spec_from_file_location("bench", os.path.join(ROOT, "bench.py"))
    bench = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(bench)
    for tb, (name, path, _) in bench.INTERIOR.items():
        rec = json.load(open(path))
        assert rec["kernel"].startswith(name)
        # the record is used only while the sources are the ones it was taken on
        assert (bench.measured_traffic(tb) is not None) == (
            rec["kernel_source_sha256"] == bench.kernel_source_hash(bench.INTERIOR[tb][2]))
        assert rec["hbm_bytes_per_launch"] > 0.9 * rec["algorithmic_bytes_per_launch"]


def test_batch_shape_is_checked_before_any_gpu_work():
    for bad in ("4,512,16", "4,512,16,2,8,-1,0,x"):
        res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--section",
                              "batch-kernels", "--batch-shape", bad],
                             capture_output=True, text=True, timeout=120)
        assert res.returncode == 2
        assert "--batch-shape takes 8" in res.stderr and res.stdout == ""
