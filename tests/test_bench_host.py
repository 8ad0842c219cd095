"""Host-side logic of bench.py (CPU only): the multi-GPU refusal, and how the
committed counter record is matched to the kernel source and launch shape."""
import hashlib
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr and r.stdout == ""


def test_counter_record_matches_source_and_shape():
    rec = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))
    key = "k_score_part<bf16>@pruned-bf16-2m"
    assert key in rec
    r = rec[key]
    for field in ("src_sha", "fetch_bytes", "write_bytes", "ms_per_launch", "launches_per_step"):
        assert field in r
    src = os.path.join(ROOT, "paper_2108_00895_amd", "csrc", "kernels_score.hip")
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    got = bench.measured_traffic("k_score_part<bf16>", "pruned-bf16-2m")
    # the record is used only when it was taken on this kernel source
    assert (got is not None) == (r["src_sha"] == sha)
    if got is not None:
        assert bench.traffic_for(got, r["launches_per_step"]) is got
        assert bench.traffic_for(got, r["launches_per_step"] + 1) is None
    assert bench.measured_traffic("k_score_part<bf16>", "no-such-workload") is None
