"""Host-side logic of bench.py (CPU only): the multi-GPU refusal, how a counter
record is built from rocprofv3 output, and how it is matched to the kernel
sources, the launch shape and the timed window."""
import csv
import json
import os
import subprocess
import sys
import types

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402

KERN = "void skm::(anonymous namespace)::k_score_part<1>(skm::ScoreArgs, skm::Partial*, long)"
MARK = "at::cuda::(anonymous namespace)::spin_kernel(long)"
COPY = "__amd_rocclr_copyBuffer"


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr and r.stdout == ""


def _write(path, fields, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=fields)
        w.writeheader()
        w.writerows(rows)


# dispatch sequence: a warm-up launch, marker, calibration copy, marker, three
# timed launches, marker, a launch after the window
SEQ = [(1, KERN), (2, MARK), (3, COPY), (4, MARK), (5, KERN), (6, KERN), (7, KERN), (8, MARK),
       (9, KERN)]


def _profile(tmp, fetch_kib, write_kib, cal_fetch, cal_write):
    _write(os.path.join(tmp, "trace", "host", "run_kernel_trace.csv"),
           ["Dispatch_Id", "Kernel_Name", "Start_Timestamp", "End_Timestamp"],
           [{"Dispatch_Id": d, "Kernel_Name": n, "Start_Timestamp": 1000 * d,
             "End_Timestamp": 1000 * d + (2_000_000 if n == KERN else 10)} for d, n in SEQ])
    for which, per, cal, counter in (("fetch", fetch_kib, cal_fetch, "FETCH_SIZE"),
                                     ("write", write_kib, cal_write, "WRITE_SIZE")):
        rows = []
        for d, n in SEQ:
            v = per if n == KERN else (cal if n == COPY else 0.0)
            rows.append({"Dispatch_Id": d, "Kernel_Name": n, "Counter_Name": counter,
                         "Counter_Value": v})
            rows.append({"Dispatch_Id": d, "Kernel_Name": n, "Counter_Name": "OTHER",
                         "Counter_Value": 1e9})
        _write(os.path.join(tmp, which, "host", "run_counter_collection.csv"),
               ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"], rows)


def test_profile_summary_scales_and_windows(tmp_path):
    tmp = str(tmp_path)
    # the copy moves 4 GiB each way; FETCH_SIZE reads half of it (factor 2)
    _profile(tmp, fetch_kib=1000.0, write_kib=10.0, cal_fetch=2 * 1024 * 1024,
             cal_write=4 * 1024 * 1024)
    shape = {"head_chunks": 4, "head_rows": 1 << 20, "workgroups_per_cu": 6}
    line = {"steps": 3, "warmup": 2, "roofline": {"kernel": "k_score_part<bf16>"},
            "config": {"workload": "wl"}, "autotune": {"best": dict(shape, ms=1.0)}}
    meta = os.path.join(tmp, "bench.json")
    open(meta, "w").write("noise\n" + json.dumps(line) + "\n")
    out = os.path.join(tmp, "traffic.json")
    args = types.SimpleNamespace(profile_summary=[os.path.join(tmp, x) for x in
                                                  ("trace", "fetch", "write")],
                                 profile_meta=meta, profile_out=out)
    bench.profile_summary(args)
    rec = json.load(open(out))["k_score_part<bf16>@wl"]
    assert rec["trace_launches"] == 3 and rec["launches_per_step"] == 1.0
    assert abs(rec["trace_ms_per_launch"] - 2.0) < 1e-12
    assert abs(rec["fetch_calibration"] - 2.0) < 1e-12
    assert abs(rec["fetch_bytes"] - 2 * 1000.0 * 1024) < 1e-6
    assert abs(rec["write_bytes"] - 10.0 * 1024) < 1e-6
    # matched only at the same sources, shape, window and launches per step
    got = bench.measured_traffic("k_score_part<bf16>", "wl", shape, 1.0, 3, 2, path=out)
    assert got is not None and got["src_sha"] == bench.kernel_sha()
    assert bench.measured_traffic("k_score_part<bf16>", "wl", shape, 2.0, 3, 2, path=out) is None
    assert bench.measured_traffic("k_score_part<bf16>", "wl", shape, 1.0, 4, 2, path=out) is None
    other = dict(shape, workgroups_per_cu=5)
    assert bench.measured_traffic("k_score_part<bf16>", "wl", other, 1.0, 3, 2, path=out) is None
    assert bench.measured_traffic("k_score_part<bf16>", "x", shape, 1.0, 3, 2, path=out) is None
    # the shape the record was taken at, for the bench to prefer among equal trials
    assert bench.profiled_shape("k_score_part<bf16>", "wl", path=out) == shape
    assert bench.profiled_shape("k_score_part<bf16>", "x", path=out) is None
    rec2 = json.load(open(out))
    rec2["k_score_part<bf16>@wl"]["src_sha"] = "0" * 16
    json.dump(rec2, open(out, "w"))
    assert bench.measured_traffic("k_score_part<bf16>", "wl", shape, 1.0, 3, 2, path=out) is None
    assert bench.profiled_shape("k_score_part<bf16>", "wl", path=out) is None


def test_committed_record_is_well_formed():
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return
    for key, r in json.load(open(path)).items():
        if "shape" not in r:
            continue
        for field in ("src_sha", "fetch_bytes", "write_bytes", "trace_ms_per_launch",
                      "launches_per_step", "steps", "warmup", "window"):
            assert field in r, (key, field)
