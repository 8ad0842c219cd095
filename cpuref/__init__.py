"""The paper's own method on CPU cores (OpenMP, FP64): baseline, NCC (Sec. 3.1)
and NCC + INDEX (Sec. 3.2) spherical k-means over map-like sparse centroids,
written from the paper's description in ``cpuref.c``.

It gives the like-for-like CPU figure beside the GPU library for the paper's
ablation (Table 1's modes on stand-ins of its corpora); it shares no code with
the GPU library (``paper_2108_00895_amd``) or with the FP64 oracle
(``oracle``), and neither of them imports it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcpuref.so")
_lib = None

NCC, INDEX = 1, 2
MODES = {"baseline": 0, "ncc": NCC, "ncc+index": NCC | INDEX, "index": INDEX}


class Stats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("seconds_assign", ctypes.c_double), ("seconds_update", ctypes.c_double),
                ("seconds_index", ctypes.c_double), ("dots", ctypes.c_int64),
                ("index_rows", ctypes.c_int64)]


def build(verbose: bool = False) -> str:
    """Compile cpuref.c into libcpuref.so (gcc, OpenMP)."""
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-Wall",
           os.path.join(_HERE, "cpuref.c"), "-o", LIB_PATH + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB_PATH + ".tmp", LIB_PATH)
    global _lib
    _lib = None
    return LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() first")
    lib = ctypes.CDLL(LIB_PATH)
    i64, i32, vp = ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p
    lib.cr_run.restype = ctypes.c_int
    lib.cr_run.argtypes = [i64, i64, vp, vp, vp, i32, vp, ctypes.c_uint32, ctypes.c_int, vp, i32,
                           ctypes.c_double, ctypes.c_double, i32, vp, vp, ctypes.POINTER(Stats)]
    _lib = lib
    return lib


def run(csr, n_terms: int, k: int, seeds, mode: str = "ncc+index", max_iter: int = 100,
        max_shift_sq: float = 1e-4, lambdas=(0.1, 0.25, 0.4, 0.6), nthreads: int = 0,
        max_seconds: float = 0.0):
    """Clusters the rows from the seed rows under the paper's stopping rule
    (max_seconds > 0: stop after the first iteration past that time).
    Returns (final assignment, rows moved per iteration, stats dict)."""
    ip = np.ascontiguousarray(csr[0], dtype=np.int64)
    ix = np.ascontiguousarray(csr[1], dtype=np.int32)
    v = np.ascontiguousarray(csr[2], dtype=np.float32)
    seeds = np.ascontiguousarray(seeds, dtype=np.int32)
    lam = np.ascontiguousarray(lambdas, dtype=np.float64)
    N = len(ip) - 1
    a = np.empty(N, dtype=np.int32)
    moved = np.zeros(max_iter, dtype=np.int64)
    st = Stats()
    rc = _load().cr_run(N, n_terms, ip.ctypes.data, ix.ctypes.data, v.ctypes.data, k,
                        seeds.ctypes.data, MODES[mode], len(lam), lam.ctypes.data, max_iter,
                        max_shift_sq, max_seconds, nthreads, a.ctypes.data, moved.ctypes.data,
                        ctypes.byref(st))
    if rc != 0:
        raise MemoryError("cpuref: out of host memory")
    out = {f: getattr(st, f) for f, _ in Stats._fields_}
    return a, moved[:st.iterations].copy(), out
