"""CPU FP64 oracle for sparse spherical k-means — TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product path (the HIP library and its
Python binding) never imports it, and it shares no code with that path; the only
module both sides use is ``synth`` (seeded input generation).

Contents:
  * ``oracle.c`` (built to ``liboracle.so``): plain FP64 assignment, update and
    seeding, the definition of the method's result (paper Sec. 2), and
    k-means++ seeding (the initialisation Sec. 2 names) with exact integer draws.
  * ``run``: the Lloyd loop with the paper's stopping rule (Sec. 2, Sec. 4.1).
  * ``index``: the dot-product index of Sec. 3.2 (G, P_lambda, query), pure Python.
  * ``quant``: BF16 and FP8-E4M3 rounding from the format definitions, exact.

Pins (``tests/test_oracle*.py``): brute force by dense numpy products, closed
forms (k = 1, planted disjoint blocks, k = N), the unit-norm invariant, the
monotone objective chain J_A(t) <= J_U(t) <= J_A(t+1), Lemma 3.1 and the
index's superset property, format values from the format definitions, and for
k-means++ an exact rational brute force plus closed forms (k = N gives every
row; groups of identical rows on disjoint terms get one seed each).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-ffp-contract=off",
           os.path.join(_HERE, "oracle.c"), "-o", LIB_PATH + ".tmp", "-lm"]
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
    lib.orc_seed.restype = ctypes.c_int
    lib.orc_seed.argtypes = [i64, i32, vp, vp, vp, i32, vp, vp]
    lib.orc_assign.restype = ctypes.c_int
    lib.orc_assign.argtypes = [i64, i32, vp, vp, vp, i32, vp, vp, i64, vp, vp, vp, i32]
    lib.orc_assign_seeds.restype = ctypes.c_int
    lib.orc_assign_seeds.argtypes = [i64, i32, vp, vp, vp, i32, vp, vp, i64, vp, vp, vp, i32]
    lib.orc_scores.restype = ctypes.c_int
    lib.orc_scores.argtypes = [i64, i32, vp, vp, vp, i32, vp, vp, i64, vp]
    lib.orc_update.restype = ctypes.c_int
    lib.orc_update.argtypes = [i64, i32, vp, vp, vp, i32, vp, vp, vp, vp, vp, vp, vp]
    lib.orc_kmeanspp.restype = ctypes.c_int
    lib.orc_kmeanspp.argtypes = [i64, i32, vp, vp, vp, i32, vp, vp]
    lib.orc_centroid_rows.restype = ctypes.c_int
    lib.orc_centroid_rows.argtypes = [i64, i32, vp, vp, vp, i32, vp, vp, i32, vp, vp]
    _lib = lib
    return lib


def _csr(csr):
    indptr, indices, values = csr
    indptr = np.ascontiguousarray(indptr, dtype=np.int64)
    indices = np.ascontiguousarray(indices, dtype=np.int32)
    values = np.ascontiguousarray(values, dtype=np.float32)
    return indptr, indices, values


def seed(csr, n_terms: int, rows) -> np.ndarray:
    """Initial centroids c_j = x_{rows[j]} / ||x_{rows[j]}|| (dense k x D)."""
    ip, ix, v = _csr(csr)
    rows = np.ascontiguousarray(rows, dtype=np.int32)
    C = np.empty((len(rows), n_terms), dtype=np.float64)
    rc = _load().orc_seed(len(ip) - 1, n_terms, ip.ctypes.data, ix.ctypes.data, v.ctypes.data,
                          len(rows), rows.ctypes.data, C.ctypes.data)
    if rc != 0:
        raise ValueError("seed row out of range")
    return C


def kmeanspp(csr, n_terms: int, k: int, draws) -> np.ndarray:
    """k-means++ seed rows from the caller's 64-bit draws (one per seed); the
    rules are in ``orc_kmeanspp`` (oracle.c)."""
    ip, ix, v = _csr(csr)
    draws = np.ascontiguousarray(draws, dtype=np.uint64)
    if len(draws) < k:
        raise ValueError("need one draw per seed")
    out = np.empty(k, dtype=np.int32)
    rc = _load().orc_kmeanspp(len(ip) - 1, n_terms, ip.ctypes.data, ix.ctypes.data, v.ctypes.data,
                              k, draws.ctypes.data, out.ctypes.data)
    if rc != 0:
        raise ValueError("k must be in [1, n_rows]" if rc == -1 else "out of memory")
    return out


def assign(csr, C: np.ndarray, docs=None, nthreads: int = 0):
    """(a, s1, s2): lowest-index argmax of the dot products, its value and the
    best value over the other centroids (Sec. 2)."""
    ip, ix, v = _csr(csr)
    C = np.ascontiguousarray(C, dtype=np.float64)
    k, D = C.shape
    if docs is None:
        n = len(ip) - 1
        dp = None
    else:
        docs = np.ascontiguousarray(docs, dtype=np.int64)
        n = len(docs)
        dp = docs.ctypes.data
    a = np.empty(n, dtype=np.int32)
    s1 = np.empty(n, dtype=np.float64)
    s2 = np.empty(n, dtype=np.float64)
    rc = _load().orc_assign(len(ip) - 1, D, ip.ctypes.data, ix.ctypes.data, v.ctypes.data, k,
                            C.ctypes.data, dp, n, a.ctypes.data, s1.ctypes.data, s2.ctypes.data,
                            nthreads)
    if rc != 0:
        raise ValueError("row index out of range")
    return a, s1, s2


def assign_seeds(csr, n_terms: int, rows, docs, nthreads: int = 0):
    """assign() against the initial centroids x_r/||x_r|| of the given seed rows,
    computed from the rows directly (no dense k x D array), for listed rows."""
    ip, ix, v = _csr(csr)
    rows = np.ascontiguousarray(rows, dtype=np.int32)
    docs = np.ascontiguousarray(docs, dtype=np.int64)
    n = len(docs)
    a = np.empty(n, dtype=np.int32)
    s1 = np.empty(n)
    s2 = np.empty(n)
    rc = _load().orc_assign_seeds(len(ip) - 1, n_terms, ip.ctypes.data, ix.ctypes.data,
                                  v.ctypes.data, len(rows), rows.ctypes.data, docs.ctypes.data, n,
                                  a.ctypes.data, s1.ctypes.data, s2.ctypes.data, nthreads)
    if rc != 0:
        raise ValueError("row index out of range")
    return a, s1, s2


def scores(csr, C: np.ndarray, docs=None) -> np.ndarray:
    """Dense FP64 similarity matrix for the listed rows (small inputs)."""
    ip, ix, v = _csr(csr)
    C = np.ascontiguousarray(C, dtype=np.float64)
    k, D = C.shape
    if docs is None:
        n, dp = len(ip) - 1, None
    else:
        docs = np.ascontiguousarray(docs, dtype=np.int64)
        n, dp = len(docs), docs.ctypes.data
    S = np.empty((n, k), dtype=np.float64)
    if _load().orc_scores(len(ip) - 1, D, ip.ctypes.data, ix.ctypes.data, v.ctypes.data, k,
                          C.ctypes.data, dp, n, S.ctypes.data) != 0:
        raise ValueError("row index out of range")
    return S


@dataclass
class UpdateResult:
    C: np.ndarray          # new centroids, k x D
    counts: np.ndarray     # members per cluster
    snorm: np.ndarray      # ||S_j|| (0 for empty clusters)
    shift_sq: np.ndarray   # ||c_j(new) - c_j(old)||^2
    dot_old: np.ndarray    # S_j . c_j(old)


def update(csr, a, C_old: np.ndarray) -> UpdateResult:
    """Centroid update (Sec. 2): normalised member sums; empty clusters keep
    their centroid."""
    ip, ix, v = _csr(csr)
    C_old = np.ascontiguousarray(C_old, dtype=np.float64)
    k, D = C_old.shape
    a = np.ascontiguousarray(a, dtype=np.int32)
    C = np.empty_like(C_old)
    counts = np.empty(k, dtype=np.int64)
    snorm = np.empty(k)
    shift = np.empty(k)
    dot_old = np.empty(k)
    rc = _load().orc_update(len(ip) - 1, D, ip.ctypes.data, ix.ctypes.data, v.ctypes.data, k,
                            a.ctypes.data, C_old.ctypes.data, C.ctypes.data, counts.ctypes.data,
                            snorm.ctypes.data, shift.ctypes.data, dot_old.ctypes.data)
    if rc != 0:
        raise ValueError("assignment out of range")
    return UpdateResult(C, counts, snorm, shift, dot_old)


def centroid_rows(csr, n_terms: int, k: int, a, clusters):
    """(rows, snorm): normalised member sums of the selected clusters only."""
    ip, ix, v = _csr(csr)
    a = np.ascontiguousarray(a, dtype=np.int32)
    clusters = np.ascontiguousarray(clusters, dtype=np.int32)
    out = np.empty((len(clusters), n_terms), dtype=np.float64)
    snorm = np.empty(len(clusters))
    rc = _load().orc_centroid_rows(len(ip) - 1, n_terms, ip.ctypes.data, ix.ctypes.data,
                                   v.ctypes.data, k, a.ctypes.data, clusters.ctypes.data,
                                   len(clusters), out.ctypes.data, snorm.ctypes.data)
    if rc != 0:
        raise ValueError("bad cluster id or assignment")
    return out, snorm


TIE_EPS = 1e-12


@dataclass
class IterRecord:
    t: int
    a: np.ndarray
    s1: np.ndarray
    s2: np.ndarray
    moved: int
    J_A: float
    ties: np.ndarray
    updated: bool = False
    J_U: float = float("nan")
    max_shift_sq: float = float("nan")
    changed: np.ndarray | None = None   # clusters whose membership changed


@dataclass
class RunResult:
    records: list = field(default_factory=list)
    C: np.ndarray | None = None          # centroids after the last executed step
    a: np.ndarray | None = None
    converged: bool = False
    stop_reason: str = "max_iter"


def run(csr, n_terms: int, k: int, init_rows, max_iter: int, min_moved_frac: float = 0.0,
        max_shift_sq: float = 1e-4, stop_rule: str = "paper", keep_centroids: bool = False):
    """Lloyd loop of spherical k-means (Sec. 2), one iteration = assign then update.

    stop_rule "paper": stop after an assignment that moved nothing (t >= 1) or
    fewer than min_moved_frac * N rows, or after an update whose largest squared
    centroid shift is below max_shift_sq (Sec. 4.1).  "fixed": run max_iter
    iterations.  When the loop stops after an assignment, no update follows and
    the returned centroids are the ones that assignment used.
    """
    ip, ix, v = _csr(csr)
    N = len(ip) - 1
    C = seed((ip, ix, v), n_terms, init_rows)
    res = RunResult()
    a_prev = None
    for t in range(max_iter):
        a, s1, s2 = assign((ip, ix, v), C)
        moved = N if a_prev is None else int(np.count_nonzero(a != a_prev))
        rec = IterRecord(t=t, a=a, s1=s1, s2=s2, moved=moved, J_A=float(np.sum(s1)),
                         ties=(s1 - s2) < TIE_EPS)
        res.records.append(rec)
        if stop_rule == "paper" and t >= 1 and (moved == 0 or moved < min_moved_frac * N):
            res.converged = True
            res.stop_reason = "moved"
            res.C, res.a = C, a
            return res
        u = update((ip, ix, v), a, C)
        rec.updated = True
        rec.J_U = float(np.sum(u.snorm))
        rec.max_shift_sq = float(np.max(u.shift_sq)) if k else 0.0
        if a_prev is None:
            rec.changed = np.arange(k)
        else:
            mv = a != a_prev
            rec.changed = np.union1d(a[mv], a_prev[mv])
        if keep_centroids:
            rec.C_before = C
        C = u.C
        a_prev = a
        if stop_rule == "paper" and rec.max_shift_sq < max_shift_sq:
            res.converged = True
            res.stop_reason = "shift"
            break
    res.C, res.a = C, a_prev
    return res
