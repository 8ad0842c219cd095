"""Seeded synthetic sparse tf-idf corpora (inputs only; no clustering arithmetic).

The paper evaluates on one million tweets and 200k arXiv abstracts (Sec. 4.1),
which are not available here.  These corpora stand in for them: Zipf-distributed
terms, tf-idf weights and unit-length rows, as Sec. 4.1 describes the inputs.
The generator itself lives in ``synth.c``; this module wraps it with ctypes and
names the workloads.

Both the GPU library and the CPU oracle consume these arrays; neither shares
any other code with the other.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, asdict

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsynth.so")
_lib = None


def build(verbose: bool = False) -> str:
    """Compile synth.c into libsynth.so (gcc, OpenMP)."""
    import subprocess

    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
           os.path.join(_HERE, "synth.c"), "-o", LIB_PATH + ".tmp", "-lm"]
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
    i64, i32, u64, dbl = ctypes.c_int64, ctypes.c_int32, ctypes.c_uint64, ctypes.c_double
    vp = ctypes.c_void_p
    lib.synth_indptr.restype = i64
    lib.synth_indptr.argtypes = [i64, i32, dbl, dbl, i64, i64, u64, vp, i32]
    lib.synth_fill.restype = ctypes.c_int
    lib.synth_fill.argtypes = [i64, i32, dbl, dbl, u64, vp, vp, vp, i32]
    lib.synth_topic_fill.restype = ctypes.c_int
    lib.synth_topic_fill.argtypes = [i64, i32, i32, i32, dbl, dbl, dbl, u64, vp, vp, vp, i32]
    lib.synth_seed_rows.restype = ctypes.c_int
    lib.synth_seed_rows.argtypes = [i64, i32, u64, vp]
    lib.synth_stream_u64.restype = None
    lib.synth_stream_u64.argtypes = [u64, u64, u64, i64, vp]
    _lib = lib
    return lib


@dataclass(frozen=True)
class Corpus:
    """Parameters of one synthetic corpus (Sec. 4.1 stand-in)."""

    n_docs: int
    n_terms: int
    nnz_mean: float
    nnz_sigma: float
    nnz_min: int
    nnz_max: int
    zipf_s: float
    seed: int
    tf_p: float = 0.6

    def asdict(self):
        return asdict(self)


@dataclass(frozen=True)
class Workload:
    name: str
    corpus: Corpus
    k: int
    precision: str  # "fp32" | "bf16" | "fp8"
    ncc: bool
    index: bool
    max_iter: int
    min_moved_frac: float
    max_shift_sq: float = 1e-4
    stop_rule: str = "paper"


def generate(c: Corpus, nthreads: int = 0):
    """Return (indptr int64[N+1], indices int32[Z], values float32[Z])."""
    lib = _load()
    indptr = np.empty(c.n_docs + 1, dtype=np.int64)
    nnz = lib.synth_indptr(c.n_docs, c.n_terms, c.nnz_mean, c.nnz_sigma, c.nnz_min,
                           c.nnz_max, c.seed, indptr.ctypes.data, nthreads)
    if nnz < 0:
        raise ValueError(f"invalid corpus parameters {c}")
    indices = np.empty(nnz, dtype=np.int32)
    values = np.empty(nnz, dtype=np.float32)
    rc = lib.synth_fill(c.n_docs, c.n_terms, c.zipf_s, c.tf_p, c.seed, indptr.ctypes.data,
                        indices.ctypes.data, values.ctypes.data, nthreads)
    if rc != 0:
        raise RuntimeError(f"synth_fill failed ({rc})")
    return indptr, indices, values


@dataclass(frozen=True)
class TopicCorpus:
    """Topic-structured corpus: shared Zipf vocabulary plus one block per topic."""

    n_docs: int
    n_terms: int
    n_topics: int
    n_shared: int
    shared_frac: float
    nnz_mean: float
    nnz_sigma: float
    nnz_min: int
    nnz_max: int
    zipf_s: float
    seed: int
    tf_p: float = 0.6


def generate_topics(c: TopicCorpus, nthreads: int = 0):
    lib = _load()
    block = (c.n_terms - c.n_shared) // c.n_topics
    indptr = np.empty(c.n_docs + 1, dtype=np.int64)
    nmax = min(c.nnz_max, c.n_shared + block)
    nnz = lib.synth_indptr(c.n_docs, c.n_terms, c.nnz_mean, c.nnz_sigma, c.nnz_min, nmax, c.seed,
                           indptr.ctypes.data, nthreads)
    if nnz < 0:
        raise ValueError(f"invalid corpus parameters {c}")
    indices = np.empty(nnz, dtype=np.int32)
    values = np.empty(nnz, dtype=np.float32)
    rc = lib.synth_topic_fill(c.n_docs, c.n_terms, c.n_topics, c.n_shared, c.shared_frac, c.zipf_s,
                              c.tf_p, c.seed, indptr.ctypes.data, indices.ctypes.data,
                              values.ctypes.data, nthreads)
    if rc != 0:
        raise RuntimeError(f"synth_topic_fill failed ({rc})")
    return indptr, indices, values


def seed_rows(n_docs: int, k: int, seed: int) -> np.ndarray:
    """k distinct document ids drawn uniformly (the initial centroids' rows)."""
    lib = _load()
    out = np.empty(k, dtype=np.int32)
    if lib.synth_seed_rows(n_docs, k, seed, out.ctypes.data) != 0:
        raise ValueError("k must be in [0, n_docs]")
    return out


def stream_u64(seed: int, purpose: int, item: int, n: int) -> np.ndarray:
    lib = _load()
    out = np.empty(n, dtype=np.uint64)
    lib.synth_stream_u64(seed, purpose, item, n, out.ctypes.data)
    return out


def subset(indptr, indices, values, rows):
    """CSR of the given rows (in the given order)."""
    rows = np.asarray(rows, dtype=np.int64)
    lens = indptr[rows + 1] - indptr[rows]
    ip = np.zeros(len(rows) + 1, dtype=np.int64)
    np.cumsum(lens, out=ip[1:])
    idx = np.empty(ip[-1], dtype=np.int32)
    val = np.empty(ip[-1], dtype=np.float32)
    for o, r in enumerate(rows):
        b, e = indptr[r], indptr[r + 1]
        idx[ip[o]:ip[o + 1]] = indices[b:e]
        val[ip[o]:ip[o + 1]] = values[b:e]
    return ip, idx, val


# --- named workloads -------------------------------------------------------------
# Sizes follow the five configurations this implementation is measured on; the
# lognormal sigma of the k=10,000 corpus is not fixed anywhere and is taken as 0.7,
# and clipping of the k=20,000 corpus is assumed to be the same [10, 2000].

SMALL = Workload(
    name="plain-fp32 N=2000 D=5000 nnz~LN(50,0.5) zipf1.1 k=20 10it",
    corpus=Corpus(2000, 5000, 50.0, 0.5, 5, 300, 1.1, seed=1),
    k=20, precision="fp32", ncc=False, index=False, max_iter=10, min_moved_frac=0.0,
    stop_rule="fixed")

PLAIN_1M = Workload(
    name="plain-fp32 N=1e6 D=262144 nnz~LN(120,0.7) zipf1.1 k=1000",
    corpus=Corpus(1_000_000, 262_144, 120.0, 0.7, 10, 2000, 1.1, seed=2),
    k=1000, precision="fp32", ncc=False, index=False, max_iter=100, min_moved_frac=0.001)

PRUNED_BF16_2M = Workload(
    name="ncc+index bf16 N=2e6 D=262144 nnz~LN(150,0.7) zipf1.05 k=10000",
    corpus=Corpus(2_000_000, 262_144, 150.0, 0.7, 10, 2000, 1.05, seed=3),
    k=10_000, precision="bf16", ncc=True, index=True, max_iter=100, min_moved_frac=0.0)

FP8_8M = Workload(
    name="ncc+index fp8 N=8e6 D=262144 nnz~LN(200,0.8) zipf1.1 k=20000 30it",
    corpus=Corpus(8_000_000, 262_144, 200.0, 0.8, 10, 2000, 1.1, seed=4),
    k=20_000, precision="fp8", ncc=True, index=True, max_iter=30, min_moved_frac=0.0,
    stop_rule="fixed")

WORKLOADS = {w.name: w for w in (SMALL, PLAIN_1M, PRUNED_BF16_2M, FP8_8M)}

# Stand-ins shaped like the paper's two evaluation corpora (Sec. 4.1): one million
# tweets over 783,304 terms with 10 non-zeros on average, and 200,000 abstracts
# over 325,556 terms with 58.  Length spreads and clipping are not given: short
# texts vary little in length (sigma 0.5 / 0.35), every row keeps at least one
# term (rows of stop words only were dropped there).
TWEETS_1M = Corpus(1_000_000, 783_304, 10.0, 0.5, 1, 40, 1.1, seed=7)
ABSTRACTS_200K = Corpus(200_000, 325_556, 58.0, 0.35, 5, 300, 1.1, seed=8)
PAPER_CORPORA = {"tweets-1m": TWEETS_1M, "abstracts-200k": ABSTRACTS_200K}
PAPER_KS = (50, 500, 5000)


def scaled(c: Corpus, n_docs: int, n_terms: int | None = None, seed: int | None = None) -> Corpus:
    """The same generator at a smaller size (for tests)."""
    d = c.asdict()
    d["n_docs"] = n_docs
    if n_terms is not None:
        d["n_terms"] = n_terms
        d["nnz_max"] = min(d["nnz_max"], n_terms)
    if seed is not None:
        d["seed"] = seed
    return Corpus(**d)
