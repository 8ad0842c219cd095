"""ctypes binding of libskm (include/skm.h): argument marshalling only.

Every step of the clustering runs in the HIP kernels behind the C ABI; this
module converts Python arguments (numpy arrays for host data, torch CUDA
tensors for device data) into the C structs and back.  It has no fallback: if
libskm.so is missing or cannot be loaded, every entry point raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libskm.so")

(SKM_OK, SKM_E_INVALID, SKM_E_NOMEM, SKM_E_DEVICE, SKM_E_STATE, SKM_E_UNSUPPORTED, SKM_E_BUSY,
 SKM_E_TIMEOUT, SKM_E_CANCELLED) = range(9)
FP32, BF16, FP8_E4M3 = 0, 1, 2
NCC, INDEX, NO_EXACT, DENSE_ONLY, BORROW_DEVICE = 1, 2, 4, 8, 16
STOP_PAPER, STOP_FIXED = 0, 1
PRECISIONS = {"fp32": FP32, "bf16": BF16, "fp8": FP8_E4M3}
CODE_BYTES = {FP32: 4, BF16: 2, FP8_E4M3: 1}

EXPORTED = [
    "skm_config_default", "skm_kmeanspp", "skm_init", "skm_assign", "skm_update", "skm_iterate",
    "skm_assign_new", "skm_get_assignments", "skm_get_centroids", "skm_get_centroid_columns",
    "skm_get_centroid_rows", "skm_set_centroids",
    "skm_save", "skm_load", "skm_get_tile", "skm_get_changed", "skm_score_dense", "skm_error_bound", "skm_head_terms",
    "skm_score_head", "skm_error_bound_head", "skm_error_bound_split", "skm_autotune", "skm_set_schedule", "skm_get_index",
    "skm_index_query", "skm_server_config_default", "skm_server_start", "skm_server_submit",
    "skm_server_wait", "skm_server_get_stats", "skm_server_stop", "skm_server_submit_job",
    "skm_server_cancel", "skm_context_bytes", "skm_tune_lambda", "skm_debug_fail_after",
    "skm_hbm_bytes", "skm_last_error", "skm_destroy", "skm_index_threshold",
    "skm_assign_new_static", "skm_static_scratch_bytes", "skm_static_max_rows",
    "skm_assign_new_index_rows",
]


class SkmError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"skm status {status}: {msg}")
        self.status = status


class Csr(ctypes.Structure):
    _fields_ = [("n_rows", ctypes.c_int64), ("n_cols", ctypes.c_int64), ("nnz", ctypes.c_int64),
                ("indptr", ctypes.c_void_p), ("indices", ctypes.c_void_p),
                ("values", ctypes.c_void_p), ("on_device", ctypes.c_int32)]


class Config(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int32), ("precision", ctypes.c_int32), ("flags", ctypes.c_uint32),
                ("n_lambda", ctypes.c_int32), ("lambda_", ctypes.c_double * 8),
                ("index_min_changed", ctypes.c_int32), ("stop_rule", ctypes.c_int32),
                ("max_iter", ctypes.c_int32), ("min_moved_frac", ctypes.c_double),
                ("max_shift_sq", ctypes.c_double), ("init_rows", ctypes.c_void_p),
                ("init_centroids", ctypes.c_void_p), ("hbm_budget_bytes", ctypes.c_size_t),
                ("stream", ctypes.c_void_p), ("validate", ctypes.c_int32),
                ("head_max_terms", ctypes.c_int32), ("head_min_df", ctypes.c_double),
                ("ncc_adaptive", ctypes.c_int32), ("index_always", ctypes.c_int32)]


class IterStats(ctypes.Structure):
    _fields_ = [("iter", ctypes.c_int32), ("changed_centroids", ctypes.c_int32),
                ("moved", ctypes.c_int64), ("flagged", ctypes.c_int64),
                ("band_overflow", ctypes.c_int64), ("ncc_rows", ctypes.c_int64),
                ("index_rows", ctypes.c_int64), ("index_no_level", ctypes.c_int64),
                ("index_guarded", ctypes.c_int64), ("index_over_cap", ctypes.c_int64),
                ("mean_candidates", ctypes.c_double),
                ("scored_products", ctypes.c_double),
                ("objective_assign", ctypes.c_double), ("objective_update", ctypes.c_double),
                ("max_shift_sq", ctypes.c_double), ("ms_assign", ctypes.c_float),
                ("ms_score", ctypes.c_float), ("ms_exact", ctypes.c_float), ("ms_update", ctypes.c_float),
                ("ms_index", ctypes.c_float), ("head_terms", ctypes.c_int32),
                ("ms_head", ctypes.c_float), ("score_launches", ctypes.c_int32),
                ("sparse_products", ctypes.c_double), ("ms_sparse", ctypes.c_float),
                ("head_launches", ctypes.c_int32), ("head_pairs", ctypes.c_double),
                ("ms_index_build", ctypes.c_float), ("index_build", ctypes.c_int32)]

    def asdict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class TuneTrial(ctypes.Structure):
    _fields_ = [("head_chunks", ctypes.c_int32), ("workgroups_per_cu", ctypes.c_int32),
                ("head_rows", ctypes.c_int64), ("ms", ctypes.c_double)]


class TuneReport(ctypes.Structure):
    _fields_ = [("n_trials", ctypes.c_int32), ("best", ctypes.c_int32),
                ("trials", TuneTrial * 16)]


class LambdaReport(ctypes.Structure):
    _fields_ = [("n_sample", ctypes.c_int32), ("n_grid", ctypes.c_int32),
                ("grid", ctypes.c_double * 20), ("qualify", ctypes.c_double * 20),
                ("mean_candidates", ctypes.c_double * 20), ("n_before", ctypes.c_int32),
                ("n_after", ctypes.c_int32), ("before", ctypes.c_double * 8),
                ("after", ctypes.c_double * 8), ("cost_before", ctypes.c_double),
                ("cost_after", ctypes.c_double), ("applied", ctypes.c_int32)]


class ServerConfig(ctypes.Structure):
    _fields_ = [("n_slots", ctypes.c_int32), ("slot_rows", ctypes.c_int32),
                ("slot_nnz", ctypes.c_int64), ("hbm_budget_bytes", ctypes.c_size_t),
                ("max_wait_us", ctypes.c_int32), ("use_graphs", ctypes.c_int32),
                ("max_jobs", ctypes.c_int32)]


class ServerStats(ctypes.Structure):
    _fields_ = [("requests_done", ctypes.c_int64), ("rows_done", ctypes.c_int64),
                ("batches", ctypes.c_int64), ("p50_ms", ctypes.c_double),
                ("p99_ms", ctypes.c_double), ("mean_ms", ctypes.c_double),
                ("max_ms", ctypes.c_double), ("rows_per_s", ctypes.c_double),
                ("slots", ctypes.c_int32), ("max_queue_depth", ctypes.c_int32),
                ("hbm_bytes", ctypes.c_size_t), ("jobs_done", ctypes.c_int64),
                ("job_iterations", ctypes.c_int64), ("jobs_running", ctypes.c_int32),
                ("jobs_queued", ctypes.c_int32)]

    def asdict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class JobInfo(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("objective", ctypes.c_double), ("hbm_bytes", ctypes.c_size_t)]

    def asdict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


_lib = None


def load():
    """Load libskm.so (raises if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
    # One HIP runtime per process: when PyTorch is present its libamdhip64 is
    # loaded first, and libskm's dependency on the same soname binds to it.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, st = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_int
    P = ctypes.POINTER
    lib.skm_config_default.argtypes = [P(Config)]
    lib.skm_config_default.restype = None
    lib.skm_init.argtypes = [P(Csr), P(Config), P(vp)]
    lib.skm_init.restype = st
    lib.skm_assign.argtypes = [vp, P(IterStats)]
    lib.skm_assign.restype = st
    lib.skm_update.argtypes = [vp, P(IterStats)]
    lib.skm_update.restype = st
    lib.skm_iterate.argtypes = [vp, i32, vp, P(i32), P(i32)]
    lib.skm_iterate.restype = st
    lib.skm_assign_new.argtypes = [vp, P(Csr), vp, vp, vp]
    lib.skm_assign_new.restype = st
    lib.skm_assign_new_static.argtypes = [vp, P(Csr), vp, vp, vp]
    lib.skm_assign_new_static.restype = st
    lib.skm_static_scratch_bytes.argtypes = []
    lib.skm_static_scratch_bytes.restype = ctypes.c_size_t
    lib.skm_static_max_rows.argtypes = [vp]
    lib.skm_static_max_rows.restype = i64
    lib.skm_get_assignments.argtypes = [vp, vp, i32]
    lib.skm_get_assignments.restype = st
    lib.skm_get_centroids.argtypes = [vp, vp, i32]
    lib.skm_get_centroids.restype = st
    lib.skm_set_centroids.argtypes = [vp, vp]
    lib.skm_set_centroids.restype = st
    lib.skm_get_tile.argtypes = [vp, vp, ctypes.c_size_t, vp, P(i64)]
    lib.skm_get_tile.restype = st
    lib.skm_get_changed.argtypes = [vp, vp]
    lib.skm_get_changed.restype = st
    lib.skm_save.argtypes = [vp, ctypes.c_char_p]
    lib.skm_save.restype = st
    lib.skm_load.argtypes = [P(vp), P(Csr), ctypes.c_char_p, P(Config)]
    lib.skm_load.restype = st
    lib.skm_kmeanspp.argtypes = [P(Csr), i32, vp, vp, vp]
    lib.skm_kmeanspp.restype = st
    lib.skm_score_dense.argtypes = [vp, P(Csr), vp]
    lib.skm_score_dense.restype = st
    lib.skm_error_bound.argtypes = [vp, ctypes.c_double, i64, ctypes.c_double]
    lib.skm_error_bound.restype = ctypes.c_double
    lib.skm_get_centroid_rows.argtypes = [vp, vp, i32, vp]
    lib.skm_get_centroid_rows.restype = st
    lib.skm_get_centroid_columns.argtypes = [vp, vp, i32, vp]
    lib.skm_get_centroid_columns.restype = st
    lib.skm_autotune.argtypes = [vp, P(TuneReport)]
    lib.skm_autotune.restype = st
    lib.skm_set_schedule.argtypes = [vp, P(TuneTrial)]
    lib.skm_set_schedule.restype = st
    lib.skm_head_terms.argtypes = [vp]
    lib.skm_head_terms.restype = ctypes.c_int32
    lib.skm_score_head.argtypes = [vp, i64, i64, vp, vp]
    lib.skm_score_head.restype = st
    lib.skm_error_bound_head.argtypes = [vp, ctypes.c_double, i64, ctypes.c_double]
    lib.skm_error_bound_head.restype = ctypes.c_double
    lib.skm_error_bound_split.argtypes = [vp, ctypes.c_double, ctypes.c_double, i64, ctypes.c_double]
    lib.skm_error_bound_split.restype = ctypes.c_double
    lib.skm_assign_new_index_rows.argtypes = [vp]
    lib.skm_assign_new_index_rows.restype = i64
    lib.skm_get_index.argtypes = [vp, i32, vp, vp, P(i64)]
    lib.skm_get_index.restype = st
    lib.skm_index_query.argtypes = [vp, P(Csr), i32, vp, vp, i64]
    lib.skm_index_query.restype = st
    lib.skm_server_config_default.argtypes = [P(ServerConfig)]
    lib.skm_server_config_default.restype = None
    lib.skm_server_start.argtypes = [vp, P(ServerConfig), P(vp)]
    lib.skm_server_start.restype = st
    lib.skm_server_submit.argtypes = [vp, P(Csr), vp, vp, P(i64)]
    lib.skm_server_submit.restype = st
    lib.skm_server_wait.argtypes = [vp, i64, ctypes.c_double]
    lib.skm_server_wait.restype = st
    lib.skm_server_get_stats.argtypes = [vp, P(ServerStats)]
    lib.skm_server_get_stats.restype = st
    lib.skm_server_stop.argtypes = [vp]
    lib.skm_server_stop.restype = st
    lib.skm_server_submit_job.argtypes = [vp, P(Csr), P(Config), vp, vp, P(JobInfo), P(i64)]
    lib.skm_server_submit_job.restype = st
    lib.skm_server_cancel.argtypes = [vp, i64]
    lib.skm_server_cancel.restype = st
    lib.skm_debug_fail_after.argtypes = [vp, i32]
    lib.skm_debug_fail_after.restype = st
    lib.skm_tune_lambda.argtypes = [vp, i32, P(LambdaReport)]
    lib.skm_tune_lambda.restype = st
    lib.skm_context_bytes.argtypes = [P(Csr), P(Config)]
    lib.skm_context_bytes.restype = ctypes.c_size_t
    lib.skm_index_threshold.argtypes = [ctypes.c_double, i64, ctypes.c_double]
    lib.skm_index_threshold.restype = ctypes.c_double
    lib.skm_hbm_bytes.argtypes = [vp]
    lib.skm_hbm_bytes.restype = ctypes.c_size_t
    lib.skm_last_error.argtypes = []
    lib.skm_last_error.restype = ctypes.c_char_p
    lib.skm_destroy.argtypes = [vp]
    lib.skm_destroy.restype = None
    _lib = lib
    return lib


def _check(status):
    if status != SKM_OK:
        raise SkmError(status, load().skm_last_error().decode(errors="replace"))


def _is_torch(x):
    return type(x).__module__.startswith("torch")


def make_csr(indptr, indices, values, n_cols):
    """Csr struct + keep-alive tuple.  numpy arrays -> host; torch CUDA tensors -> device."""
    if _is_torch(indptr):
        import torch

        assert indptr.dtype == torch.int64 and indices.dtype == torch.int32
        assert values.dtype == torch.float32
        assert indptr.is_cuda and indices.is_cuda and values.is_cuda
        indptr, indices, values = indptr.contiguous(), indices.contiguous(), values.contiguous()
        c = Csr(indptr.numel() - 1, n_cols, indices.numel(), indptr.data_ptr(),
                indices.data_ptr(), values.data_ptr(), 1)
        return c, (indptr, indices, values)
    indptr = np.ascontiguousarray(indptr, dtype=np.int64)
    indices = np.ascontiguousarray(indices, dtype=np.int32)
    values = np.ascontiguousarray(values, dtype=np.float32)
    c = Csr(len(indptr) - 1, n_cols, len(indices), indptr.ctypes.data, indices.ctypes.data,
            values.ctypes.data, 0)
    return c, (indptr, indices, values)


def kmeanspp(csr, n_cols, k, draws, stream=None):
    """k-means++ seed rows (skm_kmeanspp) from k caller-supplied 64-bit draws."""
    c, hold = make_csr(*csr, n_cols)
    d = np.ascontiguousarray(draws, dtype=np.uint64)
    if len(d) < k:
        raise ValueError("need one draw per seed")
    out = np.empty(k, dtype=np.int32)
    _check(load().skm_kmeanspp(ctypes.byref(c), k, d.ctypes.data, out.ctypes.data, stream))
    return out


@dataclass
class Options:
    precision: str = "fp32"
    ncc: bool = False
    index: bool = False
    no_exact: bool = False
    dense_only: bool = False
    lambdas: tuple = (0.1, 0.25, 0.4, 0.6)
    index_min_changed: int = 0
    stop_rule: str = "paper"
    max_iter: int = 100
    min_moved_frac: float = 0.0
    max_shift_sq: float = 1e-4
    hbm_budget_bytes: int = 0
    validate: bool = True
    head_max_terms: int | None = None   # None: the library default (4096); 0: off
    head_min_df: float | None = None    # None: the library default (1/128)
    borrow: bool = False                # device rows used in place (SKM_BORROW_DEVICE)
    ncc_adaptive: bool = False          # NCC only when its measured saving beats its preparation
    index_always: bool = False          # no back-off of the index when it decides few rows


def _config(lib, k, o, init_rows, init_centroids, stream):
    """skm_config from Options (+ the arrays it points to, to keep alive)."""
    cfg = Config()
    lib.skm_config_default(ctypes.byref(cfg))
    cfg.k = k
    cfg.precision = PRECISIONS[o.precision]
    cfg.flags = ((NCC if o.ncc else 0) | (INDEX if o.index else 0) |
                 (NO_EXACT if o.no_exact else 0) | (DENSE_ONLY if o.dense_only else 0) |
                 (BORROW_DEVICE if o.borrow else 0))
    cfg.n_lambda = len(o.lambdas)
    for i, lam in enumerate(o.lambdas):
        cfg.lambda_[i] = lam
    cfg.index_min_changed = o.index_min_changed
    cfg.stop_rule = STOP_PAPER if o.stop_rule == "paper" else STOP_FIXED
    cfg.max_iter = o.max_iter
    cfg.min_moved_frac = o.min_moved_frac
    cfg.max_shift_sq = o.max_shift_sq
    cfg.hbm_budget_bytes = o.hbm_budget_bytes
    cfg.validate = 1 if o.validate else 0
    cfg.ncc_adaptive = 1 if o.ncc_adaptive else 0
    cfg.index_always = 1 if o.index_always else 0
    if o.head_max_terms is not None:
        cfg.head_max_terms = o.head_max_terms
    if o.head_min_df is not None:
        cfg.head_min_df = o.head_min_df
    keep = []
    if init_rows is not None:
        r = np.ascontiguousarray(init_rows, dtype=np.int32)
        keep.append(r)
        cfg.init_rows = r.ctypes.data
    if init_centroids is not None:
        C = np.ascontiguousarray(init_centroids, dtype=np.float64)
        keep.append(C)
        cfg.init_centroids = C.ctypes.data
    if stream is not None:
        cfg.stream = stream
    return cfg, keep


class Context:
    """One clustering problem resident on the GPU (wraps skm_ctx)."""

    def __init__(self, csr, n_cols, k, init_rows=None, init_centroids=None, stream=None,
                 **opts):
        lib = load()
        o = Options(**opts)
        cfg, keep = _config(lib, k, o, init_rows, init_centroids, stream)
        c, hold = make_csr(*csr, n_cols)
        h = ctypes.c_void_p()
        _check(lib.skm_init(ctypes.byref(c), ctypes.byref(cfg), ctypes.byref(h)))
        self._h = h
        self._hold = hold if o.borrow else None   # borrowed rows live as long as the context
        self.k, self.n_cols, self.n_rows = k, n_cols, c.n_rows
        self.precision = cfg.precision
        self.opts = o

    @classmethod
    def from_checkpoint(cls, path, csr, n_cols, k, stream=None, **opts):
        """A context resumed from skm_save's file (skm_load): the same rows,
        k and options (precision, ncc, index, no_exact, dense_only) as the run
        that saved it."""
        lib = load()
        o = Options(**opts)
        cfg, _ = _config(lib, k, o, None, None, stream)
        c, hold = make_csr(*csr, n_cols)
        h = ctypes.c_void_p()
        _check(lib.skm_load(ctypes.byref(h), ctypes.byref(c), os.fsencode(path), ctypes.byref(cfg)))
        self = cls.__new__(cls)
        self._h = h
        self._hold = hold if o.borrow else None
        self.k, self.n_cols, self.n_rows = k, n_cols, c.n_rows
        self.precision = cfg.precision
        self.opts = o
        return self

    def save(self, path):
        """Checkpoint after an update (skm_save)."""
        _check(load().skm_save(self._h, os.fsencode(path)))


    # -- lifecycle
    def close(self):
        if getattr(self, "_h", None):
            load().skm_destroy(self._h)
            self._h = None
        self._hold = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # -- steps
    def assign(self):
        st = IterStats()
        _check(load().skm_assign(self._h, ctypes.byref(st)))
        return st.asdict()

    def update(self):
        st = IterStats()
        _check(load().skm_update(self._h, ctypes.byref(st)))
        return st.asdict()

    def iterate(self, max_iter=0):
        n = max_iter if max_iter > 0 else self.opts.max_iter
        arr = (IterStats * n)()
        done, conv = ctypes.c_int32(), ctypes.c_int32()
        _check(load().skm_iterate(self._h, max_iter, arr, ctypes.byref(done), ctypes.byref(conv)))
        return [arr[i].asdict() for i in range(done.value)], bool(conv.value)

    def assign_new(self, csr, stream=None):
        c, hold = make_csr(*csr, self.n_cols)
        n = c.n_rows
        if c.on_device:
            import torch

            dev = hold[0].device
            a = torch.empty(n, dtype=torch.int32, device=dev)
            s = torch.empty(n, dtype=torch.float64, device=dev)
            _check(load().skm_assign_new(self._h, ctypes.byref(c), a.data_ptr(), s.data_ptr(),
                                         stream))
            return a, s
        a = np.empty(n, dtype=np.int32)
        s = np.empty(n, dtype=np.float64)
        _check(load().skm_assign_new(self._h, ctypes.byref(c), a.ctypes.data, s.ctypes.data,
                                     stream))
        return a, s

    def assign_new_index_rows(self):
        """Rows of the last assign_new that the index assigned."""
        return int(load().skm_assign_new_index_rows(self._h))

    def assign_new_static(self, csr, out_assign, out_score, stream=None):
        """skm_assign_new_static: device rows (torch tensors) in, answers written
        into the caller's device tensors out_assign (int32) and out_score
        (float64); no device memory is allocated by the call."""
        c, hold = make_csr(*csr, self.n_cols)
        _check(load().skm_assign_new_static(self._h, ctypes.byref(c), out_assign.data_ptr(),
                                            out_score.data_ptr(), stream))

    def static_max_rows(self):
        return int(load().skm_static_max_rows(self._h))

    # -- getters
    def assignments(self):
        out = np.empty(self.n_rows, dtype=np.int32)
        _check(load().skm_get_assignments(self._h, out.ctypes.data, 0))
        return out

    def centroids(self):
        out = np.empty((self.k, self.n_cols), dtype=np.float64)
        _check(load().skm_get_centroids(self._h, out.ctypes.data, 0))
        return out

    def set_centroids(self, C):
        C = np.ascontiguousarray(C, dtype=np.float64)
        assert C.shape == (self.k, self.n_cols)
        _check(load().skm_set_centroids(self._h, C.ctypes.data))

    def tile(self):
        """(codes [n_cols, k] as uint32/uint16/uint8, scales [k])."""
        ld = ctypes.c_int64()
        _check(load().skm_get_tile(self._h, None, 0, None, ctypes.byref(ld)))
        dt = {FP32: np.uint32, BF16: np.uint16, FP8_E4M3: np.uint8}[self.precision]
        buf = np.empty((self.n_cols, ld.value), dtype=dt)
        sc = np.empty(self.k, dtype=np.float32)
        _check(load().skm_get_tile(self._h, buf.ctypes.data, buf.nbytes, sc.ctypes.data,
                                   ctypes.byref(ld)))
        return buf[:, :self.k], sc

    def changed(self):
        out = np.empty(self.k, dtype=np.uint8)
        _check(load().skm_get_changed(self._h, out.ctypes.data))
        return out

    def score_dense(self, csr):
        c, hold = make_csr(*csr, self.n_cols)
        out = np.empty((c.n_rows, self.k), dtype=np.float32)
        _check(load().skm_score_dense(self._h, ctypes.byref(c), out.ctypes.data))
        return out

    def error_bound(self, s, nnz, l1):
        return load().skm_error_bound(self._h, float(s), int(nnz), float(l1))

    def centroid_rows(self, ids):
        """FP64 centroids of the given ids, len(ids) x n_cols."""
        t = np.ascontiguousarray(ids, dtype=np.int32)
        out = np.empty((len(t), self.n_cols), dtype=np.float64)
        _check(load().skm_get_centroid_rows(self._h, t.ctypes.data, len(t), out.ctypes.data))
        return out

    def centroid_columns(self, terms):
        """FP64 centroid values at the given terms, k x len(terms)."""
        t = np.ascontiguousarray(terms, dtype=np.int32)
        out = np.empty((self.k, len(t)), dtype=np.float64)
        _check(load().skm_get_centroid_columns(self._h, t.ctypes.data, len(t), out.ctypes.data))
        return out

    def debug_fail_after(self, n_calls):
        """Test aid: the (n_calls + 1)-th checked HIP call reports a failure."""
        _check(load().skm_debug_fail_after(self._h, n_calls))

    def tune_lambda(self, n_sample=4096):
        """Tunes the index's threshold set on a row sample (skm_tune_lambda);
        returns the report as a dict."""
        rep = LambdaReport()
        _check(load().skm_tune_lambda(self._h, n_sample, ctypes.byref(rep)))
        g = rep.n_grid
        return {"n_sample": rep.n_sample, "grid": list(rep.grid[:g]),
                "qualify": list(rep.qualify[:g]), "mean_candidates": list(rep.mean_candidates[:g]),
                "before": list(rep.before[:rep.n_before]), "after": list(rep.after[:rep.n_after]),
                "cost_before": rep.cost_before, "cost_after": rep.cost_after,
                "applied": bool(rep.applied)}

    def autotune(self):
        """Times candidate shapes of the scoring work and keeps the fastest;
        returns {"best": {...}, "trials": [{...}, ...]}."""
        rep = TuneReport()
        _check(load().skm_autotune(self._h, ctypes.byref(rep)))
        trials = [{f: getattr(rep.trials[i], f) for f, _ in TuneTrial._fields_}
                  for i in range(rep.n_trials)]
        return {"best": trials[rep.best], "trials": trials}

    def set_schedule(self, shape):
        """Applies a shape returned by autotune() (a dict of TuneTrial fields)."""
        t = TuneTrial()
        for f, _ in TuneTrial._fields_:
            setattr(t, f, shape.get(f, 0))
        _check(load().skm_set_schedule(self._h, ctypes.byref(t)))

    def head_terms(self):
        """Terms scored on the matrix cores (0 = head off)."""
        return int(load().skm_head_terms(self._h))

    def score_head(self, row0, n_rows, parts=False):
        """Head-path low-precision scores of rows [row0, row0 + n_rows); with
        parts=True also the head parts alone: (scores, head_parts)."""
        out = np.empty((n_rows, self.k), dtype=np.float32)
        head = np.empty((n_rows, self.k), dtype=np.float32) if parts else None
        _check(load().skm_score_head(self._h, int(row0), int(n_rows), out.ctypes.data,
                                     head.ctypes.data if parts else None))
        return (out, head) if parts else out

    def error_bound_head(self, s, nnz, l1):
        return load().skm_error_bound_head(self._h, float(s), int(nnz), float(l1))

    def error_bound_split(self, hs, rs, n_rest, l1):
        return load().skm_error_bound_split(self._h, float(hs), float(rs), int(n_rest), float(l1))

    def index_level(self, level):
        lib = load()
        n = ctypes.c_int64()
        off = np.empty(self.n_cols + 1, dtype=np.int64)
        _check(lib.skm_get_index(self._h, level, off.ctypes.data, None, ctypes.byref(n)))
        ent = np.empty(n.value, dtype=np.uint32)
        _check(lib.skm_get_index(self._h, level, off.ctypes.data, ent.ctypes.data, ctypes.byref(n)))
        return off, ent

    def index_query(self, csr, level):
        """Candidate lists (list of int arrays) of the index at `level`."""
        c, hold = make_csr(*csr, self.n_cols)
        off = np.empty(c.n_rows + 1, dtype=np.int64)
        cap = max(1, c.n_rows * self.k)
        cand = np.empty(cap, dtype=np.int32)
        _check(load().skm_index_query(self._h, ctypes.byref(c), level, off.ctypes.data,
                                      cand.ctypes.data, cap))
        return [cand[off[i]:off[i + 1]].copy() for i in range(c.n_rows)]

    def hbm_bytes(self):
        return load().skm_hbm_bytes(self._h)


class Server:
    """Request server on a context (wraps skm_server): continuous batching of
    assign-new-rows requests.  submit() is thread-safe and returns a ticket;
    wait(ticket) returns (assignments, scores)."""

    def __init__(self, ctx: Context, n_slots=4, slot_rows=16384, slot_nnz=4 * 1024 * 1024,
                 hbm_budget_bytes=0, max_wait_us=100, use_graphs=True, max_jobs=2):
        lib = load()
        cfg = ServerConfig()
        lib.skm_server_config_default(ctypes.byref(cfg))
        cfg.n_slots, cfg.slot_rows, cfg.slot_nnz = n_slots, slot_rows, slot_nnz
        cfg.hbm_budget_bytes, cfg.max_wait_us = hbm_budget_bytes, max_wait_us
        cfg.use_graphs = 1 if use_graphs else 0
        cfg.max_jobs = max_jobs
        h = ctypes.c_void_p()
        _check(lib.skm_server_start(ctx._h, ctypes.byref(cfg), ctypes.byref(h)))
        self._h = h
        self._ctx = ctx
        self._out = {}
        import threading

        self._lock = threading.Lock()

    def submit(self, csr):
        c, hold = make_csr(*csr, self._ctx.n_cols)
        a = np.empty(c.n_rows, dtype=np.int32)
        s = np.empty(c.n_rows, dtype=np.float64)
        t = ctypes.c_int64()
        _check(load().skm_server_submit(self._h, ctypes.byref(c), a.ctypes.data, s.ctypes.data,
                                        ctypes.byref(t)))
        with self._lock:
            self._out[t.value] = ("rows", a, s)
        return t.value

    def submit_job(self, csr, n_cols, k, init_rows, centroids=False, **opts):
        """Queues a clustering job (skm_server_submit_job) with the same options
        as Context; wait(ticket) returns (assignments, centroids or None, info)."""
        lib = load()
        o = Options(**opts)
        cfg, keep = _config(lib, k, o, init_rows, None, None)
        c, hold = make_csr(*csr, n_cols)
        a = np.empty(c.n_rows, dtype=np.int32)
        C = np.empty((k, n_cols), dtype=np.float64) if centroids else None
        info = JobInfo()
        t = ctypes.c_int64()
        _check(lib.skm_server_submit_job(self._h, ctypes.byref(c), ctypes.byref(cfg), a.ctypes.data,
                                         C.ctypes.data if C is not None else None,
                                         ctypes.byref(info), ctypes.byref(t)))
        with self._lock:
            self._out[t.value] = ("job", a, C, info)
        return t.value

    def wait(self, ticket, timeout_s=-1.0):
        """(assignments, scores) for a request; (assignments, centroids or
        None, info dict) for a job."""
        try:
            _check(load().skm_server_wait(self._h, ticket, float(timeout_s)))
        except SkmError as e:
            if e.status != SKM_E_TIMEOUT:
                with self._lock:
                    self._out.pop(ticket, None)
            raise
        with self._lock:
            out = self._out.pop(ticket)
        if out[0] == "job":
            return out[1], out[2], out[3].asdict()
        return out[1], out[2]

    def cancel(self, ticket):
        _check(load().skm_server_cancel(self._h, ticket))

    def stats(self):
        st = ServerStats()
        _check(load().skm_server_get_stats(self._h, ctypes.byref(st)))
        return st.asdict()

    def stop(self):
        if getattr(self, "_h", None):
            h, self._h = self._h, None
            _check(load().skm_server_stop(h))

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.stop()
