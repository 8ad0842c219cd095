"""The C-ABI library loads and exports every entry point declared in
include/skm.h (CPU only: no compute call is made)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2108_00895_amd import skm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "skm.h")).read()
    return sorted(set(re.findall(r"^\s*(?:[\w\s\*]+?)\b(skm_\w+)\s*\(", text, re.M)))


def test_every_declared_symbol_is_exported():
    lib = skm.load()
    names = _declared()
    assert "skm_init" in names and "skm_assign_new" in names
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(names) == sorted(skm.EXPORTED)


def test_struct_layouts_match_header():
    # sizes follow the header's field order on x86-64
    assert ctypes.sizeof(skm.Csr) == 7 * 8
    assert ctypes.sizeof(skm.IterStats) == 4 + 4 + 8 * 8 + 5 * 8 + 5 * 4 + 4 + 4 + 4 + 8 + 4 + 4 + 8 + 4 + 4
    assert ctypes.sizeof(skm.Config) == 4 * 4 + 8 * 8 + 4 * 4 + 8 * 2 + 8 * 4 + 4 + 4 + 8 + 4 + 4
    cfg = skm.Config()
    skm.load().skm_config_default(ctypes.byref(cfg))
    assert cfg.n_lambda == 4 and list(cfg.lambda_[:4]) == [0.1, 0.25, 0.4, 0.6]
    assert cfg.max_shift_sq == 1e-4 and cfg.validate == 1
    assert cfg.head_max_terms == 4096 and cfg.head_min_df == 1.0 / 128


def test_tune_structs():
    assert ctypes.sizeof(skm.TuneTrial) == 4 + 4 + 8 + 8
    assert ctypes.sizeof(skm.TuneReport) == 4 + 4 + 16 * 24
    assert skm.load().skm_autotune(None, None) == skm.SKM_E_INVALID


def test_server_structs():
    assert ctypes.sizeof(skm.ServerConfig) == 4 + 4 + 8 + 8 + 4 + 4 + 4 + 4
    assert ctypes.sizeof(skm.ServerStats) == 3 * 8 + 5 * 8 + 4 + 4 + 8 + 8 + 8 + 4 + 4
    assert ctypes.sizeof(skm.JobInfo) == 4 + 4 + 8 + 8
    cfg = skm.ServerConfig()
    skm.load().skm_server_config_default(ctypes.byref(cfg))
    assert cfg.n_slots == 4 and cfg.slot_rows == 16384 and cfg.max_wait_us == 100
    assert cfg.use_graphs == 1 and cfg.max_jobs == 2
    assert skm.load().skm_server_start(None, None, ctypes.byref(ctypes.c_void_p())) == skm.SKM_E_INVALID


def test_null_arguments_rejected_without_device():
    lib = skm.load()
    h = ctypes.c_void_p()
    assert lib.skm_init(None, None, ctypes.byref(h)) == skm.SKM_E_INVALID
    assert b"NULL" in lib.skm_last_error()
    assert lib.skm_assign(None, None) == skm.SKM_E_INVALID
    assert lib.skm_kmeanspp(None, 1, None, None, None) == skm.SKM_E_INVALID
    # k outside [1, n_rows] is refused before any device call
    ip = np.array([0, 1], dtype=np.int64)
    ix = np.array([0], dtype=np.int32)
    v = np.array([1.0], dtype=np.float32)
    c = skm.Csr(1, 1, 1, ip.ctypes.data, ix.ctypes.data, v.ctypes.data, 0)
    out = np.zeros(2, dtype=np.int32)
    draws = np.zeros(2, dtype=np.uint64)
    assert lib.skm_kmeanspp(ctypes.byref(c), 2, draws.ctypes.data, out.ctypes.data,
                            None) == skm.SKM_E_INVALID
    assert b"k must be" in lib.skm_last_error()
    lib.skm_destroy(None)


def test_checkpoint_files_checked_without_device(tmp_path):
    """skm_load reads and checks the whole file before any device work: a
    missing file, a foreign file and a checkpoint of other rows are refused."""
    lib = skm.load()
    assert lib.skm_save(None, b"x") == skm.SKM_E_INVALID
    ip = np.array([0, 1, 2], dtype=np.int64)
    ix = np.array([0, 1], dtype=np.int32)
    v = np.array([1.0, 1.0], dtype=np.float32)
    c = skm.Csr(2, 2, 2, ip.ctypes.data, ix.ctypes.data, v.ctypes.data, 0)
    cfg = skm.Config()
    lib.skm_config_default(ctypes.byref(cfg))
    cfg.k = 1
    h = ctypes.c_void_p()
    missing = str(tmp_path / "missing.ckpt").encode()
    assert lib.skm_load(ctypes.byref(h), ctypes.byref(c), missing, ctypes.byref(cfg)) == \
        skm.SKM_E_INVALID
    foreign = tmp_path / "foreign.ckpt"
    foreign.write_bytes(b"not a checkpoint" * 16)
    assert lib.skm_load(ctypes.byref(h), ctypes.byref(c), str(foreign).encode(),
                        ctypes.byref(cfg)) == skm.SKM_E_INVALID
    assert b"not a checkpoint" in lib.skm_last_error()
    # a well-formed header for 3 rows does not fit these 2 rows
    import struct
    hdr = struct.pack("<8sIiqqqiIiiqiiiidqq", b"SKMCKPT1", 1, 1, 3, 2, 3, 0, 0, 1, 1, 0, 0, 8,
                      1, 0, 1.0, 0, 0)
    other = tmp_path / "other.ckpt"
    other.write_bytes(hdr)
    assert lib.skm_load(ctypes.byref(h), ctypes.byref(c), str(other).encode(),
                        ctypes.byref(cfg)) == skm.SKM_E_INVALID
    assert b"another shape" in lib.skm_last_error()
    assert not h.value


def test_context_bytes_estimate():
    """skm_context_bytes (job admission) bounds the allocations of skm_init from
    the sizes alone, grows with every size and is 0 for bad arguments."""
    lib = skm.load()
    cfg = skm.Config()
    lib.skm_config_default(ctypes.byref(cfg))
    cfg.k = 100
    c = skm.Csr(10_000, 50_000, 1_000_000, None, None, None, 0)
    base = lib.skm_context_bytes(ctypes.byref(c), ctypes.byref(cfg))
    # at least the FP64 centroids and sums and the rows themselves
    assert base >= 2 * 8 * 100 * 50_000 + 8 * 1_000_000
    # (rows stay longer than 64 terms on average: shorter ones change how the
    # update segments its sums, and with it the workspace bound)
    for field, val in (("n_rows", 12_000), ("n_cols", 90_000), ("nnz", 3_000_000)):
        c2 = skm.Csr(10_000, 50_000, 1_000_000, None, None, None, 0)
        setattr(c2, field, val)
        assert lib.skm_context_bytes(ctypes.byref(c2), ctypes.byref(cfg)) > base, field
    cfg.flags = skm.NCC | skm.INDEX
    assert lib.skm_context_bytes(ctypes.byref(c), ctypes.byref(cfg)) > base
    cfg.k = 0
    assert lib.skm_context_bytes(ctypes.byref(c), ctypes.byref(cfg)) == 0
    assert lib.skm_context_bytes(None, None) == 0
