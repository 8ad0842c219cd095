"""Helpers shared by the GPU parity tests."""
import sys

import numpy as np

import oracle
import synth

TIE = 1e-12


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def corpus(n, D, nnz_mean=40.0, sigma=0.6, nnz_max=300, zipf=1.1, seed=21):
    c = synth.Corpus(n, D, nnz_mean, sigma, 3, min(nnz_max, D), zipf, seed=seed)
    return synth.generate(c), c


def dense(csr, D):
    ip, ix, v = csr
    X = np.zeros((len(ip) - 1, D))
    for i in range(len(ip) - 1):
        X[i, ix[ip[i]:ip[i + 1]]] = v[ip[i]:ip[i + 1]]
    return X


def assert_assign_equal(a_gpu, a_ref, s1, s2, what=""):
    """Bit-exact except rows whose FP64 top-two gap is below 1e-12."""
    excused = (s1 - s2) < TIE
    bad = (a_gpu != a_ref) & ~excused
    assert not bad.any(), f"{what}: {int(bad.sum())} rows differ, first {np.nonzero(bad)[0][:5]}"
    return int(np.count_nonzero((a_gpu != a_ref) & excused))


def rel_centroid_err(C_gpu, C_ref):
    num = np.linalg.norm(C_gpu - C_ref, axis=1)
    den = np.maximum(np.linalg.norm(C_ref, axis=1), 1e-300)
    return float(np.max(num / den))


def to_device(csr):
    import torch

    return tuple(torch.from_numpy(np.ascontiguousarray(x)).cuda() for x in csr)
