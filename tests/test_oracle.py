"""Pins for the CPU FP64 oracle (CPU only).

Each test checks the oracle against something other than itself: dense numpy
brute force, closed forms, invariants of spherical k-means (paper Sec. 2), or
values fixed by hand.
"""
import numpy as np
import pytest

import oracle
import synth


def _tiny(n=300, D=400, seed=11, nnz_mean=20.0):
    c = synth.Corpus(n, D, nnz_mean, 0.5, 3, min(60, D), 1.1, seed=seed)
    return synth.generate(c), c


def _dense(csr, D):
    ip, ix, v = csr
    X = np.zeros((len(ip) - 1, D))
    for i in range(len(ip) - 1):
        X[i, ix[ip[i]:ip[i + 1]]] = v[ip[i]:ip[i + 1]]
    return X


def _unit_rows(rng, k, D, density=0.3):
    C = rng.random((k, D)) * (rng.random((k, D)) < density)
    C[:, 0] += 1e-3
    return C / np.linalg.norm(C, axis=1, keepdims=True)


def _first_argmax(S):
    # lowest index among the maxima, written without np.argmax's own convention
    best = np.zeros(S.shape[0], dtype=np.int64)
    for i in range(S.shape[0]):
        m = S[i].max()
        best[i] = min(j for j in range(S.shape[1]) if S[i, j] == m)
    return best


def test_assign_matches_dense_brute_force():
    csr, c = _tiny()
    rng = np.random.default_rng(5)
    C = _unit_rows(rng, 17, c.n_terms)
    a, s1, s2 = oracle.assign(csr, C)
    S = _dense(csr, c.n_terms) @ C.T
    ref = _first_argmax(S)
    gap = np.sort(S, axis=1)[:, -1] - np.sort(S, axis=1)[:, -2]
    ok = (a == ref) | (gap < 1e-12)
    assert ok.all()
    np.testing.assert_allclose(s1, S.max(axis=1), rtol=1e-13, atol=1e-15)
    other = S.copy()
    other[np.arange(len(a)), a] = -np.inf
    np.testing.assert_allclose(s2, other.max(axis=1), rtol=1e-13, atol=1e-15)
    # the dense product and the oracle's scores agree entry by entry
    np.testing.assert_allclose(oracle.scores(csr, C), S, rtol=1e-13, atol=1e-15)


def test_assign_listed_rows_and_ties():
    csr, c = _tiny()
    rng = np.random.default_rng(6)
    C = _unit_rows(rng, 5, c.n_terms)
    C = np.vstack([C, C[2:3], C[0:1]])  # duplicates of 2 and 0 at indices 5, 6
    docs = np.array([7, 3, 3, 250], dtype=np.int64)
    a, s1, _ = oracle.assign(csr, C, docs=docs)
    full, fs1, _ = oracle.assign(csr, C)
    assert (a == full[docs]).all() and (s1 == fs1[docs]).all()
    assert not np.isin(full, [5, 6]).any()   # exact duplicates never beat the lower index


def test_zero_overlap_row_goes_to_centroid_zero():
    ip = np.array([0, 2], dtype=np.int64)
    ix = np.array([1, 2], dtype=np.int32)
    v = np.array([0.6, 0.8], dtype=np.float32)
    C = np.zeros((3, 6))
    C[0, 4] = C[1, 5] = C[2, 3] = 1.0
    a, s1, s2 = oracle.assign((ip, ix, v), C)
    assert a[0] == 0 and s1[0] == 0.0 and s2[0] == 0.0


def test_update_matches_dense_sums():
    csr, c = _tiny()
    rng = np.random.default_rng(7)
    k = 9
    a = rng.integers(0, k - 1, size=c.n_docs).astype(np.int32)   # cluster k-1 stays empty
    C_old = _unit_rows(rng, k, c.n_terms)
    u = oracle.update(csr, a, C_old)
    X = _dense(csr, c.n_terms)
    for j in range(k):
        S = X[a == j].sum(axis=0)
        assert u.counts[j] == np.count_nonzero(a == j)
        if u.counts[j] == 0:
            assert np.array_equal(u.C[j], C_old[j]) and u.snorm[j] == 0.0
            continue
        np.testing.assert_allclose(u.snorm[j], np.linalg.norm(S), rtol=1e-13)
        np.testing.assert_allclose(u.C[j], S / np.linalg.norm(S), rtol=1e-12, atol=1e-15)
        np.testing.assert_allclose(u.shift_sq[j], np.sum((S / np.linalg.norm(S) - C_old[j]) ** 2),
                                   rtol=1e-10, atol=1e-15)
        np.testing.assert_allclose(u.dot_old[j], S @ C_old[j], rtol=1e-12, atol=1e-15)


def test_seed_is_normalised_row():
    csr, c = _tiny()
    rows = [4, 0, 299]
    C = oracle.seed(csr, c.n_terms, rows)
    X = _dense(csr, c.n_terms)
    for j, r in enumerate(rows):
        np.testing.assert_allclose(C[j], X[r] / np.linalg.norm(X[r]), rtol=1e-14, atol=0)


def test_k1_closed_form():
    csr, c = _tiny()
    r = oracle.run(csr, c.n_terms, 1, [10], max_iter=5)
    X = _dense(csr, c.n_terms)
    S = X.sum(axis=0)
    np.testing.assert_allclose(r.C[0], S / np.linalg.norm(S), rtol=1e-12, atol=1e-15)
    assert r.converged and len(r.records) == 2 and r.records[1].moved == 0


def test_k_equals_n_each_row_its_own_cluster():
    csr, c = _tiny(n=60, D=300, seed=3)
    X = _dense(csr, c.n_terms)
    rows = np.arange(c.n_docs)
    r = oracle.run(csr, c.n_terms, c.n_docs, rows, max_iter=3)
    rec = r.records[0]
    assert (rec.a == rows).all()
    np.testing.assert_allclose(rec.J_A, np.linalg.norm(X, axis=1).sum(), rtol=1e-12)


def test_planted_disjoint_blocks_recovered():
    # rows of block b use only terms [b*W, (b+1)*W): the clustering is exact
    rng = np.random.default_rng(9)
    B, W, per = 4, 30, 25
    ip, ix, v = [0], [], []
    truth = []
    for b in range(B):
        for _ in range(per):
            terms = np.sort(rng.choice(W, size=8, replace=False)) + b * W
            vals = rng.random(8) + 0.1
            vals /= np.linalg.norm(vals)
            ix.extend(terms)
            v.extend(vals)
            ip.append(len(ix))
            truth.append(b)
    csr = (np.array(ip, np.int64), np.array(ix, np.int32), np.array(v, np.float32))
    seeds = [b * per + 3 for b in range(B)]
    r = oracle.run(csr, B * W, B, seeds, max_iter=10)
    assert (r.a == np.array(truth)).all() and r.converged


def test_duplicate_seed_leaves_empty_cluster_unchanged():
    csr, c = _tiny()
    r = oracle.run(csr, c.n_terms, 3, [5, 5, 17], max_iter=1, stop_rule="fixed")
    C0 = oracle.seed(csr, c.n_terms, [5, 5, 17])
    # the duplicate never wins a tie against the lower index, so cluster 1 is
    # empty after the first assignment and keeps its seed centroid
    assert not (r.records[0].a == 1).any()
    assert np.array_equal(r.C[1], C0[1])
    assert not np.array_equal(r.C[0], C0[0])


def test_invariants_unit_norm_and_monotone_objective():
    w = synth.SMALL
    csr = synth.generate(w.corpus)
    rows = synth.seed_rows(w.corpus.n_docs, w.k, w.corpus.seed)
    r = oracle.run(csr, w.corpus.n_terms, w.k, rows, max_iter=w.max_iter, stop_rule="fixed")
    assert len(r.records) == 10
    nrm = np.linalg.norm(r.C, axis=1)
    assert np.all(np.abs(nrm - 1.0) < 1e-12)
    chain = []
    for rec in r.records:
        chain += [rec.J_A, rec.J_U]
    for x, y in zip(chain, chain[1:]):
        assert y >= x * (1 - 1e-12), (x, y)


def test_assign_objective_equals_sum_of_cluster_dots():
    csr, c = _tiny()
    rng = np.random.default_rng(12)
    C = _unit_rows(rng, 6, c.n_terms)
    a, s1, _ = oracle.assign(csr, C)
    u = oracle.update(csr, a, C)
    np.testing.assert_allclose(np.sum(s1), np.sum(u.dot_old), rtol=1e-12)


def test_stop_rules():
    csr, c = _tiny()
    rows = synth.seed_rows(c.n_docs, 6, 3)
    r = oracle.run(csr, c.n_terms, 6, rows, max_iter=50)
    assert r.converged
    last = r.records[-1]
    if r.stop_reason == "moved":
        assert last.moved == 0 and not last.updated
    else:
        assert last.max_shift_sq < 1e-4
    # a looser moved-fraction rule stops no later
    r2 = oracle.run(csr, c.n_terms, 6, rows, max_iter=50, min_moved_frac=0.05)
    assert len(r2.records) <= len(r.records)
    assert r2.records[-1].moved < 0.05 * c.n_docs or r2.stop_reason == "shift"


def test_centroid_rows_subset_matches_update():
    csr, c = _tiny()
    rng = np.random.default_rng(4)
    a = rng.integers(0, 7, size=c.n_docs).astype(np.int32)
    C_old = _unit_rows(rng, 7, c.n_terms)
    u = oracle.update(csr, a, C_old)
    rows, sn = oracle.centroid_rows(csr, c.n_terms, 7, a, [6, 1])
    np.testing.assert_array_equal(rows, u.C[[6, 1]])
    np.testing.assert_array_equal(sn, u.snorm[[6, 1]])


def test_assign_seeds_matches_dense_seeds():
    csr, c = _tiny()
    rows = [3, 77, 150, 151, 299, 12]
    docs = np.arange(0, c.n_docs, 3)
    C = oracle.seed(csr, c.n_terms, rows)
    a, s1, s2 = oracle.assign(csr, C, docs=docs)
    b, t1, t2 = oracle.assign_seeds(csr, c.n_terms, rows, docs)
    gap = s1 - s2
    assert np.all((a == b) | (gap < 1e-12))
    np.testing.assert_allclose(t1, s1, rtol=1e-14, atol=1e-16)
    np.testing.assert_allclose(t2, s2, rtol=1e-14, atol=1e-16)


def test_changed_set_is_the_clusters_whose_member_set_changed():
    """records[t].changed (the reference for the GPU's NCC flags, Sec. 3.1)
    against a brute-force comparison, cluster by cluster, of the member sets of
    the assignments before and after step t; iteration 0 changes every cluster."""
    c = synth.Corpus(800, 600, 20.0, 0.5, 3, 60, 1.1, seed=44)
    csr = synth.generate(c)
    k = 30
    rows = synth.seed_rows(c.n_docs, k, 3)
    ref = oracle.run(csr, c.n_terms, k, rows, max_iter=12, stop_rule="fixed")
    prev = None
    n_partial = 0
    for rec in ref.records:
        if not rec.updated:
            continue
        if prev is None:
            want = list(range(k))
        else:
            want = [j for j in range(k)
                    if set(np.nonzero(rec.a == j)[0].tolist()) !=
                    set(np.nonzero(prev == j)[0].tolist())]
        assert sorted(int(j) for j in rec.changed) == want, rec.t
        n_partial += 0 < len(want) < k
        prev = rec.a
    assert n_partial >= 5   # the run passes through partial changed sets


def test_trajectory_records_hold_each_iterations_own_assignment():
    """Each record's assignment is the lowest-index argmax against the
    centroids made from the previous record's assignment (dense numpy)."""
    csr, c = _tiny(n=300, D=400, seed=43)
    k = 9
    rows = synth.seed_rows(c.n_docs, k, 4)
    ref = oracle.run(csr, c.n_terms, k, rows, max_iter=6, stop_rule="fixed")
    X = _dense(csr, c.n_terms)
    C = X[rows] / np.linalg.norm(X[rows], axis=1, keepdims=True)
    for rec in ref.records:
        S = X @ C.T
        gap = np.sort(S, axis=1)[:, -1] - np.sort(S, axis=1)[:, -2]
        assert ((rec.a == _first_argmax(S)) | (gap < 1e-12)).all(), rec.t
        for j in range(k):
            m = rec.a == j
            if m.any():
                s = X[m].sum(axis=0)
                C[j] = s / np.linalg.norm(s)
