"""Pins of the oracle's k-means++ seeding (CPU only).

The brute force below is an independent restatement of the same rules in exact
rational arithmetic, on rows whose values make every FP64 step of the oracle
exact (unit rows of 1, 4 or 16 equal entries 1, 1/2, 1/4), so the two must agree
seed for seed.  Closed forms: groups of identical rows with disjoint supports
get one seed each; with nothing left to separate, the lowest unchosen row.
"""
from fractions import Fraction

import numpy as np
import pytest

import oracle


def _csr(row_terms, row_vals):
    ip = np.zeros(len(row_terms) + 1, dtype=np.int64)
    ip[1:] = np.cumsum([len(t) for t in row_terms])
    ix = np.concatenate(row_terms).astype(np.int32)
    v = np.concatenate([np.full(len(t), x, dtype=np.float32) for t, x in zip(row_terms, row_vals)])
    return ip, ix, v


def _dyadic_rows(n, D, rng, dup_frac=0.2):
    terms, vals = [], []
    for i in range(n):
        if i > 0 and rng.random() < dup_frac:
            j = int(rng.integers(0, i))
            terms.append(terms[j].copy())
            vals.append(vals[j])
            continue
        m = int(rng.choice([1, 4, 16]))
        terms.append(np.sort(rng.choice(D, size=m, replace=False)))
        vals.append({1: 1.0, 4: 0.5, 16: 0.25}[m])
    return terms, vals


def _brute(terms, vals, k, draws):
    """k-means++ in exact rationals: weight floor(2^32 (1 - max cos)), chosen
    rows weigh 0, seed m sits where draws[m] mod W falls in the cumulative
    weights, the lowest unchosen row when W = 0."""
    n = len(terms)
    sets = [set(int(t) for t in ts) for ts in terms]
    val = [Fraction(x) for x in vals]
    best = [Fraction(0)] * n
    chosen = [False] * n
    r = int(draws[0]) % n
    seeds = [r]
    chosen[r] = True
    for m in range(1, k):
        # the rows are unit vectors exactly, so the cosine is the dot product
        for i in range(n):
            d = len(sets[i] & sets[r]) * val[i] * val[r]
            best[i] = max(best[i], d)
        w = [0 if chosen[i] else int((max(Fraction(0), 1 - best[i]) * 2**32) // 1)
             for i in range(n)]
        W = sum(w)
        if W == 0:
            r = chosen.index(False)
        else:
            t = int(draws[m]) % W
            acc = 0
            for i in range(n):
                if acc <= t < acc + w[i]:
                    r = i
                    break
                acc += w[i]
        seeds.append(r)
        chosen[r] = True
    return seeds


@pytest.mark.parametrize("seed", range(6))
def test_kmeanspp_equals_exact_brute_force(seed):
    rng = np.random.default_rng(seed)
    n, D = 60, 24
    terms, vals = _dyadic_rows(n, D, rng)
    csr = _csr(terms, vals)
    k = int(rng.integers(2, n + 1))
    draws = rng.integers(0, 2**63, size=k, dtype=np.uint64) * np.uint64(2) + np.uint64(1)
    got = oracle.kmeanspp(csr, D, k, draws)
    assert got.tolist() == _brute(terms, vals, k, draws)


def test_kmeanspp_all_rows_is_a_permutation():
    rng = np.random.default_rng(7)
    terms, vals = _dyadic_rows(40, 16, rng, dup_frac=0.5)
    draws = rng.integers(0, 2**64 - 1, size=40, dtype=np.uint64)
    got = oracle.kmeanspp(_csr(terms, vals), 16, 40, draws)
    assert sorted(got.tolist()) == list(range(40))
    assert got[0] == draws[0] % np.uint64(40)


def test_kmeanspp_one_seed_per_group_of_identical_rows():
    """g groups of identical rows on disjoint term sets: after a group is hit,
    its rows weigh 0 and the others the full 2^32, so k = g seeds land in g
    different groups for every draw; seed g + 1 has nothing to separate and is
    the lowest row not chosen."""
    g, per, D = 5, 7, 40
    terms, vals = [], []
    for a in range(g):
        t = np.arange(a * 8, a * 8 + 4)
        for _ in range(per):
            terms.append(t)
            vals.append(0.5)
    csr = _csr(terms, vals)
    rng = np.random.default_rng(3)
    for _ in range(20):
        draws = rng.integers(0, 2**64 - 1, size=g + 1, dtype=np.uint64)
        got = oracle.kmeanspp(csr, D, g + 1, draws)
        assert sorted(int(r) // per for r in got[:g]) == list(range(g))
        chosen = set(int(r) for r in got[:g])
        assert got[g] == min(set(range(g * per)) - chosen)


def test_kmeanspp_rejects_bad_k():
    csr = _csr([np.array([0])], [1.0])
    with pytest.raises(ValueError):
        oracle.kmeanspp(csr, 2, 2, np.zeros(2, dtype=np.uint64))
