"""Pins for the oracle's dot-product index (paper Sec. 3.2, Lemma 3.1). CPU only."""
import json
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import index as ix

GOLD = os.path.join(os.path.dirname(__file__), "golden", "index_worked_example.json")


def test_worked_example_m_values():
    g = json.load(open(GOLD))
    for lam, per in g["m"].items():
        for name, want in per.items():
            c = g["centroids"][name]
            pairs = ix.sorted_entries(c["terms"], c["values"])
            assert [t for _, t in pairs] == g["sorted_terms"][name]
            assert ix.overlap_counts_naive(pairs, float(lam)) == want, (lam, name)
            assert ix.overlap_counts_linear(pairs, float(lam)) == want, (lam, name)


def test_worked_example_queries():
    g = json.load(open(GOLD))
    names = list(g["centroids"])
    cents = [(g["centroids"][n]["terms"], g["centroids"][n]["values"]) for n in names]
    for q in g["queries"]:
        G, P = ix.build(cents, q["lambda"])
        got = [names[j] for j in ix.query(G, P, q["row_terms"])]
        assert got == q["candidates"], q
        counts = {n: sum(1 for t in q["row_terms"] if j in G.get(t, [])) for j, n in enumerate(names)}
        assert counts == q["counts"]


def _rand_unit_sparse(rng, D, nnz):
    t = np.sort(rng.choice(D, size=nnz, replace=False))
    v = rng.random(nnz) ** 3 + 1e-3
    return t, v / np.linalg.norm(v)


def test_lemma_3_1_random():
    rng = np.random.default_rng(0)
    D = 60
    for _ in range(2000):
        ct, cv = _rand_unit_sparse(rng, D, rng.integers(1, D))
        xt, xv = _rand_unit_sparse(rng, D, rng.integers(1, 15))
        c = np.zeros(D); c[ct] = cv
        x = np.zeros(D); x[xt] = xv
        dot = c @ x
        lam = rng.random() * dot if dot > 0 else 0.0
        # c.x >= lam implies the squared centroid mass on supp(x) is >= lam^2
        assert np.sum(c[xt] ** 2) >= lam ** 2 * (1 - 1e-12)


@pytest.mark.parametrize("lam", [0.1, 0.25, 0.4, 0.6])
def test_naive_equals_linear_build(lam):
    rng = np.random.default_rng(int(lam * 100))
    for _ in range(60):
        t, v = _rand_unit_sparse(rng, 200, rng.integers(1, 120))
        pairs = ix.sorted_entries(t, v)
        assert ix.overlap_counts_naive(pairs, lam) == ix.overlap_counts_linear(pairs, lam)


@pytest.mark.parametrize("lam", [0.1, 0.25, 0.4, 0.6])
def test_candidates_superset_of_true_reachers(lam):
    rng = np.random.default_rng(100 + int(lam * 10))
    D, k = 80, 25
    cents = [_rand_unit_sparse(rng, D, rng.integers(3, 40)) for _ in range(k)]
    G, P = ix.build(cents, lam)
    C = np.zeros((k, D))
    for j, (t, v) in enumerate(cents):
        C[j, t] = v
    n_pruned = 0
    for _ in range(300):
        xt, xv = _rand_unit_sparse(rng, D, rng.integers(1, 12))
        x = np.zeros(D); x[xt] = xv
        cand = set(ix.query(G, P, xt))
        reach = set(np.nonzero(C @ x >= lam)[0].tolist())
        assert reach <= cand
        # every candidate has a non-zero overlap (it came from G and P)
        assert all(np.any(C[j, xt] > 0) for j in cand)
        n_pruned += k - len(cand)
    assert n_pruned > 0   # the index does prune something on these inputs


def test_m_non_decreasing_and_stop_is_suffix_rule():
    rng = np.random.default_rng(3)
    for _ in range(40):
        t, v = _rand_unit_sparse(rng, 150, rng.integers(2, 100))
        pairs = ix.sorted_entries(t, v)
        for lam in (0.1, 0.25, 0.4, 0.6):
            ms = ix.overlap_counts_naive(pairs, lam)
            lam2 = Fraction(lam) ** 2
            sq = [Fraction(x) ** 2 for x, _ in pairs]
            entered = [m for m in ms if m is not None]
            assert entered == sorted(entered)
            # P holds exactly the positions whose suffix reaches lam^2
            # (or whose value alone reaches lam)
            for p, m in enumerate(ms):
                suffix = sum(sq[p:], Fraction(0))
                reaches = suffix >= lam2 or Fraction(pairs[p][0]) >= Fraction(lam)
                first_stop = next((q for q, mm in enumerate(ms) if mm is None), len(ms))
                assert (m is not None) == (p < first_stop)
                if p < first_stop:
                    assert reaches


def test_select_level():
    lv = [0.1, 0.25, 0.4, 0.6]
    assert ix.select_level(lv, 0.3, 1.0) == 1
    assert ix.select_level(lv, 0.25, 1.0) == 1      # equality qualifies
    assert ix.select_level(lv, 0.09, 1.0) is None
    assert ix.select_level(lv, 0.6, 1.0) == 3
    assert ix.select_level(lv, 0.25, 1.0 + 1e-7) == 0   # row slightly longer than 1
