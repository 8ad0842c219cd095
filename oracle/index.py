"""The dot-product index of paper Sec. 3.2 — TEST INFRASTRUCTURE ONLY.

Pure Python, exact arithmetic (``fractions.Fraction`` over the double values),
for small inputs.  It is used to check the GPU index and candidate sets.

Definitions (Sec. 3.2, Lemma 3.1 and the construction that follows it):
  * G[t]: every centroid with a non-zero value at term t (the basic inverted
    index).
  * For one centroid, sort its non-zero entries by value, descending (equal
    values: ascending term id).  At position p with value v_p:
      - v_p >= lam gives minimum overlap count m_p = 1;
      - otherwise m_p = the least m such that v_p^2 + ... + v_{p+m-1}^2 >= lam^2;
      - if no such m exists, no further position of this centroid enters P.
    P[t] receives (centroid, m_p) for the entered positions.
  * Query for a row x: count[j] = number of terms of x that have j in G; the
    candidates are the j for which some term t of x has (j, m) in P[t] with
    count[j] >= m.

Readings: comparisons are ">=" everywhere; G receives every non-zero entry even
after P insertion stops for that centroid (G is defined as the list of all
centroids with a non-zero value at a term, and the overlap count must count all
of them for the candidate set to contain every centroid that reaches lam).
"""
from __future__ import annotations

from fractions import Fraction


def sorted_entries(terms, vals):
    """Non-zero entries of one centroid, value descending, then term ascending."""
    pairs = [(float(v), int(t)) for t, v in zip(terms, vals) if v != 0.0]
    pairs.sort(key=lambda p: (-p[0], p[1]))
    return pairs


def overlap_counts_naive(pairs, lam: float):
    """m_p for every position of one centroid, from the definition, in exact
    arithmetic: fresh sums from each position.  None where P insertion stopped."""
    lam2 = Fraction(lam) ** 2
    sq = [Fraction(v) ** 2 for v, _ in pairs]
    out = []
    stopped = False
    for p, (v, _) in enumerate(pairs):
        if stopped:
            out.append(None)
            continue
        if Fraction(v) >= Fraction(lam):
            out.append(1)
            continue
        acc = Fraction(0)
        m = None
        for q in range(p, len(pairs)):
            acc += sq[q]
            if acc >= lam2:
                m = q - p + 1
                break
        if m is None:
            stopped = True
            out.append(None)
        else:
            out.append(m)
    return out


def overlap_counts_linear(pairs, lam: float):
    """The same m_p with the linear-time two-pointer build (Sec. 3.2 footnote):
    a running sum that adds each square once when the window end advances and
    subtracts it once when the window start passes it.  Exact arithmetic, so it
    must equal overlap_counts_naive."""
    lam2 = Fraction(lam) ** 2
    sq = [Fraction(v) ** 2 for v, _ in pairs]
    n = len(pairs)
    out = [None] * n
    end = 0            # window is [p, end)
    acc = Fraction(0)  # sum of sq over the window
    for p in range(n):
        if end < p:
            end, acc = p, Fraction(0)
        if Fraction(pairs[p][0]) >= Fraction(lam):
            out[p] = 1
        else:
            while end < n and acc < lam2:
                acc += sq[end]
                end += 1
            if acc < lam2:
                break          # threshold unreachable: stop this centroid
            out[p] = end - p
        if end > p:
            acc -= sq[p]
    return out


def build(centroids, lam: float, linear: bool = False):
    """centroids: list of (terms, values).  Returns (G, P): dict term -> sorted
    list of centroid ids; dict term -> list of (centroid id, m)."""
    G, P = {}, {}
    for j, (terms, vals) in enumerate(centroids):
        pairs = sorted_entries(terms, vals)
        ms = (overlap_counts_linear if linear else overlap_counts_naive)(pairs, lam)
        for (v, t), m in zip(pairs, ms):
            G.setdefault(t, []).append(j)
            if m is not None:
                P.setdefault(t, []).append((j, m))
    return G, P


def query(G, P, row_terms):
    """Candidate set (sorted list of centroid ids) for a row with these terms."""
    count = {}
    for t in row_terms:
        for j in G.get(int(t), ()):
            count[j] = count.get(j, 0) + 1
    cand = set()
    for t in row_terms:
        for j, m in P.get(int(t), ()):
            if count.get(j, 0) >= m:
                cand.add(j)
    return sorted(cand)


def select_level(levels, baseline_lo: float, row_norm: float):
    """Index level for a row: the highest lam with lam * ||x|| <= baseline lower
    bound (Sec. 3.2 picks the highest threshold still below the baseline; the
    ||x|| factor extends Lemma 3.1 to rows that are not exactly unit length).
    None when no level qualifies."""
    best = None
    for i, lam in enumerate(levels):
        if lam * row_norm <= baseline_lo and (best is None or lam > levels[best]):
            best = i
    return best
