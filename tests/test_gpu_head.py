"""The dense head on the matrix cores, through the C ABI (needs an MI355X).

The most frequent terms are scored as a BF16 block on the matrix cores and
the rest on the sparse path.  Checked against the oracle:
  * every head-path score of a (row, centroid) pair lies within the certified
    head bound of the FP64 score (oracle centroids fed in), and for FP8 within
    the split bound of its head and sparse parts;
  * assignments with the head forced on equal the oracle's, for the first
    step, for whole trajectories, and across chunk groups with a ragged last
    group and a ragged last centroid chunk;
  * head on and head off give the same assignments;
  * the head size follows the stated selection rule.
"""
import math

import numpy as np
import pytest

import oracle
import synth
from paper_2108_00895_amd import Context, SkmError, skm

from gpu_common import assert_assign_equal, corpus, say, to_device

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mid():
    csr, c = corpus(3000, 9000, nnz_mean=60.0, nnz_max=400, seed=31)
    rows = synth.seed_rows(c.n_docs, 700, 5)
    return csr, c, rows


def expected_head(csr, n_rows, max_terms, min_df):
    """The selection rule, restated: terms in >= max(1, ceil(min_df * N)) rows,
    count rounded up to 64, capped by max_terms (to 64) and by the terms present."""
    df = np.bincount(csr[1], minlength=1)
    thr = max(1.0, math.ceil(min_df * n_rows))
    n_qual = int(np.count_nonzero(df >= thr))
    n_pos = int(np.count_nonzero(df > 0))
    H = min(-(-n_qual // 64) * 64, (max_terms // 64) * 64, (n_pos // 64) * 64)
    return H if H >= 64 else 0


def test_head_selection(mid):
    csr, c, rows = mid
    say("case: head selection")
    for prec, mx, mdf in [("bf16", 4096, 1 / 128), ("bf16", 100, 1 / 128), ("fp8", 4096, 0.05),
                          ("bf16", 4096, 0.9), ("bf16", 0, 1 / 128), ("fp32", 4096, 1 / 128),
                          ("bf16", 64, 0.0)]:
        ctx = Context(csr, c.n_terms, 50, init_rows=rows[:50], precision=prec,
                      head_max_terms=mx, head_min_df=mdf)
        want = 0 if prec == "fp32" else expected_head(csr, c.n_docs, mx, mdf)
        assert ctx.head_terms() == want, (prec, mx, mdf, ctx.head_terms(), want)
        st = ctx.assign()
        assert st["head_terms"] == want
        say(f"  {prec} max {mx} min_df {mdf:.4f}: H = {want}")
        ctx.close()


@pytest.mark.parametrize("prec", ["bf16", "fp8"])
@pytest.mark.parametrize("H", [64, 640])
def test_head_bound_holds_for_every_pair(prec, H, mid):
    csr, c, rows = mid
    say("case: head bound", prec, H)
    ref = oracle.run(csr, c.n_terms, 300, rows[:300], max_iter=2, stop_rule="fixed")
    C = ref.C
    ctx = Context(csr, c.n_terms, 300, init_centroids=C, precision=prec, head_max_terms=H,
                  head_min_df=0.0)
    assert ctx.head_terms() == H
    n = 500
    Sg = ctx.score_head(0, n).astype(np.float64)
    Sr = oracle.scores(csr, C, np.arange(n))
    ip, ix, v = csr
    nnz = np.diff(ip)[:n]
    l1 = np.add.reduceat(v.astype(np.float64), ip[:-1])[:n]
    worst = 0.0
    for i in range(n):
        E = np.array([ctx.error_bound_head(s, nnz[i], l1[i]) for s in Sg[i]])
        worst = max(worst, float(np.max(np.abs(Sg[i] - Sr[i]) / E)))
    assert worst <= 1.0, worst
    # the same rows scored in a later batch position agree bit for bit
    Sg2 = ctx.score_head(100, 50).astype(np.float64)
    np.testing.assert_array_equal(Sg2, Sg[100:150])
    say("  max |s^-s|/E =", worst)
    ctx.close()


@pytest.mark.parametrize("H", [64, 640])
def test_split_bound_holds_for_every_pair(H, mid):
    """FP8 with the head: the head part of a score comes from BF16 head codes
    rounded from the FP64 centroids, the rest from the FP8 codes, and the
    assignment step bounds each pair by the two parts' own bounds.  Checked
    on every (row, centroid) pair against the oracle's FP64 scores.  The
    library returns the total and the head part; the rest is taken as their
    difference, which differs from the kernel's own rest by at most one
    rounding of the total (2^-24 of it), covered by an extra 2^-22 * score."""
    csr, c, rows = mid
    say("case: split bound", H)
    ref = oracle.run(csr, c.n_terms, 300, rows[:300], max_iter=2, stop_rule="fixed")
    C = ref.C
    ctx = Context(csr, c.n_terms, 300, init_centroids=C, precision="fp8", head_max_terms=H,
                  head_min_df=0.0)
    assert ctx.head_terms() == H
    n = 500
    S, Hp = ctx.score_head(0, n, parts=True)
    S, Hp = S.astype(np.float64), Hp.astype(np.float64)
    Sr = oracle.scores(csr, C, np.arange(n))
    ip, ix, v = csr
    df = np.bincount(ix, minlength=c.n_terms)
    head = np.zeros(c.n_terms, dtype=bool)
    head[np.argsort(-df, kind="stable")[:H]] = True      # the selection rule, restated
    l1 = np.add.reduceat(v.astype(np.float64), ip[:-1])[:n]
    worst, ratio = 0.0, []
    for i in range(n):
        n_rest = int(np.count_nonzero(~head[ix[ip[i]:ip[i + 1]]]))
        R = np.maximum(S[i] - Hp[i], 0.0)
        E = np.array([ctx.error_bound_split(h, r, n_rest, l1[i]) for h, r in zip(Hp[i], R)])
        E += 2.0 ** -22 * S[i]
        worst = max(worst, float(np.max(np.abs(S[i] - Sr[i]) / E)))
        E1 = np.array([ctx.error_bound_head(s, ip[i + 1] - ip[i], l1[i]) for s in S[i]])
        ratio.append(float(np.sum(E) / np.sum(E1)))
    assert worst <= 1.0, worst
    assert ctx.error_bound_split(1.0, 1.0, 10, 1.0) > 0
    say(f"  max |s^-s|/E = {worst:.3f}; split bound / single bound = {np.mean(ratio):.3f}")
    ctx.close()
    bf = Context(csr, c.n_terms, 300, init_centroids=C, precision="bf16", head_max_terms=H,
                 head_min_df=0.0)
    assert bf.error_bound_split(1.0, 1.0, 10, 1.0) == -1.0
    bf.close()


@pytest.mark.parametrize("prec", ["bf16", "fp8"])
def test_head_trajectory_equals_oracle(prec, mid):
    csr, c, rows = mid
    say("case: head trajectory", prec)
    ref = oracle.run(csr, c.n_terms, len(rows), rows, max_iter=5, stop_rule="fixed")
    ctx = Context(to_device(csr), c.n_terms, len(rows), init_rows=rows, precision=prec,
                  head_max_terms=192, head_min_df=0.0, stop_rule="fixed", max_iter=5)
    for t, rec in enumerate(ref.records):
        st = ctx.assign()
        assert st["head_terms"] == 192
        n_tie = assert_assign_equal(ctx.assignments(), rec.a, rec.s1, rec.s2, f"{prec} it {t}")
        assert st["moved"] == rec.moved
        u = ctx.update()
        assert abs(u["objective_assign"] - rec.J_A) <= 1e-9 * abs(rec.J_A)
        assert abs(u["objective_update"] - rec.J_U) <= 1e-9 * abs(rec.J_U)
        say(f"  it {t}: flagged {st['flagged']} ties {n_tie}")
    ctx.close()


@pytest.mark.parametrize("prec", ["bf16", "fp8"])
def test_head_on_and_off_give_the_same_assignments(prec, mid):
    """Head off is the plain sparse path (for FP8 with bound summaries from the
    FP8 bound on every term); head on uses the head product (for FP8 the split
    bound).  Both are exact, so the assignments agree."""
    csr, c, rows = mid
    say("case: head on/off", prec)
    got = []
    for mx in [0, 4096]:
        ctx = Context(csr, c.n_terms, len(rows), init_rows=rows, precision=prec, ncc=True,
                      head_max_terms=mx, stop_rule="fixed", max_iter=4)
        assert (ctx.head_terms() > 0) == (mx > 0)
        seq = []
        for _ in range(4):
            ctx.assign()
            seq.append(ctx.assignments())
            ctx.update()
        got.append(seq)
        ctx.close()
    for a0, a1 in zip(*got):
        np.testing.assert_array_equal(a0, a1)


def test_head_chunk_groups_ragged():
    """k = 5000: ten 512-centroid chunks, scored in head groups of four
    (4, 4, 2), the last chunk 392 columns wide; 9000 rows (not a multiple of
    the 256-row GEMM tile).  Several row batches are covered at full size by
    test_gpu_fullsize.py (2e6 rows in batches of 2^20)."""
    say("case: head chunk groups")
    csr, c = corpus(9000, 3000, nnz_mean=40.0, nnz_max=200, seed=41)
    rows = synth.seed_rows(c.n_docs, 5000, 9)
    C0 = oracle.seed(csr, c.n_terms, rows)
    a_ref, s1, s2 = oracle.assign(csr, C0)
    ctx = Context(to_device(csr), c.n_terms, 5000, init_rows=rows, precision="bf16",
                  head_max_terms=256, head_min_df=0.0)
    assert ctx.head_terms() == 256
    st = ctx.assign()
    assert st["head_terms"] == 256
    n_tie = assert_assign_equal(ctx.assignments(), a_ref, s1, s2, "chunk groups")
    say(f"  flagged {st['flagged']} ties {n_tie}")
    ctx.close()


def test_autotune_changes_only_the_schedule(mid):
    csr, c, rows = mid
    say("case: autotune")
    got = []
    for tune in [False, True]:
        ctx = Context(csr, c.n_terms, len(rows), init_rows=rows, precision="bf16",
                      stop_rule="fixed", max_iter=4)
        seq = []
        for it in range(4):
            if tune and it == 2:
                rep = ctx.autotune()
                assert 1 <= len(rep["trials"]) <= 16 and rep["best"] in rep["trials"]
                assert all(t["ms"] > 0 for t in rep["trials"])
                # the fastest trial is kept
                assert min(t["ms"] for t in rep["trials"]) == rep["best"]["ms"]
                say("  autotune best", rep["best"])
            st = ctx.assign()
            if tune and it == 2:
                with pytest.raises(SkmError) as e:
                    ctx.autotune()               # an assignment is pending
                assert e.value.status == skm.SKM_E_STATE
            seq.append((ctx.assignments(), st["moved"]))
            ctx.update()
        got.append(seq)
        ctx.close()
    for (a0, m0), (a1, m1) in zip(*got):
        np.testing.assert_array_equal(a0, a1)
        assert m0 == m1


def test_set_schedule_validates(mid):
    csr, c, rows = mid
    say("case: set schedule")
    ctx = Context(csr, c.n_terms, len(rows), init_rows=rows, precision="bf16")
    a0 = ctx.assign()
    base = ctx.assignments()
    ctx.update()
    rep = ctx.autotune()
    other = Context(csr, c.n_terms, len(rows), init_rows=rows, precision="bf16")
    other.set_schedule(rep["best"])
    other.assign()
    np.testing.assert_array_equal(other.assignments(), base)
    for bad in [{"head_chunks": 99, "head_rows": 256, "workgroups_per_cu": 4},
                {"head_chunks": 1, "head_rows": 1 << 40, "workgroups_per_cu": 4},
                {"head_chunks": 1, "head_rows": 256, "workgroups_per_cu": 99}]:
        with pytest.raises(SkmError) as e:
            other.set_schedule(bad)
        assert e.value.status == skm.SKM_E_INVALID
    say("  flagged", a0["flagged"], "best", rep["best"])
    ctx.close()
    other.close()


@pytest.mark.parametrize("prec", ["bf16", "fp8"])
def test_head_with_ncc_trajectory_equals_oracle(prec):
    """NCC iterations with the head: rows keeping their centroid score the
    compacted changed centroids (head codes compacted too when more than 64
    changed, every term from the compacted codes without the head product
    when at most 64 did), the others score all centroids from their list;
    every step must equal the oracle.  40 rows per cluster keep a partial
    changed set for several iterations (86, 53, 32, 19, 9, 6, 4, ... changed
    centroids: both variants and every narrow width run)."""
    say("case: head + ncc trajectory", prec)
    csr, c = corpus(8000, 6000, nnz_mean=50.0, nnz_max=300, seed=47)
    k, T = 200, 14
    rows = synth.seed_rows(c.n_docs, k, 3)
    ref = oracle.run(csr, c.n_terms, k, rows, max_iter=T, stop_rule="fixed")
    ctx = Context(to_device(csr), c.n_terms, k, init_rows=rows, precision=prec, ncc=True,
                  head_max_terms=128, head_min_df=0.0, stop_rule="fixed", max_iter=T)
    both = 0
    widths = set()
    for t, rec in enumerate(ref.records):
        st = ctx.assign()
        assert st["head_terms"] == 128
        # both passes ran: some rows kept their centroid, some did not, and
        # some (but not all) centroids changed
        ok = 0 < st["ncc_rows"] < c.n_docs and 0 < st["changed_centroids"] <= k // 2
        both += ok
        if ok:
            n_ch = st["changed_centroids"]
            widths.add("head" if n_ch > 64 else min(w for w in (8, 16, 32, 64) if n_ch <= w))
        assert_assign_equal(ctx.assignments(), rec.a, rec.s1, rec.s2, f"{prec} it {t}")
        assert st["moved"] == rec.moved
        u = ctx.update()
        assert abs(u["objective_update"] - rec.J_U) <= 1e-9 * abs(rec.J_U)
        say(f"  it {t}: changed {st['changed_centroids']} ncc rows {st['ncc_rows']} "
            f"flagged {st['flagged']}")
    assert both >= 3, "NCC with the head did not run with a partial changed set"
    assert widths == {"head", 8, 16, 32, 64}, widths
    ctx.close()
