"""Checkpoint and resume (skm_save / skm_load through the C ABI; needs an
MI355X): a run saved after some iterations and resumed in a new context goes on
bit for bit as the uninterrupted run, with a centroid that has no members, NCC
and the index."""
import numpy as np
import pytest

import oracle
import synth
from paper_2108_00895_amd import Context, SkmError

from gpu_common import say, to_device

pytestmark = pytest.mark.gpu

TIMING = ("ms_assign", "ms_update", "ms_index", "ms_rescore", "ms_score", "ms_head", "ms_exact")


def _same_stats(a, b):
    for x, y in zip(a, b):
        for key in x:
            if key in TIMING or key.startswith("ms_"):
                continue
            assert x[key] == y[key], (key, x[key], y[key])


@pytest.mark.parametrize("prec,ncc,index", [("fp32", False, False), ("bf16", True, True),
                                            ("fp8", True, False)])
def test_resume_is_bitwise_identical(prec, ncc, index, tmp_path):
    say("case: checkpoint", prec, ncc, index)
    tc = synth.TopicCorpus(4000, 6000, 12, 400, 0.3, 40.0, 0.5, 5, 200, 1.1, seed=13)
    csr = synth.generate_topics(tc)
    k = 48
    rows = synth.seed_rows(tc.n_docs, k, 6)
    # the last centroid sits on a term no row has: it scores 0 everywhere, loses
    # every tie to a lower index and keeps no member, so its (stored) centroid
    # is the one the update leaves alone
    C0 = oracle.seed(csr, tc.n_terms, rows)
    used = np.zeros(tc.n_terms, dtype=bool)
    used[csr[1]] = True
    lonely = int(np.nonzero(~used)[0][0])
    C0[k - 1] = 0.0
    C0[k - 1, lonely] = 1.0
    dev = to_device(csr)
    opts = dict(precision=prec, ncc=ncc, index=index, stop_rule="fixed", max_iter=12)
    full = Context(dev, tc.n_terms, k, init_centroids=C0, **opts)
    head, _ = full.iterate(4)
    assert np.bincount(full.assignments(), minlength=k)[k - 1] == 0
    path = tmp_path / "run.ckpt"
    full.save(path)
    tail, _ = full.iterate(6)
    a_full, C_full = full.assignments(), full.centroids()
    full.close()

    res = Context.from_checkpoint(path, dev, tc.n_terms, k, **opts)
    tail2, _ = res.iterate(6)
    _same_stats(tail, tail2)
    assert np.array_equal(res.assignments(), a_full)
    assert np.array_equal(res.centroids(), C_full)      # bitwise
    res.close()

    assert np.array_equal(C_full[k - 1], C0[k - 1])
    say("  moved after resume:", [s["moved"] for s in tail2])


def test_checkpoint_states_and_mismatches(tmp_path):
    c = synth.Corpus(1500, 3000, 30.0, 0.5, 3, 200, 1.1, seed=41)
    csr = synth.generate(c)
    rows = synth.seed_rows(c.n_docs, 20, 2)
    ctx = Context(csr, c.n_terms, 20, init_rows=rows, stop_rule="fixed", max_iter=5)
    path = tmp_path / "x.ckpt"
    with pytest.raises(SkmError):          # nothing to save before the first update
        ctx.save(path)
    ctx.assign()
    ctx.update()
    # with an assignment pending its update the checkpoint is the state before
    # it: the resumed run repeats that assignment with the same result
    pend = ctx.assign()
    a_pend = ctx.assignments()
    ctx.save(path)
    r0 = Context.from_checkpoint(path, csr, c.n_terms, 20, stop_rule="fixed", max_iter=5)
    again = r0.assign()
    assert again["moved"] == pend["moved"] and again["changed_centroids"] == pend["changed_centroids"]
    assert np.array_equal(r0.assignments(), a_pend)
    r0.close()
    ctx.update()
    ctx.save(path)
    assert path.exists() and not (tmp_path / "x.ckpt.tmp").exists()
    with pytest.raises(SkmError):          # an unwritable place
        ctx.save(tmp_path / "no_such_dir" / "x.ckpt")
    with pytest.raises(SkmError):          # another k
        Context.from_checkpoint(path, csr, c.n_terms, 21, stop_rule="fixed")
    with pytest.raises(SkmError):          # another precision
        Context.from_checkpoint(path, csr, c.n_terms, 20, precision="bf16")
    with pytest.raises(SkmError):          # truncated
        data = path.read_bytes()
        bad = tmp_path / "short.ckpt"
        bad.write_bytes(data[: len(data) // 2])
        Context.from_checkpoint(bad, csr, c.n_terms, 20)
    r = Context.from_checkpoint(path, csr, c.n_terms, 20, stop_rule="fixed", max_iter=5)
    s1, _ = ctx.iterate(2)
    s2, _ = r.iterate(2)
    _same_stats(s1, s2)
    assert np.array_equal(ctx.assignments(), r.assignments())
    ctx.close()
    r.close()
