"""Serving: continuous batching of assign-new-rows requests (needs an MI355X).

Every request's answer must be the same alone (skm_assign_new) and in the mix
(batched with other requests by the server), and equal to the FP64 oracle.
With captured graphs every batch replays a slot's graph (sized for the slot,
the batch's row count read on the device), interleaved with the eager work of
other slots; each replay's answers are checked.
"""
import ctypes
import threading

import numpy as np
import pytest

import oracle
import synth
from paper_2108_00895_amd import Context, SkmError, skm
from paper_2108_00895_amd.skm import Server

from gpu_common import assert_assign_equal, corpus, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def resident():
    csr, c = corpus(3000, 9000, nnz_mean=60.0, nnz_max=400, seed=41)
    rows = synth.seed_rows(c.n_docs, 600, 2)
    ref = oracle.run(csr, c.n_terms, 600, rows, max_iter=2, stop_rule="fixed")
    return csr, c, ref.C


def _requests(D, n_req, seed):
    new, _ = corpus(5000, D, nnz_mean=60.0, nnz_max=400, seed=seed)
    rng = np.random.default_rng(seed)
    sizes = np.clip(np.round(rng.lognormal(np.log(16), 1.2, n_req)), 1, 300).astype(int)
    out, start = [], 0
    for sz in sizes:
        if start + sz > 5000:
            start = 0
        out.append(synth.subset(*new, np.arange(start, start + sz)))
        start += sz
    return out


@pytest.mark.parametrize("prec,graphs", [("bf16", True), ("fp8", True), ("bf16", False)])
def test_mix_equals_alone_and_oracle(prec, graphs, resident):
    csr, c, C = resident
    say("case: serving mix", prec, "graphs" if graphs else "eager")
    ctx = Context(csr, c.n_terms, 600, init_centroids=C, precision=prec)
    reqs = _requests(c.n_terms, 150, seed=7)
    alone = [ctx.assign_new(r) for r in reqs]
    got = [None] * len(reqs)
    with Server(ctx, n_slots=3, slot_rows=512, slot_nnz=512 * 400, max_wait_us=200,
                use_graphs=graphs) as srv:
        def client(ids):
            tickets = [(i, srv.submit(reqs[i])) for i in ids]
            for i, t in tickets:
                got[i] = srv.wait(t, 60.0)

        threads = [threading.Thread(target=client, args=(list(range(w, len(reqs), 4)),))
                   for w in range(4)]
        for th in threads:
            th.start()
        for th in threads:
            th.join()
        st = srv.stats()
        # the context is read-only while served
        with pytest.raises(SkmError) as e:
            ctx.assign()
        assert e.value.status == skm.SKM_E_BUSY
    say("  stats", {k: round(v, 3) if isinstance(v, float) else v for k, v in st.items()})
    assert st["requests_done"] == len(reqs) and st["batches"] < len(reqs)
    for r, (a1, s1), (a2, s2) in zip(reqs, alone, got):
        assert np.array_equal(a1, a2)
        assert np.array_equal(s1, s2)
        ar, r1, r2 = oracle.assign(r, C)
        assert_assign_equal(a2, ar, r1, r2, "served")
        np.testing.assert_allclose(s2, r1, rtol=1e-12)
    ctx.assign()   # writable again after stop
    ctx.close()


def test_server_admission_and_errors(resident):
    csr, c, C = resident
    say("case: serving errors")
    ctx = Context(csr, c.n_terms, 600, init_centroids=C, precision="bf16")
    with pytest.raises(SkmError) as e:
        Server(ctx, slot_rows=1024, slot_nnz=1 << 20, hbm_budget_bytes=1000)
    assert e.value.status == skm.SKM_E_NOMEM
    srv = Server(ctx, n_slots=8, slot_rows=64, slot_nnz=64 * 400, hbm_budget_bytes=700_000)
    assert 1 <= srv.stats()["slots"] < 8          # the budget limits the slots
    big = synth.subset(*csr, np.arange(100))
    with pytest.raises(SkmError) as e:
        srv.submit(big)                            # larger than a slot
    assert e.value.status == skm.SKM_E_INVALID
    t = srv.submit(synth.subset(*csr, np.arange(10)))
    a, s = srv.wait(t, 30.0)
    assert len(a) == 10
    empty = (np.zeros(1, np.int64), np.zeros(0, np.int32), np.zeros(0, np.float32))
    a0, _ = srv.wait(srv.submit(empty), 5.0)
    assert len(a0) == 0
    srv.stop()
    ctx.close()


def _job_corpus(n, seed):
    csr, c = corpus(n, 9000, nnz_mean=50.0, nnz_max=300, seed=seed)
    return csr, c


def test_jobs_beside_requests(resident):
    """Clustering jobs admitted by memory and run one iteration per turn beside
    request batches: each job's assignment and FP64 centroids are bit-identical
    to a standalone run of the same configuration, and every request answered
    meanwhile equals skm_assign_new and the oracle."""
    csr, c, C = resident
    say("case: jobs beside requests")
    ctx = Context(csr, c.n_terms, 600, init_centroids=C, precision="bf16")
    jobs = []
    for q, (n, k, prec) in enumerate([(4000, 40, "bf16"), (2500, 300, "fp32"), (3000, 120, "fp8")]):
        jc, jcorp = _job_corpus(n, 500 + q)
        jobs.append((jc, jcorp, k, prec, synth.seed_rows(n, k, 600 + q)))
    standalone = []
    for jc, jcorp, k, prec, rows in jobs:
        jx = Context(jc, jcorp.n_terms, k, init_rows=rows, precision=prec, ncc=True, max_iter=30)
        st, conv = jx.iterate()
        standalone.append((jx.assignments(), jx.centroids(), len(st), conv))
        jx.close()
    reqs = _requests(c.n_terms, 80, seed=17)
    alone = [ctx.assign_new(r) for r in reqs]
    with Server(ctx, n_slots=2, slot_rows=512, slot_nnz=512 * 400, max_jobs=2) as srv:
        tickets = [srv.submit_job(jc, jcorp.n_terms, k, rows, centroids=True, precision=prec,
                                  ncc=True, max_iter=30)
                   for jc, jcorp, k, prec, rows in jobs]
        got = [srv.wait(srv.submit(r), 60.0) for r in reqs]
        results = [srv.wait(t, 300.0) for t in tickets]
        st = srv.stats()
    say("  stats", {k_: v for k_, v in st.items() if "job" in k_ or k_ == "requests_done"})
    assert st["jobs_done"] == len(jobs) and st["job_iterations"] > len(jobs)
    for (a_s, C_s, it_s, conv_s), (a, Cj, info) in zip(standalone, results):
        assert np.array_equal(a, a_s)
        assert np.array_equal(Cj, C_s)
        assert info["iterations"] == it_s and bool(info["converged"]) == conv_s
        assert info["hbm_bytes"] > 0
    for r, (a1, s1), (a2, s2) in zip(reqs, alone, got):
        assert np.array_equal(a1, a2) and np.array_equal(s1, s2)
        ar, r1, r2 = oracle.assign(r, C)
        assert_assign_equal(a2, ar, r1, r2, "served beside jobs")
    ctx.close()


def test_job_admission_and_cancel(resident):
    """A job larger than the budget is refused; jobs beyond what the budget
    holds wait; cancelled requests and jobs return SKM_E_CANCELLED and write
    nothing; a request that timed out is not written later."""
    csr, c, C = resident
    say("case: job admission and cancel")
    ctx = Context(csr, c.n_terms, 600, init_centroids=C, precision="bf16")
    jc, jcorp = _job_corpus(3000, 77)
    rows = synth.seed_rows(3000, 50, 78)
    cfg, _ = skm._config(skm.load(), 50, skm.Options(precision="bf16"), rows, None, None)
    cc, _h = skm.make_csr(*jc, jcorp.n_terms)
    need = skm.load().skm_context_bytes(ctypes.byref(cc), ctypes.byref(cfg))
    slot = 2 * 1024 * 1024
    srv = Server(ctx, n_slots=1, slot_rows=64, slot_nnz=64 * 400, hbm_budget_bytes=slot + need,
                 max_jobs=4)
    # a job needing more than the whole budget is refused at once
    big, bcorp = _job_corpus(6000, 79)
    with pytest.raises(SkmError) as e:
        srv.submit_job(big, bcorp.n_terms, 600, synth.seed_rows(6000, 600, 80), precision="bf16")
    assert e.value.status == skm.SKM_E_NOMEM
    # two jobs that each fit but not together: the second waits for the first
    t1 = srv.submit_job(jc, jcorp.n_terms, 50, rows, precision="bf16", max_iter=20)
    t2 = srv.submit_job(jc, jcorp.n_terms, 50, rows, precision="bf16", max_iter=20)
    t3 = srv.submit_job(jc, jcorp.n_terms, 50, rows, precision="bf16", max_iter=20)
    srv.cancel(t3)
    with pytest.raises(SkmError) as e:
        srv.wait(t3, 30.0)
    assert e.value.status == skm.SKM_E_CANCELLED
    a1, _, i1 = srv.wait(t1, 120.0)
    a2, _, i2 = srv.wait(t2, 120.0)
    assert np.array_equal(a1, a2) and i1 == i2
    assert srv.stats()["jobs_running"] == 0
    # a cancelled request: nothing written, wait says so
    out = srv.submit(synth.subset(*csr, np.arange(5)))
    srv.cancel(out)
    with pytest.raises(SkmError) as e:
        srv.wait(out, 30.0)
    assert e.value.status in (skm.SKM_E_CANCELLED,)
    with pytest.raises(SkmError):
        srv.wait(123456, 1.0)                     # unknown ticket
    srv.stop()
    ctx.close()
