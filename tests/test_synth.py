"""The seeded input generator (CPU only)."""
import numpy as np

import synth


def test_deterministic_and_thread_independent():
    c = synth.scaled(synth.PLAIN_1M.corpus, 3000, n_terms=20000)
    a = synth.generate(c, nthreads=1)
    b = synth.generate(c, nthreads=4)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_rows_well_formed():
    c = synth.SMALL.corpus
    ip, ix, v = synth.generate(c)
    lens = np.diff(ip)
    assert lens.min() >= c.nnz_min and lens.max() <= c.nnz_max
    assert ip[0] == 0 and ip[-1] == len(ix)
    for i in range(c.n_docs):
        r = ix[ip[i]:ip[i + 1]]
        assert np.all(np.diff(r) > 0)
    assert ix.min() >= 0 and ix.max() < c.n_terms
    assert np.all(v > 0) and np.all(np.isfinite(v))
    nrm = np.sqrt(np.add.reduceat(v.astype(np.float64) ** 2, ip[:-1]))
    assert np.abs(nrm - 1).max() < 1e-6


def test_length_and_zipf_shape():
    c = synth.scaled(synth.PRUNED_BF16_2M.corpus, 20000)
    ip, ix, v = synth.generate(c)
    lens = np.diff(ip)
    assert abs(lens.mean() - 150) < 6       # clipped lognormal, mean ~150
    df = np.bincount(ix, minlength=c.n_terms)
    assert df[0] >= df[1] >= df[5] > df[100] > df[10000]
    assert df[0] > 0.95 * c.n_docs            # rank 1 is in nearly every row


def test_seed_rows_distinct():
    r = synth.seed_rows(1000, 1000, 7)
    assert sorted(r.tolist()) == list(range(1000))
    r2 = synth.seed_rows(10**6, 50, 7)
    assert len(set(r2.tolist())) == 50 and np.array_equal(r2, synth.seed_rows(10**6, 50, 7))


def test_paper_shaped_corpora():
    """The stand-ins of the paper's corpora (Sec. 4.1) keep its vocabulary sizes
    and mean row lengths (10 and 58 non-zeros); checked on a row sample of the
    same generator, which draws every row independently."""
    for c, mean in ((synth.TWEETS_1M, 10.0), (synth.ABSTRACTS_200K, 58.0)):
        s = synth.scaled(c, 20000)
        ip, ix, v = synth.generate(s)
        lens = np.diff(ip)
        assert s.n_terms == c.n_terms
        assert abs(lens.mean() - mean) < 0.03 * mean, (c, lens.mean())
        assert lens.min() >= c.nnz_min and lens.max() <= c.nnz_max
        assert ix.max() < c.n_terms and np.all(v > 0)
    assert synth.TWEETS_1M.n_terms == 783_304 and synth.ABSTRACTS_200K.n_terms == 325_556
    assert synth.TWEETS_1M.n_docs == 1_000_000 and synth.ABSTRACTS_200K.n_docs == 200_000
