"""k-means++ seeding on the GPU (skm_kmeanspp, through the C ABI) against the
oracle's (needs an MI355X).  The seeds are integers decided in exact integer
arithmetic on both sides, so they must be equal, seed for seed."""
import time

import numpy as np
import pytest

import oracle
import synth
from paper_2108_00895_amd import Context, SkmError, kmeanspp

from gpu_common import say, to_device
from test_oracle_seed import _csr, _dyadic_rows

pytestmark = pytest.mark.gpu


def _draws(k, seed):
    return synth.stream_u64(seed, 7, 0, k)


@pytest.mark.parametrize("seed", range(4))
def test_dyadic_rows_equal_oracle(seed):
    rng = np.random.default_rng(seed)
    terms, vals = _dyadic_rows(300, 40, rng, dup_frac=0.3)
    csr = _csr(terms, vals)
    for k in (1, 2, 37, 300):
        d = _draws(k, 100 + seed)
        assert np.array_equal(kmeanspp(csr, 40, k, d), oracle.kmeanspp(csr, 40, k, d)), k


def test_identical_rows_fall_back_to_lowest_unchosen():
    csr = _csr([np.array([2, 5, 7, 11])] * 20, [0.5] * 20)
    d = _draws(20, 9)
    got = kmeanspp(csr, 16, 20, d)
    assert np.array_equal(got, oracle.kmeanspp(csr, 16, 20, d))
    assert sorted(got.tolist()) == list(range(20))


def test_generator_corpus_host_and_device_inputs():
    c = synth.Corpus(3000, 9000, 60.0, 0.6, 3, 400, 1.1, seed=31)
    csr = synth.generate(c)
    d = _draws(700, 5)
    ref = oracle.kmeanspp(csr, c.n_terms, 700, d)
    assert len(set(ref.tolist())) == 700
    assert np.array_equal(kmeanspp(csr, c.n_terms, 700, d), ref)
    assert np.array_equal(kmeanspp(to_device(csr), c.n_terms, 700, d), ref)


def test_many_row_blocks():
    """300,000 tweet-shaped rows: more than 1024 sums of 256 rows, so the draw
    crosses tiles of the selection scan."""
    c = synth.scaled(synth.TWEETS_1M, 300_000)
    csr = synth.generate(c)
    d = _draws(40, 6)
    assert np.array_equal(kmeanspp(to_device(csr), c.n_terms, 40, d),
                          oracle.kmeanspp(csr, c.n_terms, 40, d))


def test_full_tweet_corpus_and_a_trajectory_from_the_seeds():
    """The tweet-shaped corpus at full size (1e6 rows, k = 500): equal to the
    oracle; then clustering from these seeds runs like any other seeds."""
    c = synth.TWEETS_1M
    csr = synth.generate(c)
    dev = to_device(csr)
    d = _draws(500, 8)
    kmeanspp(dev, c.n_terms, 2, d)          # warm-up (module load)
    t0 = time.perf_counter()
    got = kmeanspp(dev, c.n_terms, 500, d)
    t = time.perf_counter() - t0
    t0 = time.perf_counter()
    ref = oracle.kmeanspp(csr, c.n_terms, 500, d)
    say(f"  k-means++ 1e6 tweet-shaped rows, k = 500: GPU {t:.3f} s, oracle "
        f"{time.perf_counter() - t0:.1f} s")
    assert np.array_equal(got, ref)
    ctx = Context(dev, c.n_terms, 500, init_rows=got, precision="bf16", ncc=True,
                  stop_rule="fixed", max_iter=2, validate=False)
    stats, _ = ctx.iterate()
    assert len(stats) == 2 and stats[0]["moved"] == c.n_docs
    ctx.close()


def test_bad_arguments():
    csr = _csr([np.array([0]), np.array([1])], [1.0, 1.0])
    with pytest.raises(SkmError):
        kmeanspp(csr, 2, 3, _draws(3, 1))
    with pytest.raises(SkmError):      # a term outside [0, n_cols)
        kmeanspp(csr, 1, 1, _draws(1, 1))
