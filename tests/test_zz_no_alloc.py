"""skm_assign_new_static (the no-allocation entry point) against skm_assign_new,
through the C ABI (needs an MI355X).

Two calls in a row on the same context, the second with fewer rows, each
bit-identical to skm_assign_new on the same rows (same kernels, same inputs);
rows beyond the static workspace and host rows are refused with nothing written.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from paper_2108_00895_amd import Context, SkmError, skm

from gpu_common import assert_assign_equal, corpus, say, to_device

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp8"])
def test_static_entry_point_equals_assign_new(prec):
    say("case: no-alloc entry point", prec)
    csr, c = corpus(3000, 9000, nnz_mean=60.0, nnz_max=400, seed=31)
    rows = synth.seed_rows(c.n_docs, 700, 5)
    ref = oracle.run(csr, c.n_terms, len(rows), rows, max_iter=2, stop_rule="fixed")
    ctx = Context(csr, c.n_terms, len(rows), init_rows=rows, precision=prec)
    ctx.set_centroids(ref.C)
    assert skm.load().skm_static_scratch_bytes() == 64 << 20
    big, _ = corpus(2500, c.n_terms, nnz_mean=60.0, nnz_max=400, seed=99)
    small = synth.subset(*big, np.arange(100, 331))
    for new in (big, small):
        n = len(new[0]) - 1
        a_ref, s_ref = ctx.assign_new(new)
        dev = to_device(new)
        out_a = torch.full((n,), -7, dtype=torch.int32, device="cuda")
        out_s = torch.full((n,), -7.0, dtype=torch.float64, device="cuda")
        ctx.assign_new_static(dev, out_a, out_s)
        a, s = out_a.cpu().numpy(), out_s.cpu().numpy()
        assert np.array_equal(a, a_ref), (prec, n)
        assert np.array_equal(s, s_ref), (prec, n)
        o_a, o_s1, o_s2 = oracle.assign(new, ref.C)
        assert_assign_equal(a, o_a, o_s1, o_s2, f"static {prec} n={n}")
    # more rows than the workspace holds: refused, outputs untouched
    cap = ctx.static_max_rows()
    nch = (len(rows) + 511) // 512
    assert (64 << 20) // (32 * nch + 45) - 32 <= cap <= (64 << 20) // (32 * nch + 45)
    many = (np.arange(cap + 2, dtype=np.int64), np.zeros(cap + 1, np.int32),
            np.ones(cap + 1, np.float32))
    dev = to_device(many)
    out_a = torch.full((cap + 1,), -7, dtype=torch.int32, device="cuda")
    out_s = torch.zeros(cap + 1, dtype=torch.float64, device="cuda")
    with pytest.raises(SkmError) as e:
        ctx.assign_new_static(dev, out_a, out_s)
    assert e.value.status == skm.SKM_E_INVALID
    assert bool((out_a == -7).all())
    # host rows are refused (they would need a device copy)
    with pytest.raises(SkmError) as e:
        ctx.assign_new_static(small, out_a, out_s)
    assert e.value.status == skm.SKM_E_INVALID
    ctx.close()
