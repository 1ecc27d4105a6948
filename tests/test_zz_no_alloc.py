"""The allocation-free batched step against pmf_batch_step: twin filter sets
stepped through both entry points must agree exactly (same kernels, same
inputs, fixed-order reductions), on two calls in a row, the second smaller, and
the first call's results agree with the FP64 oracle within the FP32 bar."""
import numpy as np
import pytest

import oracle
import workloads as W
from gpu_common import l1_vs_oracle, note

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    from paper_2412_07240_amd import binding
    binding.lib()
    return binding


def zmat(scs, k):
    nz = max(sc.model.nz for sc in scs)
    z = np.zeros((len(scs), nz))
    for i, sc in enumerate(scs):
        z[i, :sc.model.nz] = sc.z[k]
    return z


def test_noalloc_matches_batch_step(B):
    ctx = B.pmf_ctx_create(0)
    try:
        for call, nf in enumerate((40, 12)):
            scs = W.batched_workload(nf, K=2)
            note(f"case: no-allocation step call {call}, {nf} mixed-size 2-D filters")
            fa = [B.pmf_create(ctx, sc.model, sc.prior) for sc in scs]
            fb = [B.pmf_create(ctx, sc.model, sc.prior) for sc in scs]
            try:
                before = [B.pmf_get_state(f)[1:] for f in fa]
                z = zmat(scs, 0)
                ll_a = B.pmf_batch_step_noalloc(ctx, fa, scs[0].T, z)
                ll_b = B.pmf_batch_step(ctx, fb, scs[0].T, z, want_loglik=True)
                assert np.array_equal(ll_a, ll_b, equal_nan=True), (call, np.nanmax(np.abs(ll_a - ll_b)))
                worst = 0.0
                for i, (f, g, sc) in enumerate(zip(fa, fb, scs)):
                    _, c1, M1, t1, P1 = B.pmf_get_state(f)
                    _, c2, M2, t2, P2 = B.pmf_get_state(g)
                    assert np.array_equal(c1, c2) and np.array_equal(M1, M2) and t1 == t2, (call, i)
                    assert np.array_equal(P1, P2), (call, i, np.abs(P1 - P2).max())
                    if i % 4 == 0:
                        c, M, t, P = before[i]
                        st = oracle.State(np.array(c), np.array(M), t, np.asarray(P, float))
                        st, _ = oracle.predict(sc.model, st, sc.T)
                        st, ll_o, _, _, _ = oracle.update(sc.model, st, sc.z[0])
                        err = l1_vs_oracle(sc.model, c1, M1, P1, st)
                        worst = max(worst, err)
                        assert err <= 1e-5, (call, i, err)
                        assert abs(ll_a[i] - ll_o) <= 1e-4 * max(1.0, abs(ll_o)), (call, i, ll_a[i], ll_o)
                note(f"  identical to pmf_batch_step; worst sampled L1 vs oracle {worst:.2e}")
            finally:
                for f in fa + fb:
                    B.pmf_destroy(f)
    finally:
        B.pmf_ctx_destroy(ctx)


def test_noalloc_rejects_more_than_its_limit(B):
    ctx = B.pmf_ctx_create(0)
    try:
        sc = W.batched_workload(1, K=1)[0]
        f = B.pmf_create(ctx, sc.model, sc.prior)
        try:
            fs = [f] * 4097
            with pytest.raises(B.PmfError) as ei:
                B.pmf_batch_step_noalloc(ctx, fs, sc.T, np.zeros((4097, sc.model.nz)))
            assert "4096" in str(ei.value)
            # a filter listed twice is refused before anything runs
            with pytest.raises(B.PmfError):
                B.pmf_batch_step_noalloc(ctx, [f, f], sc.T, np.zeros((2, sc.model.nz)))
        finally:
            B.pmf_destroy(f)
    finally:
        B.pmf_ctx_destroy(ctx)
