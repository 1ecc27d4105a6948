"""A context created with an allocator puts every device allocation of its filters
and batches through it: here PyTorch's caching allocator, from the binding.
Results equal those of a context on hipMalloc, bit for bit."""
import numpy as np
import pytest

import workloads as W
from gpu_common import note

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    from paper_2412_07240_amd import binding
    binding.lib()
    return binding


def test_torch_caching_allocator_backs_filters_and_batches(B):
    import torch
    torch.cuda.init()
    counter = {}
    base = torch.cuda.memory_allocated(0)
    ctx_t = B.pmf_ctx_create(0, allocator=B.torch_allocator(0, counter))
    ctx_h = B.pmf_ctx_create(0)
    sc = W.config2(K=3, N=48, precision=W.FP32)
    scs = W.batched_workload(6, K=2)
    note("case: filters and a batched step on a context backed by torch's caching allocator")
    try:
        f_t = B.pmf_create(ctx_t, sc.model, sc.prior)
        f_h = B.pmf_create(ctx_h, sc.model, sc.prior)
        assert counter.get("alloc", 0) >= 8, counter
        assert torch.cuda.memory_allocated(0) - base >= counter["bytes"], (torch.cuda.memory_allocated(0), counter)
        for k in range(3):
            for f in (f_t, f_h):
                B.pmf_predict(f, sc.T)
                B.pmf_update(f, sc.z[k])
        a, b = B.pmf_get_state(f_t), B.pmf_get_state(f_h)
        assert np.array_equal(a[2], b[2]) and np.array_equal(a[4], b[4])
        # a batched step (its launch set-up allocates through the allocator too)
        n0 = counter["alloc"]
        bt = [B.pmf_create(ctx_t, s.model, s.prior) for s in scs]
        bh = [B.pmf_create(ctx_h, s.model, s.prior) for s in scs]
        z = np.array([s.z[0] for s in scs])
        l_t = B.pmf_batch_step(ctx_t, bt, scs[0].T, z, want_loglik=True)
        l_h = B.pmf_batch_step(ctx_h, bh, scs[0].T, z, want_loglik=True)
        assert counter["alloc"] > n0 + 6 * 8, counter
        assert np.array_equal(l_t, l_h)
        for x, y in zip(bt, bh):
            assert np.array_equal(B.pmf_get_state(x)[4], B.pmf_get_state(y)[4])
        for f in bt + bh + [f_t, f_h]:
            B.pmf_destroy(f)
    finally:
        B.pmf_ctx_destroy(ctx_t)
        B.pmf_ctx_destroy(ctx_h)
    note(f"  allocator calls: {counter}")
    assert counter["free"] == counter["alloc"], counter
    assert torch.cuda.memory_allocated(0) == base


def test_batch_refuses_grids_without_a_fused_form_up_front(B):
    """The fused kernel has forms for N0 x N1 with N0, N1 in {32, 48, 64, 96, 128}
    (square and rectangular): any other 2-D grid is refused before anything runs,
    and still steps through pmf_predict / pmf_update."""
    ctx = B.pmf_ctx_create(0)
    try:
        sc = W.batched_workload(1, K=1)[0]
        for N in ((80, 64), (64, 40)):
            m = sc.model.with_(N=N)
            f = B.pmf_create(ctx, m, sc.prior)
            try:
                with pytest.raises(B.PmfError) as e:
                    B.pmf_batch_step(ctx, [f], sc.T, np.asarray(sc.z[:1]))
                assert e.value.status == B.PMF_E_INVALID and "fused form" in str(e.value), (N, str(e.value))
                B.pmf_predict(f, sc.T)
                assert np.isfinite(B.pmf_update(f, sc.z[0], want_loglik=True))
            finally:
                B.pmf_destroy(f)
    finally:
        B.pmf_ctx_destroy(ctx)
