"""K batched steps captured into one HIP graph (pmf_batch_run) against K calls
of pmf_batch_step: twin filter sets stepped through both entry points agree bit
for bit (same kernels, same inputs, fixed-order reductions), on the first call
(capture), on replays with other work of the program between them, and after K
changes (a new capture); the first step of the captured run is held to the FP64
oracle's bar."""
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


def zrows(scs, k0, K):
    z = np.zeros((K, len(scs), 2))
    for k in range(K):
        for i, sc in enumerate(scs):
            z[k, i] = sc.z[k0 + k]
    return z


def same_state(B, fa, fb, what):
    for i, (f, g) in enumerate(zip(fa, fb)):
        _, c1, M1, t1, P1 = B.pmf_get_state(f)
        _, c2, M2, t2, P2 = B.pmf_get_state(g)
        assert np.array_equal(c1, c2) and np.array_equal(M1, M2) and t1 == t2, (what, i)
        assert np.array_equal(P1, P2), (what, i, np.abs(P1 - P2).max())


def test_batch_run_matches_steps_and_replays(B):
    ctx = B.pmf_ctx_create(0)
    scs = W.batched_workload(40, K=20)
    T = scs[0].T
    fa = [B.pmf_create(ctx, sc.model, sc.prior) for sc in scs]
    fb = [B.pmf_create(ctx, sc.model, sc.prior) for sc in scs]
    try:
        k0 = 0
        for call, K in enumerate((6, 6, 3, 5)):
            note(f"case: pmf_batch_run call {call}, K = {K}, 40 mixed-size 2-D filters")
            before = [B.pmf_get_state(f)[1:] for f in fa[:3]] if call == 0 else None
            z = zrows(scs, k0, K)
            ll_run = B.pmf_batch_run(ctx, fa, T, z)
            ll_step = np.stack([B.pmf_batch_step(ctx, fb, T, z[k], want_loglik=True) for k in range(K)])
            assert np.array_equal(ll_run, ll_step, equal_nan=True), (call, np.nanmax(np.abs(ll_run - ll_step)))
            same_state(B, fa, fb, f"call {call}")
            if before is not None:
                # one filter's first step against the oracle, from a twin that stops after it
                for i in range(3):
                    c, M, t, P = before[i]
                    st = oracle.State(np.array(c), np.array(M), t, np.asarray(P, float))
                    st, _ = oracle.predict(scs[i].model, st, T)
                    st, ll_o, _, _, _ = oracle.update(scs[i].model, st, scs[i].z[0])
                    g = B.pmf_create(ctx, scs[i].model, scs[i].prior)
                    try:
                        ll1 = B.pmf_batch_run(ctx, [g], T, z[:1, i:i + 1])
                        _, c1, M1, t1, P1 = B.pmf_get_state(g)
                        err = l1_vs_oracle(scs[i].model, c1, M1, P1, st)
                        assert err <= 1e-5, (i, err)
                        assert abs(ll1[0, 0] - ll_o) <= 1e-4 * max(1.0, abs(ll_o)), (i, ll1[0, 0], ll_o)
                    finally:
                        B.pmf_destroy(g)
            # other work of the program between replays: moments of a few filters
            for f in fa[:4] + fb[:4]:
                B.pmf_moments(f, 2)
            k0 += K
        note("  every call bit for bit equal to the per-step calls")
    finally:
        for f in fa + fb:
            B.pmf_destroy(f)
        B.pmf_ctx_destroy(ctx)


def test_batch_run_rejects_bad_arguments(B):
    note("case: pmf_batch_run argument checks")
    ctx = B.pmf_ctx_create(0)
    scs = W.batched_workload(4, K=3)
    fs = [B.pmf_create(ctx, sc.model, sc.prior) for sc in scs]
    try:
        z = zrows(scs, 0, 3)
        bad = z.copy()
        bad[2, 3, 1] = np.nan
        with pytest.raises(B.PmfError):
            B.pmf_batch_run(ctx, fs, scs[0].T, bad)
        with pytest.raises(B.PmfError):
            B.pmf_batch_run(ctx, fs, scs[0].T, np.zeros((257, 4, 2)))
        with pytest.raises(B.PmfError):
            B.pmf_batch_run(ctx, fs, -1.0, z)
        # nothing ran: the filters are still at their priors' time
        assert all(B.pmf_get_state(f)[3] == 0.0 for f in fs)
        ll = B.pmf_batch_run(ctx, fs, scs[0].T, z)
        assert np.all(np.isfinite(ll)) and ll.shape == (3, 4)
    finally:
        for f in fs:
            B.pmf_destroy(f)
        B.pmf_ctx_destroy(ctx)
