"""Serving runtime (pmf_server_*) through the C ABI.

A served track must end where the same ops applied directly to a twin filter
end: fused pairs against pmf_batch_step of the twin alone (the same kernels),
single ops against pmf_predict / pmf_update (bit for bit).  The twins'
numerics are held to the oracle by the other GPU parity tests."""
import numpy as np
import pytest

import oracle
import workloads as W
from gpu_common import note

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    from paper_2412_07240_amd import binding
    binding.lib()
    return binding


@pytest.fixture(scope="module")
def ctx(B):
    c = B.pmf_ctx_create(0)
    yield c
    B.pmf_ctx_destroy(c)


def _mix():
    """Tracks of the serving mix plus filters that take the single-op path."""
    scs = [W.serving_track(i, K=4) for i in range(24)]
    extra = W.config3(K=4, N=32, precision=W.FP32)           # Chebyshev 3-D (MFMA)
    scs.append(extra)
    fp64 = W.serving_track(3, K=4)
    fp64.model = fp64.model.with_(precision=W.FP64)          # FP64 2-D or 1-D
    scs.append(fp64)
    return scs


def _l1(model, M, a, b):
    q = oracle.quadrature_weights(model, np.asarray(M))
    return float(np.sum(q * np.abs(np.asarray(a, float) - np.asarray(b, float))))


def test_served_tracks_match_direct_calls(B, ctx):
    scs = _mix()
    note(f"case: {len(scs)} served tracks, 3 predict+update cycles each, vs direct twins")
    srv = B.pmf_server_create(ctx, 1 << 36, 64)
    twins = []
    try:
        ids = [B.pmf_server_add_track(srv, sc.model, sc.prior) for sc in scs]
        twins = [B.pmf_create(ctx, sc.model, sc.prior) for sc in scs]
        K = 3
        tag = 0
        for k in range(K):
            for i, sc in enumerate(scs):
                B.pmf_server_submit_cycle(srv, ids[i], sc.T, sc.z[k], tag=tag)
                tag += 2
        B.pmf_server_drain(srv)
        done = B.pmf_server_poll(srv, cap=4 * tag)
        assert sorted(c["tag"] for c in done) == list(range(tag))
        assert all(c["status"] == B.PMF_OK for c in done), [c for c in done if c["status"]]
        by_tag = {c["tag"]: c for c in done}
        fused_tracks = {c["track"] for c in done if c["fused"]}
        note(f"fused tracks: {len(fused_tracks)} of {len(scs)}")
        assert len(fused_tracks) >= 12
        # twins: the same ops, directly (a cycle submitted as one unit either
        # ran fused or as two single ops; the completion says which)
        for i, sc in enumerate(scs):
            any_fused = False
            for k in range(K):
                t_upd = 2 * (k * len(scs) + i) + 1
                c = by_tag[t_upd]
                assert c["track"] == ids[i] and by_tag[t_upd - 1]["fused"] == c["fused"]
                if c["fused"]:
                    any_fused = True
                    ll = B.pmf_batch_step(ctx, [twins[i]], sc.T, np.asarray(sc.z[k])[None, :],
                                          want_loglik=True)[0]
                else:
                    B.pmf_predict(twins[i], sc.T)
                    ll = B.pmf_update(twins[i], sc.z[k], want_loglik=True)
                assert abs(c["loglik"] - ll) <= 1e-9 * max(1.0, abs(ll)), (i, k, c["loglik"], ll)
            _, c1, M1, _, P1 = B.pmf_get_state(B.pmf_server_filter(srv, ids[i]))
            _, c2, M2, _, P2 = B.pmf_get_state(twins[i])
            if not any_fused:
                np.testing.assert_array_equal(np.asarray(M1), np.asarray(M2))
                np.testing.assert_array_equal(np.asarray(P1), np.asarray(P2))
            else:
                sM = np.abs(np.asarray(M2)).max()
                np.testing.assert_allclose(np.asarray(M1), np.asarray(M2), rtol=0, atol=1e-9 * sM)
                np.testing.assert_allclose(np.asarray(c1), np.asarray(c2), rtol=0, atol=1e-9 * (1 + sM))
                err = _l1(sc.model, M2, P1, P2)
                assert err <= 1e-6, (i, err)
        st = B.pmf_server_stats_get(srv)
        assert st["completed"] == st["submitted"] == tag
        assert st["fused_ops"] + st["single_ops"] == tag
    finally:
        for f in twins:
            B.pmf_destroy(f)
        B.pmf_server_destroy(srv)


def test_per_track_fifo_order(B, ctx):
    note("case: one 2-D and one 3-D track, interleaved predicts and updates, completion order")
    sc2 = W.serving_track(1, K=6)
    sc3 = W.config3(K=6, N=16, precision=W.FP32)
    srv = B.pmf_server_create(ctx, 1 << 34, 4)
    try:
        a = B.pmf_server_add_track(srv, sc2.model, sc2.prior)
        b = B.pmf_server_add_track(srv, sc3.model, sc3.prior)
        ops = [(B.PMF_OP_PREDICT, 0), (B.PMF_OP_PREDICT, 0), (B.PMF_OP_UPDATE, 0), (B.PMF_OP_PREDICT, 0),
               (B.PMF_OP_UPDATE, 1), (B.PMF_OP_UPDATE, 2), (B.PMF_OP_PREDICT, 0), (B.PMF_OP_UPDATE, 3)]
        tag = 0
        for op, k in ops:
            for tr, sc in ((a, sc2), (b, sc3)):
                B.pmf_server_submit(srv, tr, op, T=0.02, z=sc.z[k], tag=tag)
                tag += 1
        B.pmf_server_drain(srv)
        done = B.pmf_server_poll(srv, cap=100)
        assert len(done) == tag
        for tr in (a, b):
            tags = [c["tag"] for c in done if c["track"] == tr]
            assert tags == sorted(tags), (tr, tags)
            assert len(tags) == len(ops)
    finally:
        B.pmf_server_destroy(srv)


def test_admission_budget(B, ctx):
    note("case: admission control by device-memory budget")
    sc = W.serving_track(1, K=1)
    srv = B.pmf_server_create(ctx, 1 << 40, 8)
    try:
        t0 = B.pmf_server_add_track(srv, sc.model, sc.prior)
        one = B.pmf_server_stats_get(srv)["used_bytes"]
    finally:
        B.pmf_server_destroy(srv)
    srv = B.pmf_server_create(ctx, int(2.5 * one), 8)
    try:
        a = B.pmf_server_add_track(srv, sc.model, sc.prior)
        b = B.pmf_server_add_track(srv, sc.model, sc.prior)
        with pytest.raises(B.PmfError) as ei:
            B.pmf_server_add_track(srv, sc.model, sc.prior)
        assert ei.value.status == B.PMF_E_NOMEM
        st = B.pmf_server_stats_get(srv)
        assert st["tracks"] == 2 and st["used_bytes"] <= st["budget_bytes"]
        B.pmf_server_remove_track(srv, a)
        c = B.pmf_server_add_track(srv, sc.model, sc.prior)
        assert c == a                                   # the freed slot is reused
        assert B.pmf_server_stats_get(srv)["tracks"] == 2
    finally:
        B.pmf_server_destroy(srv)


def test_rejected_update_and_invalid_requests(B, ctx):
    note("case: degenerate update on fused and single paths; invalid submissions")
    sc1 = W.serving_track(0, K=1)            # fusable 1-D or 2-D
    sc3 = W.config3(K=1, N=16, precision=W.FP32)
    srv = B.pmf_server_create(ctx, 1 << 34, 4)
    try:
        a = B.pmf_server_add_track(srv, sc1.model, sc1.prior)
        b = B.pmf_server_add_track(srv, sc3.model, sc3.prior)
        far1 = np.full(sc1.model.nz, 1e4)
        B.pmf_server_submit(srv, a, B.PMF_OP_PREDICT, T=0.05, tag=1)
        B.pmf_server_submit(srv, a, B.PMF_OP_UPDATE, z=far1, tag=2)
        B.pmf_server_submit(srv, b, B.PMF_OP_UPDATE, z=[1e4], tag=3)
        B.pmf_server_drain(srv)
        done = {c["tag"]: c for c in B.pmf_server_poll(srv)}
        assert done[1]["status"] == B.PMF_OK
        assert done[2]["status"] == B.PMF_E_DEGENERATE and np.isnan(done[2]["loglik"])
        assert done[3]["status"] == B.PMF_E_DEGENERATE and np.isnan(done[3]["loglik"])
        for bad in (dict(track=99, op=B.PMF_OP_PREDICT, T=0.1), dict(track=a, op=7, T=0.1),
                    dict(track=a, op=B.PMF_OP_PREDICT, T=float("nan")),
                    dict(track=a, op=B.PMF_OP_UPDATE, z=[float("inf")] * sc1.model.nz)):
            with pytest.raises(B.PmfError) as ei:
                B.pmf_server_submit(srv, **bad)
            assert ei.value.status == B.PMF_E_INVALID
        assert B.pmf_server_stats_get(srv)["submitted"] == 3
    finally:
        B.pmf_server_destroy(srv)
