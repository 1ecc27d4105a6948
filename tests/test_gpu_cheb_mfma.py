"""Chebyshev RK4 time update on MFMA (FP32 densities, every N a multiple of 16)
against the FP64 oracle, through the C ABI.

Each predict is checked in lockstep: the GPU is given the oracle's grid and
density first, so the figure is one predict's own error, held to the FP32 bar of
the other FP32 parity tests (L1 <= 1e-5).  FP32 rounding in one evaluation of a
row of D2 is ~ n eps32 |D2| |y|, and the clamp keeps h |D2| Dy near 2.5, so each
substep adds O(10) eps32 (eps32 = 6e-8) to the L1 error, damped by the RK4
amplification of the high modes: the measured errors stay below 1e-6 up to the
several hundred substeps of the 64^3 grid."""
import numpy as np
import pytest

import oracle
import workloads as W
from gpu_common import Pair, fp32_update_tol, note

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


def tol_for(l):
    return 1e-5


def lockstep_predicts(B, ctx, model, prior, T, zs, what):
    p = Pair(B, ctx, model, prior)
    try:
        errs = []
        for k, z in enumerate(zs):
            p.inject_oracle_state()
            l = p.predict(T)
            assert B.pmf_last_substeps(p.f) == l, f"{what}: substeps differ"
            err = p.compare(tol_for(l), what=f"{what} predict {k} (l={l})")
            note(f"{what}: predict {k} l={l} L1={err:.3e} pointwise={p.last[1]:.3e}")
            errs.append(err)
            if z is not None:
                p.inject_oracle_state()
                ll, ll_o, status = p.update(z)
                assert abs(ll - ll_o) <= 1e-4 * max(1.0, abs(ll_o)), (what, k, ll, ll_o)
                p.compare(fp32_update_tol(p.amp), designed=True, what=f"{what} update {k} (A {p.amp:.0f})")
                note(f"{what}: update {k} L1={p.last[0]:.3e} pointwise={p.last[1]:.3e} "
                     f"dM={p.last[2]:.1e} dc={p.last[3]:.1e} cells")
        return errs
    finally:
        p.close()


def test_mfma_3d_n32(B, ctx):
    note("case: config3 recipe, Chebyshev 3-D N=32 FP32 (MFMA), 2 cycles lockstep")
    sc = W.config3(K=2, N=32, precision=W.FP32)
    lockstep_predicts(B, ctx, sc.model, sc.prior, sc.T, list(sc.z), "cheb3d-32")


def test_mfma_3d_n48(B, ctx):
    note("case: config3 recipe, Chebyshev 3-D N=48 FP32 (MFMA, 3-wave workgroups), 1 cycle lockstep")
    sc = W.config3(K=1, N=48, precision=W.FP32)
    lockstep_predicts(B, ctx, sc.model, sc.prior, sc.T, list(sc.z), "cheb3d-48")


def test_mfma_3d_ragged_axes(B, ctx):
    # axis lengths 16, 128 and 80: workgroups of 1, 8 and 5 waves, the rows
    # and the strided tile layouts on each; a short interval keeps l small
    note("case: Chebyshev 3-D N=(16,128,80) FP32 (MFMA), T=2e-4")
    sc = W.config3(K=1, N=16, precision=W.FP32)
    m = sc.model.with_(N=(16, 128, 80))
    lockstep_predicts(B, ctx, m, sc.prior, 2e-4, [None], "cheb3d-ragged")


def test_mfma_3d_plane_pass_rectangular(B, ctx):
    # square planes (N_1 = N_2 = 48) on a shorter first axis (N_0 = 32): the fused
    # plane pass with 3-wave workgroups and three 16-column chunks per plane
    note("case: Chebyshev 3-D N=(32,48,48) FP32 (MFMA, fused plane pass), T=0.01")
    sc = W.config3(K=1, N=16, precision=W.FP32)
    m = sc.model.with_(N=(32, 48, 48))
    lockstep_predicts(B, ctx, m, sc.prior, 0.01, [None], "cheb3d-plane-rect")


def test_mfma_2d_sheared(B, ctx):
    note("case: Chebyshev 2-D N=(64,32) FP32 (MFMA), sheared A, linear measurement")
    sc = W.config3(K=2, N=16, precision=W.FP32)
    m = sc.model.with_(nx=2, A=np.array([[-0.3, 0.8], [-0.6, -0.5]]), Q=np.array([[0.3, 0.0], [0.1, 0.4]]),
                       N=(64, 32), meas_kind=W.H_LINEAR, nz=1, H=np.array([[1.0, 0.5]]))
    prior = W.gaussian_prior([0.2, -0.1], [[0.5, 0.1], [0.1, 0.4]])
    lockstep_predicts(B, ctx, m, prior, 0.02, [np.array([0.3]), np.array([0.1])], "cheb2d-64x32")


def test_mfma_3d_64cubed_against_oracle(B, ctx):
    # the config-3 grid itself (the fused plane pass with 4-wave workgroups on
    # square 64 x 64 planes), in lockstep with the oracle; a short interval keeps
    # the oracle's substeps few, then the range-measurement update (3-D cubic
    # Lagrange re-interpolation on the sheared Chebyshev grid)
    note("case: config3 Chebyshev 3-D N=64 FP32 (MFMA plane pass), T=2e-4, lockstep vs oracle")
    sc = W.config3(K=1, N=64, precision=W.FP32)
    lockstep_predicts(B, ctx, sc.model, sc.prior, 2e-4, [sc.z[0]], "cheb3d-64")


def test_mfma_matches_fp64_gpu_at_64cubed(B, ctx):
    # full-size config-3 grid: the FP64 generic GPU path (itself parity-tested
    # against the oracle) as the reference for one predict of the MFMA path
    note("case: config3 Chebyshev 3-D N=64, one predict, MFMA FP32 vs generic FP64")
    sc = W.config3(K=1, N=64, precision=W.FP32)
    f32 = B.pmf_create(ctx, sc.model, sc.prior)
    f64 = B.pmf_create(ctx, sc.model.with_(precision=W.FP64), sc.prior)
    try:
        _, c0, M0, t0, P0 = B.pmf_get_state(f64)
        B.pmf_set_state(f32, c0, M0, t0, P0, W.CHEBYSHEV, W.FP32)
        B.pmf_predict(f32, sc.T)
        B.pmf_predict(f64, sc.T)
        l = B.pmf_last_substeps(f32)
        assert l == B.pmf_last_substeps(f64)
        _, c1, M1, _, P1 = B.pmf_get_state(f32)
        _, c2, M2, _, P2 = B.pmf_get_state(f64)
        np.testing.assert_allclose(M1, M2, rtol=0, atol=1e-12 * np.abs(M2).max())
        q = oracle.quadrature_weights(sc.model, np.asarray(M2))
        err = float(np.sum(q * np.abs(np.asarray(P1, float) - np.asarray(P2, float))))
        note(f"cheb3d-64: l={l} L1(MFMA FP32, FP64) = {err:.3e}")
        assert err <= tol_for(l), err
    finally:
        B.pmf_destroy(f32)
        B.pmf_destroy(f64)
