"""HIP path vs the FP64 oracle, element by element, through the C ABI.

Bar: L1 = sum_j q_j |P_gpu - P_oracle| <= 1e-10 for FP64 densities and <= 1e-5 for
FP32 densities (q_j the node's integration weight), and every point within the
same fraction of the oracle's peak; grids equal to rounding (designed FP32 grids:
the bars derived in gpu_common), log-likelihoods to 1e-9 (FP64) / 1e-4 (FP32),
substep counts equal (FP32 free-running: within one).
FP32 runs are checked in lockstep (before each cycle the GPU is given the
oracle's state, so each cycle's own error is measured) and free-running (both
sides carry their own state through every cycle).
"""
import numpy as np
import pytest

import oracle
import workloads as W
from gpu_common import Pair, l1, note, run_free, run_lockstep

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


def test_cfg1_1d_fp64_100_cycles(B, ctx):
    note("case: config1 1-D N=64 FP64 RK4, 100 cycles")
    run_free(B, ctx, W.config1(K=100), 100, 1e-10, what="cfg1")


def test_cfg2_2d_fp64_small_grid(B, ctx):
    note("case: config2 2-D N=48 FP64 RK4 cubic measurement, 12 cycles")
    run_free(B, ctx, W.config2(K=12, N=48), 12, 1e-10, what="cfg2-48")


def test_cfg2_2d_fp64_full_grid(B, ctx):
    note("case: config2 2-D N=128 FP64 RK4, 3 cycles")
    run_free(B, ctx, W.config2(K=3, N=128), 3, 1e-10, what="cfg2-128")


def test_cfg2_2d_fp32_full_grid_lockstep(B, ctx):
    note("case: config2 2-D N=128 FP32 RK4 lockstep, 3 cycles")
    run_lockstep(B, ctx, W.config2(K=3, N=128, precision=W.FP32), 3, 1e-5, what="cfg2-128-fp32")


@pytest.mark.parametrize("integ", [W.INT_EXACT, W.INT_RK4, W.INT_EULER])
def test_integrators_sheared_2d_ragged(B, ctx, integ):
    note(f"case: integrator {integ} 2-D N=(48,36) sheared grid")
    sc = W.config2(K=3, N=48, integrator=integ)
    sc.model = sc.model.with_(N=(48, 36), substeps=3)
    run_free(B, ctx, sc, 3, 1e-10, what=f"integ{integ}")


def test_axis_aligned_trig_regrid_2d(B, ctx):
    note("case: diagonal A, 2-D N=(32,48): separable trigonometric re-interpolation")
    sc = W.config2(K=4, N=32, integrator=W.INT_EXACT)
    sc.model = sc.model.with_(A=np.diag([-0.3, -0.7]), N=(32, 48))
    run_free(B, ctx, sc, 4, 1e-10, what="trig2d")


def test_forced_lagrange_1d(B, ctx):
    note("case: 1-D forced cubic Lagrange re-interpolation")
    sc = W.config1(K=10)
    sc.model = sc.model.with_(interp=W.INTERP_LAGRANGE)
    run_free(B, ctx, sc, 10, 1e-10, what="lagrange1d")


def test_3d_fourier_norm_measurement_fp64(B, ctx):
    note("case: 3-D Fourier N=(16,24,18) exact, range measurement")
    sc = W.config3(K=2, N=16)
    sc.model = sc.model.with_(grid=W.FOURIER, N=(16, 24, 18), integrator=W.INT_EXACT, precision=W.FP64)
    run_free(B, ctx, sc, 2, 1e-10, what="fourier3d")


def test_gaussian_mixture_noise_1d(B, ctx):
    note("case: 1-D two-component mixture measurement noise")
    sc = W.config1(K=6, N=96)
    sc.model = sc.model.with_(**W.gm_measurement_noise())
    # each measurement near one of the two modes: a posterior that sits in the far
    # tails of the predictive amplifies rounding noise and is not a parity case
    sc.z = sc.z * 0 + np.array([[0.3], [20.1], [-0.5], [19.6], [0.0], [20.4]])
    run_free(B, ctx, sc, 6, 1e-10, what="gm-noise")


def test_cfg1_1d_fp32_free_running_100_cycles(B, ctx):
    note("case: config1 1-D N=64 FP32 RK4, free-running 100 cycles (no resynchronisation)")
    run_free(B, ctx, W.config1(K=100, precision=W.FP32), 100, 1e-5, ll_tol=1e-4, what="cfg1-fp32-free",
             report=True)


def test_cfg2_2d_fp32_free_running_50_cycles(B, ctx):
    note("case: config2 2-D N=128 FP32 RK4 cubic measurement, free-running 50 cycles")
    run_free(B, ctx, W.config2(K=50, N=128, precision=W.FP32), 50, 1e-5, ll_tol=1e-4, what="cfg2-128-fp32-free",
             report=True)


def test_fp32_1d_lockstep(B, ctx):
    note("case: config1 FP32 lockstep, 10 cycles")
    run_lockstep(B, ctx, W.config1(K=10, precision=W.FP32), 10, 1e-5, what="cfg1-fp32")


def test_chebyshev_3d_fp64_small(B, ctx):
    note("case: config3 recipe, Chebyshev 3-D N=24 FP64, 2 cycles")
    sc = W.config3(K=2, N=24, precision=W.FP64)
    run_free(B, ctx, sc, 2, 1e-10, what="cheb3d")


def test_chebyshev_2d_fp64_axis_aligned(B, ctx):
    note("case: Chebyshev 2-D N=(20,24) diagonal A (polynomial re-interpolation)")
    sc = W.config3(K=2, N=12, precision=W.FP64)
    m = sc.model
    sc.model = m.with_(nx=2, A=np.diag([-0.4, -0.8]), Q=np.array([[0.3, 0.0], [0.1, 0.4]]), N=(20, 24),
                       meas_kind=W.H_LINEAR, nz=1, H=np.array([[1.0, 0.5]]))
    sc.prior = W.gaussian_prior([0.2, -0.1], [[0.5, 0.1], [0.1, 0.4]])
    sc.z = np.array([[0.3], [0.1]])
    run_free(B, ctx, sc, 2, 1e-10, what="cheb2d-sep")


def test_edge_sizes(B, ctx):
    for N in (4, 6, 256):
        note(f"case: 1-D exact N={N}")
        sc = W.config1(K=3, N=N)
        sc.model = sc.model.with_(integrator=W.INT_EXACT)
        run_free(B, ctx, sc, 3, 1e-10, what=f"N{N}")


def test_zero_interval_predict_is_identity(B, ctx):
    note("case: predict(0)")
    sc = W.config1(K=1)
    p = Pair(B, ctx, sc.model, sc.prior)
    try:
        c0, M0, t0, P0 = p.gpu_state()
        B.pmf_predict(p.f, 0.0)
        c1, M1, t1, P1 = p.gpu_state()
        assert np.array_equal(P0, P1) and np.array_equal(M0, M1) and t0 == t1
    finally:
        p.close()


def test_degenerate_update_leaves_state_unchanged(B, ctx):
    note("case: degenerate update (no mass where the likelihood lives)")
    sc = W.config1(K=1, N=32)
    model = sc.model.with_(integrator=W.INT_EXACT, **W.gaussian_noise([[1e-6]]))
    p = Pair(B, ctx, model, sc.prior)
    try:
        P = p.st.P.copy()
        P[16:] = 0.0
        p.st.P = P
        p.inject_oracle_state()
        X = oracle.nodes(model, p.st.c, p.st.M)
        z = np.array([X[24, 0]])
        before = p.gpu_state()
        ll = B.pmf_update(p.f, z, want_loglik=True)
        after = p.gpu_state()
        st = B.pmf_sync_status(p.f)
        assert np.isnan(ll)
        assert np.array_equal(before[3], after[3]) and np.array_equal(before[1], after[1])
        # the status word was read by pmf_get_state's header: the sticky bit is set
        _, _, st2 = B.pmf_moments(p.f, 1)
        hdr = B.pmf_get_state(p.f)[0]
        assert (st & B.PMF_E_DEGENERATE) or (st2 & B.PMF_E_DEGENERATE) or (hdr.status & B.PMF_E_DEGENERATE)
        _, ll_o, status, _, _ = oracle.update(model, p.st, z)
        assert status == oracle.pmf.STATUS_DEGENERATE
    finally:
        p.close()


def test_checkpoint_resume_is_bitwise(B, ctx):
    note("case: get_state / set_state resume")
    sc = W.config2(K=6, N=32)
    a = B.pmf_create(ctx, sc.model, sc.prior)
    b = B.pmf_create(ctx, sc.model, sc.prior)
    try:
        for k in range(3):
            B.pmf_predict(a, sc.T)
            B.pmf_update(a, sc.z[k])
        h, c, M, t, P = B.pmf_get_state(a)
        B.pmf_set_state(b, c, M, t, P, sc.model.grid, sc.model.precision)
        for k in range(3, 6):
            for f in (a, b):
                B.pmf_predict(f, sc.T)
                B.pmf_update(f, sc.z[k])
        sa, sb = B.pmf_get_state(a), B.pmf_get_state(b)
        assert np.array_equal(sa[4], sb[4]) and np.array_equal(sa[2], sb[2])
    finally:
        B.pmf_destroy(a)
        B.pmf_destroy(b)


def test_runs_are_deterministic(B, ctx):
    note("case: two identical runs are bitwise equal")
    sc = W.config2(K=4, N=48, precision=W.FP32)
    outs = []
    for _ in range(2):
        f = B.pmf_create(ctx, sc.model, sc.prior)
        lls = []
        for k in range(4):
            B.pmf_predict(f, sc.T)
            lls.append(B.pmf_update(f, sc.z[k], want_loglik=True))
        outs.append((B.pmf_get_state(f)[4], lls))
        B.pmf_destroy(f)
    assert np.array_equal(outs[0][0], outs[1][0]) and outs[0][1] == outs[1][1]


def test_invalid_arguments_are_rejected(B, ctx):
    note("case: invalid models / arguments")
    sc = W.config1(K=1)
    for bad in (dict(N=(62,)), dict(N=(2,)), dict(nx=1, substeps=0), dict(span_sigmas=-1.0),
                dict(grid=W.CHEBYSHEV, integrator=W.INT_EXACT)):
        with pytest.raises(B.PmfError) as e:
            B.pmf_create(ctx, sc.model.with_(**bad), sc.prior)
        assert e.value.status == B.PMF_E_INVALID
    f = B.pmf_create(ctx, sc.model, sc.prior)
    try:
        with pytest.raises(B.PmfError):
            B.pmf_predict(f, -1.0)
        with pytest.raises(B.PmfError):
            B.pmf_update(f, [float("nan")])
    finally:
        B.pmf_destroy(f)


def test_large_grid_update_recomputes_likelihood(B, ctx):
    """A grid of more than 2^21 points (160^3) has reduction chunks longer than the
    likelihood cache of a block, so the multiply pass evaluates each log-likelihood again
    instead of reading it back: one update from the prior against the oracle (FP64,
    diagonal A: separable trigonometric re-interpolation)."""
    from gpu_common import check_density
    note("case: 3-D Fourier N=160^3 FP64, one update from the prior (likelihood recomputed per pass)")
    sc = W.config3(K=1, N=16)
    m = sc.model.with_(grid=W.FOURIER, N=(160, 160, 160), integrator=W.INT_EXACT, precision=W.FP64,
                       A=np.diag([-0.3, -0.5, -0.7]), Q=np.diag([0.4, 0.5, 0.6]), meas_kind=W.H_LINEAR, nz=3,
                       H=np.eye(3), **W.gaussian_noise(0.3 ** 2 * np.eye(3)))
    prior = W.gaussian_prior(np.zeros(3), 0.5 ** 2 * np.eye(3))
    z = np.array([0.1, 0.0, -0.1])
    st = oracle.create(m, prior)
    st_o, ll_o, *_ = oracle.update(m, st, z)
    f = B.pmf_create(ctx, m, prior)
    try:
        ll = B.pmf_update(f, z, want_loglik=True)
        _, c, M, t, P = B.pmf_get_state(f)
        e1, em, _, _ = check_density(m, c, M, P, st_o, 1e-10, what="160^3 update")
        assert abs(ll - ll_o) <= 1e-9 * max(1.0, abs(ll_o)), (ll, ll_o)
        note(f"  L1 {e1:.2e}, pointwise {em:.2e} of the peak")
    finally:
        B.pmf_destroy(f)
