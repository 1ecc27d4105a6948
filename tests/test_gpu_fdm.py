"""Finite-difference baseline (sine-transform route of eq. FST, with the fast sine
transform: an FFT of the odd extension of length 2 (N + 1) per axis), the
sine-series variant of the spectral update, and the FFT radices their sizes need
(5, 7, 11, 13, 17), HIP path vs the FP64 oracle (dense sine matrices, dense DFT)
through the C ABI.  Same bars as the other parity tests: L1 <= 1e-10 (FP64),
<= 1e-5 per cycle in lockstep (FP32)."""
import numpy as np
import pytest

import workloads as W
from gpu_common import note, run_free, run_lockstep

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


def _diag_scenario(nx, N, K, precision=W.FP64, seed=11, integrator=W.INT_FDM):
    rng = np.random.default_rng(seed)
    A = np.diag(rng.uniform(-1.0, -0.1, size=nx))
    Q = np.diag(rng.uniform(0.3, 0.9, size=nx))
    T = 0.05
    m = W.ModelSpec(nx=nx, A=A, Q=Q, N=N, t_nominal=T, integrator=integrator, substeps=2,
                    precision=precision, meas_kind=W.H_LINEAR, nz=nx, H=np.eye(nx),
                    **W.gaussian_noise(0.3 ** 2 * np.eye(nx)))
    prior = W.gaussian_prior(np.zeros(nx), 0.5 ** 2 * np.eye(nx))
    return W.simulate(m, prior, T, K, rng)


def test_fdm_1d_n80(B, ctx):
    note("case: config1 recipe, finite differences, N=80, FP64, 5 cycles")
    sc = W.config1(K=5, N=80)
    sc.model = sc.model.with_(integrator=W.INT_FDM)
    run_free(B, ctx, sc, 5, 1e-10, what="fdm1d-80")


def test_fdm_2d(B, ctx):
    note("case: finite differences 2-D N=(48,50) FP64, 3 cycles (extensions 98 = 2 7^2, 102 = 2 3 17)")
    run_free(B, ctx, _diag_scenario(2, (48, 50), 3), 3, 1e-10, what="fdm2d")


@pytest.mark.parametrize("N", [90, 120, 224])
def test_fdm_1d_fast_sine_transform_sizes(B, ctx, N):
    # odd extensions of length 182 = 2 7 13, 242 = 2 11^2, 450 = 2 3^2 5^2
    note(f"case: config1 recipe, finite differences, N={N} (sine transform by an FFT of length {2 * (N + 1)}), FP64")
    sc = W.config1(K=3, N=N)
    sc.model = sc.model.with_(integrator=W.INT_FDM)
    run_free(B, ctx, sc, 3, 1e-10, what=f"fdm1d-{N}")


def test_sine_1d_n168(B, ctx):
    note("case: config1 recipe, sine-series update, N=168 (FFT of length 338 = 2 13^2), FP64")
    sc = W.config1(K=3, N=168)
    sc.model = sc.model.with_(integrator=W.INT_SINE)
    run_free(B, ctx, sc, 3, 1e-10, what="sine1d-168")


@pytest.mark.parametrize("N", [22, 26, 98])
def test_radix_7_11_13_exact_1d(B, ctx, N):
    note(f"case: config1 recipe, exact integrator, N={N} (radix-7/11/13 FFT passes), FP64")
    sc = W.config1(K=3, N=N)
    sc.model = sc.model.with_(integrator=W.INT_EXACT)
    run_free(B, ctx, sc, 3, 1e-10, what=f"radix-{N}")


def test_fdm_refuses_sizes_without_a_fast_sine_transform(B, ctx):
    # 2 (40 + 1) = 82 = 2 41: no radix plan for the odd extension
    sc = W.config1(K=1, N=40)
    with pytest.raises(B.PmfError) as e:
        B.pmf_create(ctx, sc.model.with_(integrator=W.INT_FDM), sc.prior)
    assert e.value.status == B.PMF_E_INVALID


def test_fdm_3d(B, ctx):
    note("case: finite differences 3-D N=(16,20,24) FP64, 2 cycles")
    run_free(B, ctx, _diag_scenario(3, (16, 20, 24), 2), 2, 1e-10, what="fdm3d")


def test_fdm_2d_fp32_lockstep(B, ctx):
    note("case: finite differences 2-D N=(64,48) FP32 lockstep, 3 cycles")
    run_lockstep(B, ctx, _diag_scenario(2, (64, 48), 3, precision=W.FP32), 3, 1e-5, what="fdm2d-fp32")


@pytest.mark.parametrize("N", [80, 200])
def test_radix5_exact_1d(B, ctx, N):
    note(f"case: config1 recipe, exact integrator, N={N} (radix-5 FFT passes), FP64")
    sc = W.config1(K=4, N=N)
    sc.model = sc.model.with_(integrator=W.INT_EXACT)
    run_free(B, ctx, sc, 4, 1e-10, what=f"radix5-{N}")


def test_radix5_rk4_2d(B, ctx):
    note("case: config2 recipe N=(40,50), RK4 (radix-5 FFT passes), FP64, 2 cycles")
    sc = W.config2(K=2, N=40, precision=W.FP64)
    sc.model = sc.model.with_(N=(40, 50))
    run_free(B, ctx, sc, 2, 1e-10, what="radix5-2d")


def test_fdm_rejects_non_diagonal_models(B, ctx):
    sc = W.config2(K=1, N=32)
    with pytest.raises(B.PmfError) as e:
        B.pmf_create(ctx, sc.model.with_(integrator=W.INT_FDM), sc.prior)
    assert e.value.status == B.PMF_E_INVALID
    sc3 = W.config3(K=1, N=16)
    with pytest.raises(B.PmfError) as e:
        B.pmf_create(ctx, sc3.model.with_(integrator=W.INT_FDM, A=np.diag([-0.1, -0.2, -0.3]),
                                          Q=np.eye(3)), sc3.prior)
    assert e.value.status == B.PMF_E_INVALID


def test_sine_1d_n80(B, ctx):
    note("case: config1 recipe, sine-series update, N=80, FP64, 5 cycles")
    sc = W.config1(K=5, N=80)
    sc.model = sc.model.with_(integrator=W.INT_SINE)
    run_free(B, ctx, sc, 5, 1e-10, what="sine1d-80")


def test_sine_3d(B, ctx):
    note("case: sine-series update 3-D N=(20,16,24) FP64, 2 cycles")
    run_free(B, ctx, _diag_scenario(3, (20, 16, 24), 2, integrator=W.INT_SINE), 2, 1e-10, what="sine3d")


def test_sine_2d_fp32_lockstep(B, ctx):
    note("case: sine-series update 2-D N=(48,64) FP32 lockstep, 3 cycles")
    run_lockstep(B, ctx, _diag_scenario(2, (48, 64), 3, precision=W.FP32, integrator=W.INT_SINE), 3, 1e-5,
                 what="sine2d-fp32")


def test_batch_refuses_fdm_and_sine_filters(B, ctx):
    for integ in (W.INT_FDM, W.INT_SINE):
        sc = W.config1(K=1, N=64, precision=W.FP32)
        f = B.pmf_create(ctx, sc.model.with_(integrator=integ), sc.prior)
        try:
            with pytest.raises(B.PmfError) as e:
                B.pmf_batch_step(ctx, [f], sc.T, sc.z[:1])
            assert e.value.status == B.PMF_E_INVALID
        finally:
            B.pmf_destroy(f)


@pytest.mark.parametrize("integ", ["exact", "rk4"])
def test_odd_prime_radices_2d(B, ctx, integ):
    """Radix-7 and radix-17 passes on both kinds of generic axis kernel in FP64: axis 0
    (N = 28 = 4 7: forward transform, gain and inverse transform in one launch) and
    axis 1 (N = 34 = 2 17: a separate axis pass each way), sheared grid."""
    note(f"case: config2 recipe N=(28,34), {integ} (radix-7 and radix-17 passes on both axis kernels), FP64, 2 cycles")
    sc = W.config2(K=2, N=28, precision=W.FP64)
    sc.model = sc.model.with_(N=(28, 34), integrator=W.INT_EXACT if integ == "exact" else W.INT_RK4)
    run_free(B, ctx, sc, 2, 1e-10, what=f"odd-2d-{integ}")
