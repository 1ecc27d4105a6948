"""Finite-difference baseline (sine-transform route of eq. FST), the sine-series
variant of the spectral update, and the radix-5 FFT sizes they are compared at
(N = 80, 200 in the convergence study), HIP path vs the FP64 oracle through the
C ABI.  Same bars as the other parity tests: L1 <=
1e-10 (FP64), <= 1e-5 per cycle in lockstep (FP32)."""
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
    note("case: finite differences 2-D N=(48,40) FP64, 3 cycles")
    run_free(B, ctx, _diag_scenario(2, (48, 40), 3), 3, 1e-10, what="fdm2d")


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
