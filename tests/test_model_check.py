"""Host-side model checks through the C ABI (pmf_model_check: no device used).

The library's validation of a model (the rules pmf_create applies) and its
decision whether the fused batched step takes filters of that model, checked on
the CPU: grid sizes and radix forms, the sine transform's 2(N + 1) form, the
integrator and grid-kind rules, noise covariances, and the fused forms (square
and rectangular 2-D grids, 1-D sizes, precision, integrator, measurement)."""
import dataclasses

import numpy as np
import pytest

import workloads as W


@pytest.fixture(scope="module")
def B():
    from paper_2412_07240_amd import binding
    binding.lib()
    return binding


@pytest.fixture(scope="module")
def base():
    return W.batched_workload(1, K=1)[0].model


def refused(B, m, words):
    with pytest.raises(B.PmfError) as e:
        B.pmf_model_check(m)
    assert e.value.status == B.PMF_E_INVALID
    assert words in str(e.value), str(e.value)


@pytest.mark.parametrize("N", [(4, 4), (14, 22), (26, 34), (80, 64), (256, 256), (34, 34)])
def test_valid_fourier_sizes(B, base, N):
    ok, why = B.pmf_model_check(base.with_(N=N))
    assert isinstance(ok, bool)


@pytest.mark.parametrize("N,words", [((38, 32), "2^a"), ((33, 32), "even"), ((2, 32), "4..256"),
                                     ((258, 32), "4..256")])
def test_invalid_fourier_sizes(B, base, N, words):
    refused(B, base.with_(N=N), words)


def test_sine_transform_needs_a_smooth_extension(B):
    m = W.ModelSpec(nx=1, A=np.zeros((1, 1)), Q=np.ones((1, 1)), N=(80,), integrator=W.INT_FDM,
                    **W.gaussian_noise(np.eye(1)))
    assert B.pmf_model_check(m)[0] is False            # valid (2 * 81 = 162 = 2 * 3^4), not fused
    refused(B, m.with_(N=(36,)), "2 (N + 1)")          # 2 * 37: 37 has no radix
    refused(B, m.with_(integrator=W.INT_SINE, N=(36,)), "2 (N + 1)")


def test_rules_of_grid_kinds_and_integrators(B, base):
    refused(B, base.with_(grid=W.CHEBYSHEV, integrator=W.INT_EXACT), "RK4 integrator only")
    A3 = np.diag([-0.1, -0.2, -0.3])
    A3[0, 1] = 0.1
    m3 = W.ModelSpec(nx=3, A=A3, Q=np.eye(3) * 0.3, N=(16, 16, 16), integrator=W.INT_FDM, nz=3, H=np.eye(3),
                     **W.gaussian_noise(np.eye(3) * 0.1))
    refused(B, m3, "diagonal A and D")
    assert B.pmf_model_check(m3.with_(A=np.diag([-0.1, -0.2, -0.3])))[0] is False   # valid, not fused
    refused(B, base.with_(substeps=0), "substeps")


def test_noise_covariance_must_be_positive_definite(B, base):
    bad = dataclasses.replace(base, noise_cov=np.array([[[1.0, 2.0], [2.0, 1.0]]]))
    refused(B, bad, "positive definite")


@pytest.mark.parametrize("N", [(32, 32), (48, 48), (64, 64), (96, 96), (128, 128),
                               (128, 32), (32, 128), (96, 48), (64, 128), (48, 32)])
def test_fused_2d_forms(B, base, N):
    ok, why = B.pmf_model_check(base.with_(N=N))
    assert ok and why == "", (N, why)


@pytest.mark.parametrize("N,words", [((80, 64), "fused form"), ((256, 256), "above 128"),
                                     ((16, 16), "fused form"), ((64, 40), "fused form")])
def test_not_fused_2d(B, base, N, words):
    ok, why = B.pmf_model_check(base.with_(N=N))
    assert not ok and words in why, (N, why)


def test_fused_1d_sizes_and_other_refusals(B, base):
    m1 = W.config1(K=1).model.with_(precision=W.FP32, integrator=W.INT_EXACT)
    for N in (32, 48, 64, 96, 128, 192, 256):
        assert B.pmf_model_check(m1.with_(N=(N,)))[0], N
    assert not B.pmf_model_check(m1.with_(N=(80,)))[0]
    for m, words in ((base.with_(precision=W.FP64), "FP64"),
                     (base.with_(integrator=W.INT_FDM, A=np.diag([-0.1, -0.2]), N=(64, 64)), "finite-difference"),
                     (base.with_(A=np.diag([-0.1, -0.2])), "diagonal A"),
                     (base.with_(integrator=W.INT_RK4, substeps=65), "64 substeps"),
                     (base.with_(grid=W.CHEBYSHEV, integrator=W.INT_RK4, precision=W.FP32), "Chebyshev")):
        ok, why = B.pmf_model_check(m)
        assert not ok and words in why, (words, why)
    # a nonlinear measurement and the RK4 integrator stay in the fused form
    ok, why = B.pmf_model_check(W.config2(K=1).model.with_(precision=W.FP32, N=(64, 64)))
    assert ok, why
