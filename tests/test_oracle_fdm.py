"""Pins of the oracle's finite-difference baseline (eqs. FDM, fdiff, FST) and of
the spectral-vs-FDM convergence behaviour the comparison rests on.

* the oracle's general explicit step reduces, in 1-D, to the paper's tridiagonal
  step matrix with its a_t, b_t (eq. fdiff);
* l explicit steps equal the sine-transform route of eq. FST, with the Toeplitz
  eigenvalues b_t + 2 a_t cos(j pi / (N + 1)) and the DST-I of scipy as the
  transform (a library routine);
* against the heat kernel (A = 0, Gaussian and Gaussian-mixture densities) the
  scheme converges at second order in the grid step, the spectral exact
  integrator far faster.
"""
import math

import numpy as np
import pytest
import scipy.fft

import oracle
import workloads as W
from oracle import pmf


def _model_1d(a, q, N, l_min=1):
    return W.ModelSpec(nx=1, A=np.array([[a]]), Q=np.array([[q]]), N=(N,), t_nominal=0.1,
                       integrator=W.INT_FDM, substeps=l_min, precision=W.FP64,
                       meas_kind=W.H_LINEAR, nz=1, H=np.array([[1.0]]), **W.gaussian_noise([[0.01]]))


def _state_1d(N, delta, c=0.0, seed=0):
    rng = np.random.default_rng(seed)
    P = rng.uniform(0.0, 1.0, size=N)
    return oracle.State(np.array([c]), np.array([[delta]]), 0.0, P)


def test_one_step_is_the_tridiagonal_matrix_of_eq_fdiff():
    a, q, N, delta, T = -0.4, 0.7, 24, 0.15, 0.004
    m = _model_1d(a, q, N)
    st = _state_1d(N, delta)
    assert oracle.substeps(m, st, T) == 1          # T (q^2 / delta^2) < 1
    out, l = oracle.predict(m, st, T)
    assert l == 1
    a_t = q * q * T / (2.0 * delta ** 2)           # Q of the paper = diffusion = q^2 (reading R1)
    b_t = 1.0 - q * q * T / delta ** 2 - T * a
    F = pmf.fdm_step_matrix(N, a_t, b_t)
    np.testing.assert_allclose(out.P, F @ st.P, rtol=0, atol=1e-14)
    # the grid moves with x' = A x
    np.testing.assert_allclose(out.M, [[delta * math.exp(a * T)]], rtol=1e-14)


def _eigen(N, a_t, b_t):
    j = np.arange(1, N + 1)
    return b_t + 2.0 * a_t * np.cos(j * np.pi / (N + 1))


@pytest.mark.parametrize("N,l_min", [(16, 5), (40, 12), (63, 3)])
def test_l_steps_equal_the_sine_transform_route_1d(N, l_min):
    a, q, delta, T = -0.8, 0.5, 0.1, 0.05
    m = _model_1d(a, q, N, l_min)
    st = _state_1d(N, delta, seed=N)
    out, l = oracle.predict(m, st, T)
    assert l >= l_min
    h = T / l
    lam = np.ones(N)
    for n in range(l):
        dn = delta * math.exp(a * n * h)            # grid step at t_n (eq. gridMov)
        a_t = q * q * h / (2.0 * dn ** 2)
        b_t = 1.0 - q * q * h / dn ** 2 - h * a
        lam *= _eigen(N, a_t, b_t)
    # scipy's DST-I: y_k = 2 sum_n x_n sin(pi (k+1)(n+1) / (N+1)); R^-1 = 2/(N+1) R
    ref = scipy.fft.dst(lam * scipy.fft.dst(st.P, type=1), type=1) / (2.0 * (N + 1))
    np.testing.assert_allclose(out.P, ref, rtol=0, atol=1e-12 * np.abs(ref).max())


def test_l_steps_equal_the_sine_transform_route_2d():
    A = np.diag([-0.5, -1.2])
    Q = np.diag([0.6, 0.3])
    N = (20, 30)
    m = W.ModelSpec(nx=2, A=A, Q=Q, N=N, t_nominal=0.1, integrator=W.INT_FDM, substeps=4,
                    precision=W.FP64, meas_kind=W.H_LINEAR, nz=2, H=np.eye(2),
                    **W.gaussian_noise(0.01 * np.eye(2)))
    rng = np.random.default_rng(5)
    d0 = np.array([0.12, 0.07])
    st = oracle.State(np.zeros(2), np.diag(d0), 0.0, rng.uniform(0, 1, size=N))
    T = 0.03
    out, l = oracle.predict(m, st, T)
    h = T / l
    th = [np.arange(1, n + 1) * np.pi / (n + 1) for n in N]
    lam = np.ones(N)
    D = Q @ Q.T
    for n in range(l):
        dn = d0 * np.exp(np.diag(A) * n * h)
        Dy = np.diag(D) / dn ** 2
        lam *= (1.0 - h * np.trace(A) + h * Dy[0] * (np.cos(th[0])[:, None] - 1.0)
                + h * Dy[1] * (np.cos(th[1])[None, :] - 1.0))
    ref = scipy.fft.dstn(lam * scipy.fft.dstn(st.P, type=1), type=1) / (4.0 * (N[0] + 1) * (N[1] + 1))
    np.testing.assert_allclose(out.P, ref, rtol=0, atol=1e-12 * np.abs(ref).max())


def test_non_diagonal_model_is_rejected():
    m = _model_1d(-0.4, 0.7, 16).with_(nx=2, A=np.array([[-0.4, 0.2], [0.0, -0.3]]), Q=np.eye(2), N=(16, 16),
                                         nz=2, H=np.eye(2), **W.gaussian_noise(0.01 * np.eye(2)))
    st = oracle.State(np.zeros(2), np.eye(2) * 0.1, 0.0, np.ones((16, 16)))
    with pytest.raises(ValueError):
        oracle.predict(m, st, 0.01)


def _heat_case(N, integ, mixture, span=10.0, T=0.05, l_min=1):
    """A = 0, D = 1: p(T) is the initial density convolved with N(0, T)."""
    if mixture:
        w = np.array([0.3, 0.4, 0.3])
        mu = np.array([-1.2, 0.3, 1.5])
        var = np.array([0.15, 0.1, 0.2])
    else:
        w, mu, var = np.array([1.0]), np.array([0.0]), np.array([0.3])
    delta = 2.0 * span / N
    m = W.ModelSpec(nx=1, A=np.zeros((1, 1)), Q=np.ones((1, 1)), N=(N,), t_nominal=T, integrator=integ,
                    substeps=l_min, precision=W.FP64, meas_kind=W.H_LINEAR, nz=1, H=np.ones((1, 1)),
                    **W.gaussian_noise([[0.01]]))
    x = (np.arange(N) - N // 2) * delta

    def gm(x, extra):
        v = var + extra
        return np.sum(w * np.exp(-0.5 * (x[:, None] - mu) ** 2 / v) / np.sqrt(2 * np.pi * v), axis=1)

    st = oracle.State(np.zeros(1), np.array([[delta]]), 0.0, gm(x, 0.0))
    out, l = oracle.predict(m, st, T)
    return float(np.max(np.abs(out.P - gm(x, T)))), l


@pytest.mark.parametrize("mixture", [False, True])
def test_fdm_converges_at_second_order(mixture):
    # h D / delta^2 = 1/4 at every N (delta = 8 / N, T = 1/16, l = N^2 / 256), so
    # the explicit scheme's error is C delta^2 with one C: halving delta quarters it
    errs = []
    for N in (64, 128, 256):
        e, l = _heat_case(N, W.INT_FDM, mixture, span=4.0, T=1.0 / 16, l_min=N * N // 256)
        assert l == N * N // 256
        errs.append(e)
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.7 < r1 < 4.3 and 3.85 < r2 < 4.15, (errs, r1, r2)


def test_spectral_exact_integrator_outruns_fdm():
    for mixture in (False, True):
        e_sd, _ = _heat_case(64, W.INT_EXACT, mixture, span=6.0)
        e_fd, _ = _heat_case(64, W.INT_FDM, mixture, span=6.0)
        assert e_sd < 1e-8 and e_fd > 1e-4, (mixture, e_sd, e_fd)


# ------------------------------------------------ sine-series variant of the spectral update

def _sine_model(A, Q, N):
    nx = len(N)
    return W.ModelSpec(nx=nx, A=A, Q=Q, N=N, t_nominal=0.1, integrator=W.INT_SINE, substeps=1,
                       precision=W.FP64, meas_kind=W.H_LINEAR, nz=nx, H=np.eye(nx),
                       **W.gaussian_noise(0.01 * np.eye(nx)))


def test_sine_modes_decay_exactly():
    # a product of sine modes is an eigenfunction: it decays by exp(-1/2 sum_a Wy_aa k_a^2)
    # times e^{-tr(A) T}, with W(T)_aa = D_aa (1 - e^{-2 a T}) / (2 a) for diagonal A
    A = np.diag([-0.7, -0.2])
    Q = np.diag([0.9, 0.4])
    N = (24, 18)
    d0 = np.array([0.2, 0.3])
    T = 0.07
    l0, l1 = 5, 11
    i0, i1 = np.arange(1, N[0] + 1), np.arange(1, N[1] + 1)
    P = np.outer(np.sin(i0 * l0 * np.pi / (N[0] + 1)), np.sin(i1 * l1 * np.pi / (N[1] + 1)))
    st = oracle.State(np.zeros(2), np.diag(d0), 0.0, P)
    out, _ = oracle.predict(_sine_model(A, Q, N), st, T)
    a = np.diag(A)
    Wd = np.diag(Q) ** 2 * (1.0 - np.exp(-2.0 * a * T)) / (2.0 * a)
    Wy = Wd / d0 ** 2
    k = np.array([l0 * np.pi / (N[0] + 1), l1 * np.pi / (N[1] + 1)])
    g = math.exp(-np.trace(A) * T) * math.exp(-0.5 * float(np.sum(Wy * k ** 2)))
    np.testing.assert_allclose(out.P, g * P, rtol=0, atol=1e-13)


def test_sine_variant_equals_library_dst_route():
    A = np.diag([-0.3])
    Q = np.diag([0.8])
    N = (37,)
    rng = np.random.default_rng(9)
    P = rng.uniform(0, 1, size=N)
    d0 = 0.11
    T = 0.02
    out, _ = oracle.predict(_sine_model(A, Q, N), oracle.State(np.zeros(1), np.array([[d0]]), 0.0, P), T)
    Wy = 0.64 * (1.0 - math.exp(0.6 * T)) / (-0.6) / d0 ** 2
    k = np.arange(1, N[0] + 1) * np.pi / (N[0] + 1)
    g = math.exp(0.3 * T) * np.exp(-0.5 * Wy * k ** 2)
    ref = scipy.fft.dst(g * scipy.fft.dst(P, type=1), type=1) / (2.0 * (N[0] + 1))
    np.testing.assert_allclose(out.P, ref, rtol=0, atol=1e-13)


def test_sine_variant_matches_heat_kernel_on_a_wide_grid():
    # a Gaussian negligible at the grid ends: the Dirichlet problem and the free one
    # coincide to rounding, and the sine series resolves it spectrally
    errs = [_heat_case(N, W.INT_SINE, True, span=8.0)[0] for N in (48, 64, 80, 128)]
    assert errs[0] > errs[1] * 50 > errs[2] * 50 ** 2     # geometric, not algebraic
    assert errs[3] < 1e-13, errs
