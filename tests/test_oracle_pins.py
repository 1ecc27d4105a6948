"""Pins of the CPU oracle to facts fixed by the paper and by mathematics.

None of these compares the oracle with itself: each checks a library routine,
a closed form (Kalman-Bucy prediction, Kalman update, heat kernel, W(T) for a
scalar and a nilpotent A), an exactness property (band-limited trigonometric
data, polynomials), an invariant (mass conservation) or the per-mode
implicit diffusion step of Sec. V.A for single Fourier modes.
"""
import math

import numpy as np
import pytest
import scipy.stats

import oracle
import workloads as W
from oracle import chebyshev as cheb
from oracle import fourier as fou
from oracle import linear as lin
from oracle import pmf


# ---------------------------------------------------------------- DFT (eq. fourtrsf)

@pytest.mark.parametrize("N", [6, 16, 48, 64])
def test_dft_matches_library_and_inverts(N):
    rng = np.random.default_rng(N)
    x = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    X = fou.dft_matrix(N) @ x
    np.testing.assert_allclose(X, np.fft.fft(x) / N, atol=1e-13)
    np.testing.assert_allclose(fou.idft_matrix(N) @ X, x, atol=1e-12)
    assert abs(np.sum(np.abs(x) ** 2) - N * np.sum(np.abs(X) ** 2)) < 1e-10   # Parseval


# ------------------------------------------------ spectral derivatives (Sec. IV)

@pytest.mark.parametrize("N", [8, 48, 64])
def test_derivatives_exact_on_sines(N):
    D1, D2 = fou.diff_matrices(N)
    u = np.arange(N, dtype=float)
    for s in range(0, N // 2):
        k = 2 * np.pi * s / N
        f = np.sin(k * u + 0.3)
        np.testing.assert_allclose(D1 @ f, k * np.cos(k * u + 0.3), atol=1e-11)
        np.testing.assert_allclose(D2 @ f, -k * k * f, atol=1e-10)
    nyq = np.cos(np.pi * u)
    np.testing.assert_allclose(D1 @ nyq, 0.0, atol=1e-11)                 # no Nyquist term in d/dx
    np.testing.assert_allclose(D2 @ nyq, -np.pi ** 2 * nyq, atol=1e-10)   # kept in d2/dx2


def test_d2_differs_from_d1_squared_by_nyquist_projection():
    N = 16
    D1, D2 = fou.diff_matrices(N)
    i = np.arange(N)
    proj = np.outer((-1.0) ** i, (-1.0) ** i) / N
    np.testing.assert_allclose(D2 - D1 @ D1, -np.pi ** 2 * proj, atol=1e-11)


def test_derivative_of_resolved_gaussian():
    N, sig = 64, 1.0
    delta = 16 * sig / N
    x = (np.arange(N) - N // 2) * delta
    f = np.exp(-0.5 * x ** 2 / sig ** 2)
    D1, D2 = fou.diff_matrices(N)
    np.testing.assert_allclose(D1 @ f / delta, -x * f, atol=1e-12)
    np.testing.assert_allclose(D2 @ f / delta ** 2, (x ** 2 - 1) * f, atol=1e-11)


def test_trig_interpolant_band_limited_and_nyquist():
    N = 32
    rng = np.random.default_rng(1)
    j = np.arange(N, dtype=float)
    a = rng.standard_normal(N // 2)
    b = rng.standard_normal(N // 2)
    c_nyq = 0.7

    def f(u):
        out = c_nyq * np.cos(np.pi * u)
        for s in range(N // 2):
            out = out + a[s] * np.cos(2 * np.pi * s * u / N) + b[s] * np.sin(2 * np.pi * s * u / N)
        return out

    u = rng.uniform(0, N - 1, size=50)
    np.testing.assert_allclose(fou.interpolation_matrix(N, u) @ f(j), f(u), atol=1e-11)
    np.testing.assert_allclose(fou.interpolation_matrix(N, j) @ f(j), f(j), atol=1e-12)


# ------------------------------------------------------- linear SDE quantities

def test_W_scalar_closed_form():
    a, d, T = -0.7, 2.0, 0.3
    got = lin.W_integral(np.array([[a]]), np.array([[d]]), T)[0, 0]
    assert abs(got - d * (1 - math.exp(-2 * a * T)) / (2 * a)) < 1e-14


def test_W_nilpotent_closed_form():
    d1, d2, T = 0.01, 0.25, 0.05
    A = np.array([[0.0, 1.0], [0.0, 0.0]])
    got = lin.W_integral(A, np.diag([d1, d2]), T)
    want = np.array([[d1 * T + d2 * T ** 3 / 3, -d2 * T ** 2 / 2],
                     [-d2 * T ** 2 / 2, d2 * T]])
    np.testing.assert_allclose(got, want, atol=1e-16, rtol=1e-12)


# ------------------------------------------- time update closed forms (Sec. II)

def _gauss_model(nx, A, D, N, integrator, substeps=1, grid=W.FOURIER, T=0.1, span=8.0):
    Q = np.linalg.cholesky(D)
    return W.ModelSpec(nx=nx, A=np.asarray(A, float), Q=Q, N=tuple(N), grid=grid,
                       integrator=integrator, substeps=substeps, t_nominal=T,
                       span_sigmas=span, meas_kind=W.H_LINEAR, nz=nx, H=np.eye(nx),
                       **W.gaussian_noise(np.eye(nx)))


def _predict_error(model, prior_mean, prior_cov, T):
    st = oracle.create(model, W.gaussian_prior(prior_mean, prior_cov))
    # the created density is the prior sampled at nodes, renormalised: compare the
    # prediction with the Gaussian it came from, pushed through the closed form
    A, D = model.A, model.D
    Phi = lin.expm(A * T)
    Wt = lin.W_integral(A, D, T)
    m1 = Phi @ prior_mean
    C1 = Phi @ (prior_cov + Wt) @ Phi.T
    st1, l = oracle.predict(model, st, T)
    X = oracle.nodes(model, st1.c, st1.M)
    want = scipy.stats.multivariate_normal(m1, C1).pdf(X.reshape(-1, model.nx)).reshape(X.shape[:-1])
    q = oracle.quadrature_weights(model, st1.M)
    return float(np.sum(q * np.abs(st1.P - want))), l, st, st1


def test_exact_predict_is_kalman_bucy_1d():
    m = _gauss_model(1, [[-0.5]], [[1.0]], (64,), W.INT_EXACT)
    err, *_ = _predict_error(m, np.array([0.3]), np.array([[0.8]]), 0.1)
    assert err < 1e-12


def test_exact_predict_is_kalman_bucy_2d_sheared():
    A = [[-0.3, 1.0], [-0.4, -0.2]]
    D = [[0.2, 0.05], [0.05, 0.3]]
    m = _gauss_model(2, A, D, (48, 64), W.INT_EXACT, T=0.2)
    err, *_ = _predict_error(m, np.array([0.5, -1.0]), np.array([[1.0, 0.3], [0.3, 0.5]]), 0.2)
    assert err < 1e-11


def test_exact_predict_is_kalman_bucy_3d():
    rng = np.random.default_rng(3)
    A = W.random_stable_A(rng, 3, -1.0, -0.1)
    B = rng.uniform(0, 0.5, (3, 3))
    D = B @ B.T + 0.05 * np.eye(3)
    m = _gauss_model(3, A, D, (40, 44, 40), W.INT_EXACT, T=0.2, span=7.0)
    err, *_ = _predict_error(m, np.zeros(3), np.diag([0.5, 0.4, 0.6]), 0.2)
    assert err < 1e-9


def test_heat_kernel_when_A_is_zero():
    D = np.array([[0.4, 0.1], [0.1, 0.3]])
    m = _gauss_model(2, np.zeros((2, 2)), D, (40, 40), W.INT_EXACT, T=0.5)
    err, _, st0, st1 = _predict_error(m, np.array([1.0, 2.0]), np.eye(2), 0.5)
    assert err < 1e-11
    np.testing.assert_allclose(st1.M, st0.M)           # the grid does not move
    mm, C = oracle.moments(m, st1)
    np.testing.assert_allclose(C, np.eye(2) + D * 0.5, atol=1e-11)


def test_rk4_is_fourth_order_and_euler_first_order():
    A = [[-0.5, 0.4], [0.0, -0.3]]
    D = [[0.3, 0.1], [0.1, 0.2]]
    errs = {}
    for integ, ls in ((W.INT_RK4, (4, 8)), (W.INT_EULER, (8, 16))):
        for l in ls:
            m = _gauss_model(2, A, D, (48, 48), integ, substeps=l, T=0.5, span=8.0)
            err, used, *_ = _predict_error(m, np.zeros(2), 4.0 * np.eye(2), 0.5)
            assert used == l
            errs[(integ, l)] = err
    r4 = errs[(W.INT_RK4, 4)] / errs[(W.INT_RK4, 8)]
    r1 = errs[(W.INT_EULER, 8)] / errs[(W.INT_EULER, 16)]
    assert 12.0 < r4 < 20.0, r4
    assert 1.7 < r1 < 2.3, r1


def test_rk4_substep_clamp_keeps_it_stable():
    m = _gauss_model(1, [[-0.5]], [[1.0]], (64,), W.INT_RK4, substeps=1, T=0.1)
    err, l, *_ = _predict_error(m, np.array([0.0]), np.array([[0.01]]), 0.1)
    assert l > 1 and err < 1e-6


@pytest.mark.parametrize("integ", [W.INT_EXACT, W.INT_RK4, W.INT_EULER])
def test_mass_is_conserved_on_the_moving_grid(integ):
    rng = np.random.default_rng(7)
    A = np.array([[-0.8, 0.5], [-0.2, 0.3]])                 # nonzero trace
    m = _gauss_model(2, A, [[0.2, 0.0], [0.0, 0.1]], (32, 48), integ, substeps=3, T=0.3)
    st = oracle.create(m, W.PriorSpec(np.array([0.3, 0.7]), rng.standard_normal((2, 2)),
                                      np.array([np.eye(2) * 0.5, np.diag([0.3, 0.8])])))
    st.P = st.P * (1.0 + 0.1 * np.sin(np.arange(st.P.size).reshape(st.P.shape)))
    mass0 = float(np.sum(oracle.quadrature_weights(m, st.M) * st.P))
    st1, _ = oracle.predict(m, st, 0.3)
    mass1 = float(np.sum(oracle.quadrature_weights(m, st1.M) * st1.P))
    assert abs(mass1 - mass0) < 1e-13 * mass0


def _euler_mode_gain(kappa2, deltas, A_diag, D_diag, T, l, factors=None):
    """Implicit diffusion step of Sec. V.A for one Fourier mode of an axis-aligned
    grid with diagonal A and D: the step at t_n divides the mode by
    1 + h/2 sum_a D_aa kappa_a^2 / delta_a(t_n)^2, where the grid step moves as
    delta_a(t) = delta_a e^{A_aa t} (x' = A x); l factors at t_n = n h."""
    h = T / l
    g = 1.0
    for n in range(l if factors is None else factors):
        sig = sum(D_diag[a] * kappa2[a] / (deltas[a] * math.exp(A_diag[a] * n * h)) ** 2
                  for a in range(len(deltas)))
        g /= 1.0 + 0.5 * h * sig
    return g


def _euler_case(l=7, factors=None):
    A = np.diag([-0.4, -0.9])
    D = np.diag([0.3, 0.6])
    N = (32, 48)
    m = _gauss_model(2, A, D, N, W.INT_EULER, substeps=l, T=0.4, span=6.0)
    st = oracle.create(m, W.gaussian_prior([0.5, -0.5], np.diag([0.4, 0.3])))
    j0, j1 = np.meshgrid(np.arange(N[0]), np.arange(N[1]), indexing="ij")
    k0, k1 = 2 * np.pi * 3 / N[0], 2 * np.pi * 5 / N[1]
    # the mean, one oblique mode and the Nyquist mode of axis 0 (symbol pi^2 kept)
    st.P = 1.0 + 0.3 * np.cos(k0 * j0 + 0.4) * np.cos(k1 * j1) + 0.1 * np.cos(np.pi * j0)
    st1, used = oracle.predict(m, st, 0.4)
    deltas = np.diag(st.M)
    g1 = _euler_mode_gain((k0 ** 2, k1 ** 2), deltas, np.diag(A), np.diag(D), 0.4, l, factors)
    gn = _euler_mode_gain((np.pi ** 2, 0.0), deltas, np.diag(A), np.diag(D), 0.4, l, factors)
    want = math.exp(-np.trace(A) * 0.4) * (
        1.0 + 0.3 * g1 * np.cos(k0 * j0 + 0.4) * np.cos(k1 * j1) + 0.1 * gn * np.cos(np.pi * j0))
    return st1.P, want, used


def test_oracle_euler_is_the_per_mode_implicit_step():
    got, want, used = _euler_case()
    assert used == 7
    np.testing.assert_allclose(got, want, atol=1e-13, rtol=1e-12)


def test_euler_pin_tells_the_product_endpoints_apart():
    """The pin separates the reading of l factors at t_0..t_{l-1} from one with
    l + 1 factors (the product endpoints are ambiguous in the paper)."""
    got, want_more, _ = _euler_case(factors=8)
    assert np.max(np.abs(got - want_more)) > 1e-4


# ---------------------------------------------------- measurement update (Sec. I.A)

def test_update_is_kalman_update_2d():
    A = np.array([[-0.2, 0.7], [-0.3, -0.1]])
    D = np.array([[0.3, 0.0], [0.0, 0.2]])
    m = _gauss_model(2, A, D, (64, 64), W.INT_EXACT, T=0.1)
    Hm = np.array([[1.0, 0.5]])
    R = np.array([[0.5]])
    m = m.with_(H=Hm, nz=1, **W.gaussian_noise(R))
    pm, pc = np.array([0.2, -0.1]), np.array([[1.0, 0.2], [0.2, 0.6]])
    st = oracle.create(m, W.gaussian_prior(pm, pc))
    st, _ = oracle.predict(m, st, 0.1)
    Phi = lin.expm(A * 0.1)
    mk = Phi @ pm
    Pk = Phi @ (pc + lin.W_integral(A, D, 0.1)) @ Phi.T
    z = np.array([0.7])
    X = oracle.nodes(m, st.c, st.M)
    st2, ll, status, mp, Cp = oracle.update(m, st, z)
    S = Hm @ Pk @ Hm.T + R
    K = Pk @ Hm.T @ np.linalg.inv(S)
    m_kf = mk + K @ (z - Hm @ mk)
    P_kf = Pk - K @ S @ K.T
    ll_kf = scipy.stats.multivariate_normal(Hm @ mk, S).logpdf(z)
    assert status == 0
    np.testing.assert_allclose(mp, m_kf, atol=1e-11)
    np.testing.assert_allclose(Cp, P_kf, atol=1e-11)
    assert abs(ll - ll_kf) < 1e-11
    # the re-gridded density is the Kalman posterior on the new grid (cubic
    # Lagrange: the old grid is sheared, so only interpolation accuracy)
    X2 = oracle.nodes(m, st2.c, st2.M)
    want = scipy.stats.multivariate_normal(m_kf, P_kf).pdf(X2.reshape(-1, 2)).reshape(X2.shape[:-1])
    q2 = oracle.quadrature_weights(m, st2.M)
    assert np.sum(q2 * np.abs(st2.P - want)) < 5e-3


def test_update_1d_trig_regrid_is_exact_kalman():
    m = _gauss_model(1, [[-0.5]], [[1.0]], (128,), W.INT_EXACT, T=0.1)
    m = m.with_(**W.gaussian_noise([[0.3]]))
    st = oracle.create(m, W.gaussian_prior([0.0], [[1.0]]))
    st, _ = oracle.predict(m, st, 0.1)
    mom_m, mom_C = oracle.moments(m, st)
    st2, ll, status, mp, Cp = oracle.update(m, st, np.array([0.4]))
    S = mom_C + 0.3
    m_kf = mom_m + mom_C / S * (0.4 - mom_m)
    P_kf = mom_C - mom_C ** 2 / S
    X2 = oracle.nodes(m, st2.c, st2.M)
    want = scipy.stats.norm(m_kf[0], math.sqrt(P_kf[0, 0])).pdf(X2[..., 0])
    assert np.sum(abs(np.linalg.det(st2.M)) * np.abs(st2.P - want)) < 1e-9


def test_gaussian_mixture_noise_likelihood():
    m = _gauss_model(1, [[-0.5]], [[1.0]], (16,), W.INT_EXACT)
    m = m.with_(**W.gm_measurement_noise())
    X = np.linspace(-5, 25, 16)[:, None]
    z = np.array([12.0])
    got = oracle.loglik_field(m, X, z)
    r = z[0] - X[:, 0]
    want = np.log(0.5 * scipy.stats.norm(0, 1).pdf(r) + 0.5 * scipy.stats.norm(20, 1).pdf(r))
    np.testing.assert_allclose(got, want, rtol=1e-12)


def test_nonlinear_measurement_functions():
    X = np.array([[1.5, -2.0, 0.5], [0.1, 0.2, -0.3]])
    m = _gauss_model(3, -np.eye(3), np.eye(3), (4, 4, 4), W.INT_EXACT)
    mn = m.with_(meas_kind=W.H_NORM, nz=1, **W.gaussian_noise([[0.01]]))
    np.testing.assert_allclose(pmf.measurement(mn, X)[:, 0], [math.sqrt(6.5), math.sqrt(0.14)])
    mc = m.with_(meas_kind=W.H_CUBIC1, nz=1, hparam=np.array([1.0, 0.05, 0, 0]),
                 **W.gaussian_noise([[0.04]]))
    np.testing.assert_allclose(pmf.measurement(mc, X)[:, 0], [1.5 + 0.05 * 3.375, 0.1 + 0.05e-3])


def test_degenerate_update_leaves_state():
    m = _gauss_model(1, [[-0.5]], [[1.0]], (32,), W.INT_EXACT)
    m = m.with_(**W.gaussian_noise([[1e-6]]))
    st = oracle.create(m, W.gaussian_prior([0.0], [[1.0]]))
    st.P[16:] = 0.0                                    # no mass on the right half
    X = oracle.nodes(m, st.c, st.M)
    z = np.array([X[24, 0]])                           # likelihood peaks there
    st2, ll, status, _, _ = oracle.update(m, st, z)
    assert status == pmf.STATUS_DEGENERATE and st2 is st


def test_boundary_flag():
    m = _gauss_model(1, [[-0.5]], [[1.0]], (32,), W.INT_EXACT)
    m = m.with_(**W.gaussian_noise([[1.0]]))
    st = oracle.create(m, W.gaussian_prior([0.0], [[1.0]]))
    X = oracle.nodes(m, st.c, st.M)
    _, _, status, _, _ = oracle.update(m, st, np.array([X[0, 0] - 3.0]))
    assert status & pmf.STATUS_BOUNDARY


# ------------------------------------------------------------- grid design

def test_design_grid_hand_values():
    m = _gauss_model(1, [[-0.5]], [[1.0]], (64,), W.INT_EXACT, T=0.1)
    c, M = oracle.design_grid(m, np.array([1.5]), np.array([[0.04]]))
    S = 0.04 + (math.exp(0.1) - 1.0)         # int_0^0.1 e^{s} ds for A = -1/2, D = 1
    assert c[0] == 1.5
    assert abs(M[0, 0] - 2 * 8 * math.sqrt(S) / 64) < 1e-15


# ----------------------------------------------------------- re-interpolation

def test_lagrange3_is_exact_on_cubics_and_zero_outside():
    A = np.array([[-0.3, 1.0], [0.0, -0.1]])
    m = _gauss_model(2, A, np.eye(2) * 0.1, (32, 40), W.INT_EXACT, T=0.1)
    c_old = np.array([0.1, -0.2])
    M_old = np.array([[0.2, 0.05], [-0.03, 0.15]])
    X = oracle.nodes(m, c_old, M_old)
    U = (X - c_old) @ np.linalg.inv(M_old).T + np.array([16, 20])

    def poly(u):
        return 1 + 0.3 * u[..., 0] - 0.02 * u[..., 1] ** 2 + 1e-3 * u[..., 0] ** 2 * u[..., 1] \
            + 2e-4 * u[..., 1] ** 3

    st = pmf.State(c_old, M_old, 0.0, poly(U))
    c_new, M_new = np.array([0.0, 0.1]), np.diag([0.25, 0.2])
    out = oracle.interpolate(m, st, c_new, M_new)
    Xn = oracle.nodes(m, c_new, M_new)
    Un = (Xn - c_old) @ np.linalg.inv(M_old).T + np.array([16, 20])
    inner = np.all((Un >= 1) & (Un <= np.array([30, 38])), axis=-1)
    outside = np.any((Un < 0) | (Un > np.array([31, 39])), axis=-1)
    assert inner.sum() > 100 and outside.sum() > 100
    np.testing.assert_allclose(out[inner], poly(Un[inner]), atol=1e-11)
    assert np.all(out[outside] == 0.0)


def test_trig_separable_regrid_exact_for_band_limited():
    m = _gauss_model(2, -np.eye(2), np.eye(2), (32, 16), W.INT_EXACT)
    c_old, M_old = np.array([0.0, 0.0]), np.diag([0.1, 0.2])
    X = oracle.nodes(m, c_old, M_old)
    U = (X - c_old) / np.diag(M_old) + np.array([16, 8])

    def f(u):
        return np.cos(2 * np.pi * 3 * u[..., 0] / 32 + 0.2) * np.sin(2 * np.pi * 5 * u[..., 1] / 16 + 1.0) + 0.5

    st = pmf.State(c_old, M_old, 0.0, f(U))
    c_new, M_new = np.array([0.05, -0.1]), np.diag([0.08, 0.17])
    out = oracle.interpolate(m, st, c_new, M_new)
    Xn = oracle.nodes(m, c_new, M_new)
    Un = (Xn - c_old) / np.diag(M_old) + np.array([16, 8])
    inside = np.all((Un >= 0) & (Un <= np.array([31, 15])), axis=-1)
    np.testing.assert_allclose(out[inside], f(Un[inside]), atol=1e-12)
    assert np.all(out[~inside] == 0.0)


# ------------------------------------------------------------- Chebyshev

@pytest.mark.parametrize("N", [8, 17, 32])
def test_chebyshev_derivatives_exact_on_polynomials(N):
    u = cheb.interior_nodes(N)
    D1, D2 = cheb.diff_matrices(N)
    rng = np.random.default_rng(N)
    coef = rng.standard_normal(N)                  # p = (1 - u^2) * q, deg q = N-1
    q = np.polynomial.Polynomial(coef)
    p = np.polynomial.Polynomial([1, 0, -1]) * q    # degree N+1, zero at +-1
    np.testing.assert_allclose(D1 @ p(u), p.deriv(1)(u), rtol=1e-8, atol=1e-8 * np.abs(p(u)).max())
    np.testing.assert_allclose(D2 @ p(u), p.deriv(2)(u), rtol=1e-7,
                               atol=1e-7 * np.abs(p.deriv(2)(u)).max())


@pytest.mark.parametrize("N", [6, 31, 64])
def test_clenshaw_curtis_integrates_polynomials(N):
    v = cheb.cgl_nodes(N)
    w = cheb.cc_weights(N)
    for k in range(0, N + 2):
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert abs(np.dot(w, v ** k) - exact) < 1e-12
    assert np.all(w > 0)


def test_chebyshev_interpolation_exact_on_polynomials():
    N = 12
    u = cheb.interior_nodes(N)
    p = np.polynomial.Polynomial([1, 0, -1]) * np.polynomial.Polynomial([0.3, -1, 0.5, 2.0])
    x = np.linspace(-1.2, 1.2, 37)
    Wm = cheb.poly_interp_matrix(N, x)
    want = np.where(np.abs(x) <= 1, p(x), 0.0)
    np.testing.assert_allclose(Wm @ p(u), want, atol=1e-12)


def test_chebyshev_d2_radius_grows_like_N4():
    r = [cheb.d2_spectral_radius(n) for n in (16, 32, 64)]
    assert 12 < r[1] / r[0] < 17 and 13 < r[2] / r[1] < 17


def test_chebyshev_predict_gaussian_closed_form():
    A = [[-0.4, 0.3], [-0.1, -0.6]]
    D = [[0.2, 0.05], [0.05, 0.15]]
    m = _gauss_model(2, A, D, (64, 64), W.INT_RK4, grid=W.CHEBYSHEV, T=0.1)
    err, l, *_ = _predict_error(m, np.array([0.2, 0.1]), np.array([[0.5, 0.1], [0.1, 0.4]]), 0.1)
    assert err < 1e-9, (err, l)


def test_chebyshev_mass_conserved_to_quadrature_accuracy():
    A = [[-0.4, 0.3], [-0.1, -0.6]]
    m = _gauss_model(2, A, [[0.2, 0.05], [0.05, 0.15]], (64, 64), W.INT_RK4,
                     grid=W.CHEBYSHEV, T=0.1)
    st = oracle.create(m, W.gaussian_prior([0.0, 0.0], np.eye(2) * 0.5))
    st1, _ = oracle.predict(m, st, 0.1)
    mass = float(np.sum(oracle.quadrature_weights(m, st1.M) * st1.P))
    assert abs(mass - 1.0) < 1e-10


# ------------------------------------------------------- a full linear cycle

def test_full_filter_tracks_kalman_filter():
    """Linear-Gaussian 1-D filter over 30 cycles: PMF moments = KF moments."""
    sc = W.config1(K=30)
    m = sc.model.with_(N=(128,), **W.gaussian_noise([[0.25]]))
    st = oracle.create(m, sc.prior)
    mk, Pk = sc.prior.mean[0].copy(), sc.prior.cov[0].copy()
    Phi = lin.expm(m.A * sc.T)
    Wt = lin.W_integral(m.A, m.D, sc.T)
    for k in range(30):
        st, _ = oracle.predict(m, st, sc.T)
        mk, Pk = Phi @ mk, Phi @ (Pk + Wt) @ Phi.T
        st, ll, status, mp, Cp = oracle.update(m, st, sc.z[k])
        S = Pk[0, 0] + 0.25
        Kk = Pk[0, 0] / S
        mk = mk + Kk * (sc.z[k] - mk)
        Pk = Pk - Kk * Pk
        assert status == 0
    np.testing.assert_allclose(mp, mk, atol=1e-9)
    np.testing.assert_allclose(Cp, Pk, atol=1e-9)


# ----------------------------------- planted mistakes must be caught by the pins

def test_planted_trace_sign_breaks_mass_conservation(monkeypatch):
    real_predict = pmf.predict

    def wrong(model, state, T):
        st, l = real_predict(model, state, T)
        st.P = st.P * math.exp(2 * np.trace(model.A) * T)   # as if +tr(A)
        return st, l

    monkeypatch.setattr(oracle, "predict", wrong)
    with pytest.raises(AssertionError):
        test_mass_is_conserved_on_the_moving_grid(W.INT_EXACT)


def test_planted_transposed_grid_matrix_breaks_closed_form(monkeypatch):
    real = lin.Dy

    def wrong(A, D, M0, t):
        return real(A, D, M0.T, t)

    monkeypatch.setattr(lin, "Dy", wrong)
    A = [[-0.3, 1.0], [-0.4, -0.2]]
    m = _gauss_model(2, A, [[0.2, 0.05], [0.05, 0.3]], (32, 32), W.INT_RK4, substeps=4, T=0.2)
    st = oracle.create(m, W.gaussian_prior([0.5, -1.0], [[1.0, 0.3], [0.3, 0.5]]))
    st = pmf.State(st.c, np.array([[st.M[0, 0], 0.02], [0.0, st.M[1, 1]]]), 0.0, st.P)
    # rebuild the sampled prior on the sheared grid so the closed form applies
    X = oracle.nodes(m, st.c, st.M)
    st.P = scipy.stats.multivariate_normal([0.5, -1.0], [[1.0, 0.3], [0.3, 0.5]]).pdf(X)
    st1, _ = oracle.predict(m, st, 0.2)
    Phi = lin.expm(np.array(A) * 0.2)
    C1 = Phi @ (np.array([[1.0, 0.3], [0.3, 0.5]]) + lin.W_integral(np.array(A), m.D, 0.2)) @ Phi.T
    want = scipy.stats.multivariate_normal(Phi @ [0.5, -1.0], C1).pdf(oracle.nodes(m, st1.c, st1.M))
    err = np.sum(abs(np.linalg.det(st1.M)) * np.abs(st1.P - want))
    assert err > 1e-6


def test_planted_missing_nyquist_breaks_derivative_pin(monkeypatch):
    real = fou.kappa_second

    def wrong(N):
        k = real(N).copy()
        k[N // 2] = 0.0
        return k

    monkeypatch.setattr(fou, "kappa_second", wrong)
    with pytest.raises(AssertionError):
        test_derivatives_exact_on_sines(8)
