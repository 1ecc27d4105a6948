"""Pins of the oracle's re-interpolation, prior moments and boundary share.

Each expected value comes from a route other than the oracle's own code:

* the error formula of polynomial interpolation: for a quartic f with leading
  coefficient 1, the cubic interpolant through nodes x_0..x_3 equals
  f(u) - prod_i (u - x_i), so the value pins which four nodes the stencil takes;
* exactness of cubic interpolation on cubics that vanish where the grid's zero
  boundary values sit (the Chebyshev end points +-1);
* the Kalman update (Sec. I.A, eq. filt with linear h) on a sheared Chebyshev grid;
* hand values for Gaussian-mixture moments and the boundary share.

Planted mistakes at the end show that each pin fails on a plausible error.
"""
import math

import numpy as np
import pytest
import scipy.stats

import oracle
import workloads as W
from oracle import chebyshev as cheb
from oracle import linear as lin
from oracle import pmf


def _model(nx, N, grid=W.FOURIER, interp=W.INTERP_AUTO, A=None, D=None, integrator=W.INT_EXACT,
           T=0.1, span=8.0):
    A = -np.eye(nx) if A is None else np.asarray(A, float)
    D = np.eye(nx) * 0.2 if D is None else np.asarray(D, float)
    return W.ModelSpec(nx=nx, A=A, Q=np.linalg.cholesky(D), N=tuple(N), grid=grid, interp=interp,
                       integrator=integrator, substeps=1, t_nominal=T, span_sigmas=span,
                       meas_kind=W.H_LINEAR, nz=nx, H=np.eye(nx), **W.gaussian_noise(np.eye(nx)))


def _stencil_by_blocks(nodes, u):
    """The four consecutive nodes whose middle interval holds u; the first or the
    last four where no such block exists (u in the first or last interval)."""
    blocks = [nodes[i:i + 4] for i in range(len(nodes) - 3)]
    for b in blocks:
        if b[1] <= u < b[2]:
            return b
    return blocks[0] if u < blocks[0][2] else blocks[-1]


def _omega(nodes, u):
    return float(np.prod([u - x for x in _stencil_by_blocks(nodes, u)]))


def _old_coords(model, c_old, M_old, c_new, M_new):
    Xn = oracle.nodes(model, c_new, M_new)
    U = (Xn - c_old) @ np.linalg.inv(M_old).T
    if model.grid == W.FOURIER:
        U = U + np.array([n // 2 for n in model.N], float)
    return U


# ------------------------------------------------------------ Fourier stencil

def test_fourier_lagrange_error_formula_pins_the_stencil():
    """f(u) = (u + 1)(u - N)(u - 3)(u - 7) along each index axis vanishes at the two
    zero taps -1 and N, so the tensor cubic interpolant of f0(u0) f1(u1) is
    (f0 - w0)(f1 - w1), w the node product of each axis's stencil."""
    N = (24, 20)
    m = _model(2, N)
    c_old, M_old = np.array([0.1, -0.2]), np.array([[0.2, 0.05], [-0.03, 0.15]])
    U_old = _old_coords(m, c_old, M_old, c_old, M_old)

    def f(u, n):
        return (u + 1) * (u - n) * (u - 3) * (u - 7)

    P = f(U_old[..., 0], N[0]) * f(U_old[..., 1], N[1])
    st = pmf.State(c_old, M_old, 0.0, P)
    c_new, M_new = np.array([0.05, 0.1]), np.diag([0.22, 0.16])
    out = oracle.interpolate(m, st, c_new, M_new)
    U = _old_coords(m, c_old, M_old, c_new, M_new)
    idx_nodes = [np.arange(-1, n + 1, dtype=float) for n in N]   # the zero taps included
    checked = 0
    for p in np.ndindex(*N):
        u0, u1 = U[p]
        if not (0.0 <= u0 <= N[0] - 1 and 0.0 <= u1 <= N[1] - 1):
            assert out[p] == 0.0
            continue
        want = (f(u0, N[0]) - _omega(idx_nodes[0], u0)) * (f(u1, N[1]) - _omega(idx_nodes[1], u1))
        assert abs(out[p] - want) <= 1e-9 * max(1.0, abs(want)), (p, out[p], want)
        checked += 1
    assert checked > 200


# ---------------------------------------------------------- Chebyshev stencil

def _cheb_sheared_case(N, sub=0.0):
    m = _model(2, N, grid=W.CHEBYSHEV)
    c_old = np.array([0.05, -0.1])
    M_old = np.array([[1.0, 0.12], [-0.08, 0.9]])
    c_new, M_new = np.array([0.02, 0.03]), np.diag([1.08, 0.97])
    return m, c_old, M_old, c_new, M_new


def test_chebyshev_lagrange_exact_on_cubics_vanishing_at_the_ends():
    """p(u) = (1 - u0^2)(0.3 + u0) (1 - u1^2)(1 - 0.4 u1) is cubic in each variable
    and zero at the end points, where the taps are zero: the interpolant is p
    itself inside [-1, 1]^2 (stencils touching the ends included), zero outside."""
    N = (14, 17)
    m, c_old, M_old, c_new, M_new = _cheb_sheared_case(N)

    def p(u):
        return (1 - u[..., 0] ** 2) * (0.3 + u[..., 0]) * (1 - u[..., 1] ** 2) * (1 - 0.4 * u[..., 1])

    st = pmf.State(c_old, M_old, 0.0, p(_old_coords(m, c_old, M_old, c_old, M_old)))
    out = oracle.interpolate(m, st, c_new, M_new)
    U = _old_coords(m, c_old, M_old, c_new, M_new)
    inside = np.all(np.abs(U) <= 1.0, axis=-1)
    v = cheb.cgl_nodes(N[0])
    near_end = inside & ((U[..., 0] < v[2]) | (U[..., 0] > v[-3]))
    assert inside.sum() > 100 and (~inside).sum() > 10 and near_end.sum() > 5
    np.testing.assert_allclose(out[inside], p(U[inside]), atol=1e-13)
    assert np.all(out[~inside] == 0.0)


@pytest.mark.parametrize("N", [(12, 9), (33, 16)])
def test_chebyshev_lagrange_error_formula_pins_the_stencil(N):
    """f(u) = u^4 - 1 vanishes at the end points: on each axis the interpolant is
    f - w with w the node product of the stencil (two Chebyshev-Gauss-Lobatto
    nodes on either side, the first or last four at the ends)."""
    m, c_old, M_old, c_new, M_new = _cheb_sheared_case(N)
    Uo = _old_coords(m, c_old, M_old, c_old, M_old)
    st = pmf.State(c_old, M_old, 0.0, (Uo[..., 0] ** 4 - 1) * (Uo[..., 1] ** 4 - 1))
    out = oracle.interpolate(m, st, c_new, M_new)
    U = _old_coords(m, c_old, M_old, c_new, M_new)
    v = [cheb.cgl_nodes(n) for n in N]
    checked = 0
    for p in np.ndindex(*N):
        u0, u1 = U[p]
        if abs(u0) > 1.0 or abs(u1) > 1.0:
            assert out[p] == 0.0
            continue
        want = (u0 ** 4 - 1 - _omega(v[0], u0)) * (u1 ** 4 - 1 - _omega(v[1], u1))
        assert abs(out[p] - want) <= 1e-12, (p, out[p], want)
        checked += 1
    assert checked > 50


def test_chebyshev_1d_lagrange_mode_error_formula():
    """1-D with Lagrange forced: the same error formula along the single axis."""
    N = 21
    m = _model(1, (N,), grid=W.CHEBYSHEV, interp=W.INTERP_LAGRANGE)
    c_old, M_old = np.array([0.0]), np.array([[1.0]])
    u_old = cheb.interior_nodes(N)
    st = pmf.State(c_old, M_old, 0.0, u_old ** 4 - 1)
    c_new, M_new = np.array([0.07]), np.array([[0.95]])
    out = oracle.interpolate(m, st, c_new, M_new)
    U = (c_new + M_new[0, 0] * u_old - c_old) / M_old[0, 0]
    v = cheb.cgl_nodes(N)
    for i, u in enumerate(U):
        want = (u ** 4 - 1 - _omega(v, u)) if abs(u) <= 1 else 0.0
        assert abs(out[i] - want) <= 1e-13, (i, out[i], want)


# ---------------------------------------- Kalman update on a sheared Chebyshev grid

def test_chebyshev_update_is_kalman_on_a_sheared_grid():
    """Linear-Gaussian model on a Chebyshev grid: after a time update with a
    non-diagonal A (the grid is sheared) the measurement update reproduces the
    Kalman mean, covariance and log-likelihood (Sec. I.A), and the re-gridded
    density is the Kalman posterior up to cubic-interpolation accuracy."""
    A = np.array([[-0.4, 0.6], [-0.3, -0.5]])
    D = np.array([[0.2, 0.04], [0.04, 0.15]])
    m = _model(2, (48, 48), grid=W.CHEBYSHEV, A=A, D=D, integrator=W.INT_RK4, T=0.1, span=7.0)
    Hm = np.array([[1.0, 0.4]])
    R = np.array([[0.3]])
    m = m.with_(H=Hm, nz=1, **W.gaussian_noise(R))
    pm, pc = np.array([0.3, -0.2]), np.array([[0.6, 0.15], [0.15, 0.4]])
    st = oracle.create(m, W.gaussian_prior(pm, pc))
    st, _ = oracle.predict(m, st, 0.1)
    assert abs(st.M[0, 1]) > 1e-3 and abs(st.M[1, 0]) > 1e-3          # sheared
    Phi = lin.expm(A * 0.1)
    mk = Phi @ pm
    Pk = Phi @ (pc + lin.W_integral(A, D, 0.1)) @ Phi.T
    z = np.array([0.5])
    st2, ll, status, mp, Cp = oracle.update(m, st, z)
    S = Hm @ Pk @ Hm.T + R
    K = Pk @ Hm.T @ np.linalg.inv(S)
    m_kf = mk + K @ (z - Hm @ mk)
    P_kf = Pk - K @ S @ K.T
    assert status == 0
    np.testing.assert_allclose(mp, m_kf, atol=1e-8)
    np.testing.assert_allclose(Cp, P_kf, atol=1e-8)
    assert abs(ll - scipy.stats.multivariate_normal(Hm @ mk, S).logpdf(z)) < 1e-8
    X2 = oracle.nodes(m, st2.c, st2.M)
    want = scipy.stats.multivariate_normal(m_kf, P_kf).pdf(X2.reshape(-1, 2)).reshape(X2.shape[:-1])
    q2 = oracle.quadrature_weights(m, st2.M)
    # the Chebyshev nodes are widest at the centre (about 0.46 sigma here), where
    # cubic interpolation errs by about 1 % of the peak
    assert np.sum(q2 * np.abs(st2.P - want)) < 3e-2


# ------------------------------------------------------------ prior moments

def test_prior_moments_of_a_gaussian_mixture_hand_values():
    # 1-D: w = (1/4, 3/4), means (-1, 3), variances (0.5, 2):
    # mean = -1/4 + 9/4 = 2; variance = 1/4 (0.5 + 9) + 3/4 (2 + 1) = 4.625
    pr = W.PriorSpec(np.array([1.0, 3.0]), np.array([[-1.0], [3.0]]), np.array([[[0.5]], [[2.0]]]))
    m, C = pmf.prior_moments(pr)
    assert abs(m[0] - 2.0) < 1e-15 and abs(C[0, 0] - 4.625) < 1e-14
    # 2-D, equal weights, means (1, 0) and (-1, 2), covariances I and diag(2, 3):
    # mean (0, 1); covariance (I + diag(2, 3))/2 + the spread of the means,
    # 1/2 [(1, -1)(1, -1)^T + (-1, 1)(-1, 1)^T] = [[1, -1], [-1, 1]]
    pr2 = W.PriorSpec(np.array([0.5, 0.5]), np.array([[1.0, 0.0], [-1.0, 2.0]]),
                      np.array([np.eye(2), np.diag([2.0, 3.0])]))
    m2, C2 = pmf.prior_moments(pr2)
    np.testing.assert_allclose(m2, [0.0, 1.0], atol=1e-15)
    np.testing.assert_allclose(C2, [[2.5, -1.0], [-1.0, 3.0]], atol=1e-15)


def test_created_mixture_density_has_the_mixture_moments():
    """The created grid density's moments (point sums) equal the mixture's
    moments computed by hand above, to the grid's quadrature accuracy."""
    pr = W.PriorSpec(np.array([0.5, 0.5]), np.array([[1.0, 0.0], [-1.0, 2.0]]),
                     np.array([np.eye(2) * 0.3, np.diag([0.2, 0.4])]))
    m = _model(2, (96, 96), span=10.0)
    st = oracle.create(m, pr)
    mm, C = oracle.moments(m, st)
    np.testing.assert_allclose(mm, [0.0, 1.0], atol=1e-10)
    # (0.3 I + diag(0.2, 0.4))/2 plus the spread of the means [[1, -1], [-1, 1]]
    np.testing.assert_allclose(C, [[1.25, -1.0], [-1.0, 1.35]], atol=1e-9)


# ------------------------------------------------------------ boundary share

def test_boundary_fraction_hand_values():
    # uniform weights on a 4 x 5 Fourier grid: the outer layer holds 20 - 2 * 3 = 14 nodes
    m = _model(2, (4, 5))
    st = pmf.State(np.zeros(2), np.diag([0.3, 0.2]), 0.0, np.ones((4, 5)))
    assert abs(oracle.boundary_fraction(m, st) - 14 / 20) < 1e-15
    # all the mass on one corner node -> 1; on the centre node of a 5 x 5 grid -> 0
    m5 = _model(2, (5, 5))
    P = np.zeros((5, 5))
    P[4, 0] = 1.0
    assert oracle.boundary_fraction(m5, pmf.State(np.zeros(2), np.eye(2), 0.0, P)) == 1.0
    P = np.zeros((5, 5))
    P[2, 2] = 1.0
    assert oracle.boundary_fraction(m5, pmf.State(np.zeros(2), np.eye(2), 0.0, P)) == 0.0
    # Chebyshev, N = 3: the Clenshaw-Curtis weights of the 5-point rule are
    # 1/15, 8/15, 12/15, 8/15, 1/15, so a uniform density has 16/28 = 4/7 of its
    # mass on the two outer interior nodes
    mc = _model(1, (3,), grid=W.CHEBYSHEV)
    st = pmf.State(np.zeros(1), np.eye(1), 0.0, np.ones(3))
    assert abs(oracle.boundary_fraction(mc, st) - 4 / 7) < 1e-14


# ----------------------------------- planted mistakes must be caught by the pins

def _planted_stencil(shift=0, end_taps_kept=False):
    real = pmf.lagrange_stencil

    def wrong(model, a, ua):
        arr_idx, pts, valid, inside = real(model, a, ua)
        if shift and model.grid == W.CHEBYSHEV:
            v = cheb.cgl_nodes(model.N[a])
            k = np.searchsorted(v, pts[:, 0]) + shift
            k = np.clip(k, 0, len(v) - 4)
            kidx = k[:, None] + np.arange(4)[None, :]
            return np.clip(kidx - 1, 0, model.N[a] - 1), v[kidx], (kidx >= 1) & (kidx <= model.N[a]), inside
        if shift:
            pts = pts + shift
            idx = pts.astype(int)
            return np.clip(idx, 0, model.N[a] - 1), pts, (idx >= 0) & (idx <= model.N[a] - 1), inside
        if end_taps_kept:
            return arr_idx, pts, np.ones_like(valid), inside
        return arr_idx, pts, valid, inside

    return wrong


def test_planted_shifted_fourier_stencil_is_caught(monkeypatch):
    monkeypatch.setattr(pmf, "lagrange_stencil", _planted_stencil(shift=1))
    with pytest.raises(AssertionError):
        test_fourier_lagrange_error_formula_pins_the_stencil()


def test_planted_shifted_chebyshev_stencil_is_caught(monkeypatch):
    monkeypatch.setattr(pmf, "lagrange_stencil", _planted_stencil(shift=1))
    with pytest.raises(AssertionError):
        test_chebyshev_lagrange_error_formula_pins_the_stencil((12, 9))


def test_planted_nonzero_chebyshev_end_taps_are_caught(monkeypatch):
    monkeypatch.setattr(pmf, "lagrange_stencil", _planted_stencil(end_taps_kept=True))
    with pytest.raises(AssertionError):
        test_chebyshev_lagrange_exact_on_cubics_vanishing_at_the_ends()


def test_planted_mixture_moments_without_spread_are_caught(monkeypatch):
    def wrong(prior):
        w = np.asarray(prior.w, float) / np.sum(prior.w)
        return np.einsum("g,gi->i", w, prior.mean), np.einsum("g,gij->ij", w, prior.cov)

    monkeypatch.setattr(pmf, "prior_moments", wrong)
    with pytest.raises(AssertionError):
        test_prior_moments_of_a_gaussian_mixture_hand_values()


def test_planted_one_sided_boundary_is_caught(monkeypatch):
    def wrong(model, state):
        q = oracle.quadrature_weights(model, state.M) * state.P
        mask = np.zeros(q.shape, bool)
        for a in range(model.nx):
            idx = [slice(None)] * model.nx
            idx[a] = 0
            mask[tuple(idx)] = True
        return float(np.abs(q[mask]).sum() / q.sum())

    monkeypatch.setattr(oracle, "boundary_fraction", wrong)
    with pytest.raises(AssertionError):
        test_boundary_fraction_hand_values()


def test_planted_uniform_chebyshev_weights_break_the_kalman_pin(monkeypatch):
    real = pmf.quadrature_weights

    def wrong(model, M):
        w = real(model, M)
        if model.grid == W.CHEBYSHEV:
            return np.full(w.shape, abs(np.linalg.det(M)) * (2.0 / (model.N[0] + 1)) ** model.nx)
        return w

    monkeypatch.setattr(pmf, "quadrature_weights", wrong)
    monkeypatch.setattr(oracle, "quadrature_weights", wrong)
    with pytest.raises(AssertionError):
        test_chebyshev_update_is_kalman_on_a_sheared_grid()
