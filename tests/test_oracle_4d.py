"""Pins of the oracle in four dimensions (the coordinated-turn workload of Sec. VI)
and of the terrain measurement.

* Kalman-Bucy in 4-D: a Gaussian prior under the coordinated-turn drift with the
  rank-deficient diffusion diag(0, 1, 0, 1) stays Gaussian with mean e^{AT} m and
  covariance e^{AT} (P + W(T)) e^{AT}^T, W(T) from the block exponential (Van
  Loan) computed here with scipy; the trace of A is zero, so the mass is kept.
* Kalman update in 4-D with a linear measurement of the positions.
* Terrain measurement: a map without slope (all frequencies zero) is a constant
  h; the update then keeps the density and the log-likelihood is the noise
  log-density at z - h.
"""
import math

import numpy as np
import pytest
import scipy.linalg
import scipy.stats

import oracle
import workloads as W


def _moments(model, st):
    m, C = oracle.moments(model, st)
    return np.asarray(m), np.asarray(C)


def _ct_model(N, meas=W.H_LINEAR, **kw):
    al = W.CT_TURN_RATE
    A = np.array([[0.0, 1.0, 0.0, 0.0], [0.0, 0.0, 0.0, -al], [0.0, 0.0, 0.0, 1.0], [0.0, al, 0.0, 0.0]])
    base = dict(nx=4, A=A, Q=np.diag([0.0, 1.0, 0.0, 1.0]), N=(N,) * 4, t_nominal=1.0,
                integrator=W.INT_EXACT, substeps=1, precision=W.FP64, meas_kind=meas, nz=2,
                H=np.array([[1.0, 0, 0, 0], [0, 0, 1.0, 0]]), **W.gaussian_noise(np.diag([4.0, 4.0])))
    base.update(kw)
    return W.ModelSpec(**base)


def _van_loan(A, D, T):
    n = A.shape[0]
    blk = np.zeros((2 * n, 2 * n))
    blk[:n, :n] = -A
    blk[:n, n:] = D
    blk[n:, n:] = A.T
    E = scipy.linalg.expm(blk * T)
    return E[:n, n:] @ scipy.linalg.expm(-A.T * T)


def test_kalman_bucy_coordinated_turn_4d():
    N = 32          # a node every half standard deviation: aliasing below 1e-8
    m = _ct_model(N)
    m0 = np.array([10.0, 5.0, -3.0, 2.0])
    P0 = np.diag([9.0, 4.0, 6.0, 3.0])
    st = oracle.create(m, W.gaussian_prior(m0, P0))
    mass0 = float(np.sum(oracle.quadrature_weights(m, st.M) * st.P))
    T = 1.0
    st1, _ = oracle.predict(m, st, T)
    Phi = scipy.linalg.expm(m.A * T)
    Wt = _van_loan(m.A, m.D, T)
    mean, C = _moments(m, st1)
    np.testing.assert_allclose(mean, Phi @ m0, atol=1e-6)
    np.testing.assert_allclose(C, Phi @ (P0 + Wt) @ Phi.T, atol=1e-5)
    # tr(A) = 0: the predicted density keeps its mass on the moved grid
    mass1 = float(np.sum(oracle.quadrature_weights(m, st1.M) * st1.P))
    assert abs(mass1 - mass0) < 1e-12


def test_kalman_update_4d():
    N = 32
    m = _ct_model(N)
    m0 = np.array([1.0, 0.5, -1.0, 0.2])
    P0 = np.diag([2.0, 1.0, 1.5, 0.8])
    st = oracle.create(m, W.gaussian_prior(m0, P0))
    z = np.array([1.7, -2.1])
    st1, ll, status, mean, C = oracle.update(m, st, z)
    H = np.asarray(m.H)
    R = np.diag([4.0, 4.0])
    S = H @ P0 @ H.T + R
    K = P0 @ H.T @ np.linalg.inv(S)
    np.testing.assert_allclose(mean, m0 + K @ (z - H @ m0), atol=1e-7)
    np.testing.assert_allclose(C, P0 - K @ H @ P0, atol=1e-6)
    ll_ref = scipy.stats.multivariate_normal(H @ m0, S).logpdf(z)
    assert abs(ll - ll_ref) < 1e-8


def test_flat_terrain_keeps_the_density():
    # all frequencies zero: h(x) = sum_m a_m cos(phi_m), a constant
    terr = np.array([[3.0, 0.4, 0, 0, 0, 0], [-1.5, 2.0, 0, 0, 0, 0]])
    m = _ct_model(12, meas=W.H_TERRAIN, nz=1, terrain=terr, noise_w=np.array([0.5, 0.5]),
                  noise_mean=np.array([[0.0], [20.0]]), noise_cov=np.array([[[1.0]], [[1.0]]]))
    st = oracle.create(m, W.gaussian_prior(np.zeros(4), np.diag([4.0, 1.0, 4.0, 1.0])))
    z = np.array([5.0])
    st1, ll, status, mean, C = oracle.update(m, st, z)
    h = 3.0 * math.cos(0.4) - 1.5 * math.cos(2.0)
    ref = math.log(0.5 * scipy.stats.norm.pdf(z[0] - h) + 0.5 * scipy.stats.norm.pdf(z[0] - h - 20.0))
    assert abs(ll - ref) < 1e-12
    m_before, C_before = _moments(m, st)
    np.testing.assert_allclose(mean, m_before, atol=1e-12)
    np.testing.assert_allclose(C, C_before, atol=1e-10)


def test_terrain_measurement_values():
    # one cosine along p_x: h = a cos(w p_x + phi); the oracle's field at the
    # nodes against the noise density of z - h at those nodes
    terr = np.array([[4.0, 0.3, 0.05, 0.0, 0.0, 0.0]])
    m = _ct_model(8, meas=W.H_TERRAIN, nz=1, terrain=terr, **W.gaussian_noise([[2.0]]))
    X = np.zeros((3, 4))
    X[:, 0] = [0.0, 10.0, -31.4]
    z = np.array([1.0])
    L = oracle.loglik_field(m, X, z)
    h = 4.0 * np.cos(0.05 * X[:, 0] + 0.3)
    np.testing.assert_allclose(L, scipy.stats.norm.logpdf(z[0] - h, scale=math.sqrt(2.0)), atol=1e-13)
