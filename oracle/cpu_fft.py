"""A CPU implementation of the filter cycle with library FFTs, for throughput
comparison only.

TEST INFRASTRUCTURE, NOT A PARITY REFERENCE.  The oracle (oracle.pmf) is the
definition the GPU path is checked against; this module computes the same
predict + update cycle for the batched workload's filters (2-D Fourier grid,
exact integrator, Gaussian measurement noise) the way a tuned CPU program would:
real FFTs of scipy.fft instead of dense DFT matrices, a closed-form W(T) (Van
Loan's block exponential) instead of quadrature, vectorised gathers for the
cubic Lagrange re-interpolation.  tests/test_cpu_fft_reference.py checks it
against the oracle; bench.py times it on the host cores beside the oracle.

Steps (Sec. I.A, I.B, III.A, IV, Algorithm of Sec. V; readings as in the oracle):
predict: P <- IDFT[e^{-tr(A)T} exp(-1/2 kappa^T W_y kappa) DFT(P)], W_y = M^-1 W(T)
M^-T, first-derivative symbol (Nyquist 0) in the cross term, squares keep the
Nyquist wavenumber; grid c <- e^{AT} c, M <- e^{AT} M.
update: P~ = P exp(log l - max log l), normalise, moments, axis-aligned grid
c' = mean, M' = diag(2 span sqrt(diag(cov + W(T_nom))) / N), tensor cubic
Lagrange interpolation in old index coordinates (zero outside the old grid),
renormalise.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.fft
import scipy.linalg

from .pmf import State


def w_integral(A: np.ndarray, D: np.ndarray, T: float) -> np.ndarray:
    """W(T) = int_0^T e^{-As} D e^{-A^T s} ds by Van Loan's block exponential:
    exp([[A, D], [0, -A^T]] T) has upper-right block G = int_0^T e^{A(T-s)} D
    e^{-A^T s} ds = e^{AT} W(T)."""
    n = A.shape[0]
    C = np.zeros((2 * n, 2 * n))
    C[:n, :n] = A
    C[:n, n:] = D
    C[n:, n:] = -A.T
    E = scipy.linalg.expm(C * T)
    W = scipy.linalg.solve(E[:n, :n], E[:n, n:])
    return 0.5 * (W + W.T)


class Filter:
    """One 2-D filter of the batched workload (Fourier grid, exact integrator,
    linear measurement with Gaussian noise)."""

    def __init__(self, model, T: float):
        self.m = model
        self.T = T
        A = np.asarray(model.A, float)[:2, :2]
        D = np.asarray(model.D, float)[:2, :2]
        self.A = A
        self.Phi = scipy.linalg.expm(A * T)
        self.W = w_integral(A, D, T)
        self.Wnom = w_integral(A, D, model.t_nominal)
        self.etr = math.exp(-np.trace(A) * T)
        N0, N1 = model.N[0], model.N[1]
        self.N = (N0, N1)
        k0 = 2.0 * np.pi * np.fft.fftfreq(N0, 1.0 / N0) / N0          # full axis
        k1 = 2.0 * np.pi * np.arange(N1 // 2 + 1) / N1                # half axis (rfft)
        a1 = k0.copy()
        a1[N0 // 2] = 0.0
        b1 = k1.copy()
        b1[N1 // 2] = 0.0
        self.k0sq, self.k1sq = (k0 * k0)[:, None], (k1 * k1)[None, :]
        self.cross = a1[:, None] * b1[None, :]
        self.u0 = (np.arange(N0) - N0 // 2).astype(float)
        self.u1 = (np.arange(N1) - N1 // 2).astype(float)
        H = np.asarray(model.H, float)[:model.nz, :2]
        R = np.asarray(model.noise_cov, float)[0][:model.nz, :model.nz]
        self.H = H
        self.Ri = np.linalg.inv(R)
        self.nmean = np.asarray(model.noise_mean, float)[0][:model.nz]
        self.span = model.span_sigmas

    def predict(self, st: State) -> State:
        Mi = np.linalg.inv(st.M)
        Wy = Mi @ self.W @ Mi.T
        g = self.etr * np.exp(-0.5 * (Wy[0, 0] * self.k0sq + Wy[1, 1] * self.k1sq) - Wy[0, 1] * self.cross)
        P = scipy.fft.irfft2(scipy.fft.rfft2(st.P) * g, s=self.N)
        return State(self.Phi @ st.c, self.Phi @ st.M, st.t + self.T, P)

    def update(self, st: State, z):
        c, M, P = st.c, st.M, st.P
        # nodes x = c + M u; residual r = z - mean - H x
        U0, U1 = self.u0[:, None], self.u1[None, :]
        X0 = c[0] + M[0, 0] * U0 + M[0, 1] * U1
        X1 = c[1] + M[1, 0] * U0 + M[1, 1] * U1
        r = [np.asarray(z, float)[i] - self.nmean[i] - (self.H[i, 0] * X0 + self.H[i, 1] * X1)
             for i in range(self.H.shape[0])]
        L = np.zeros(P.shape)
        for i in range(len(r)):
            for k in range(len(r)):
                L -= 0.5 * self.Ri[i, k] * r[i] * r[k]
        s = L.max()
        Pt = P * np.exp(L - s)
        vol = abs(np.linalg.det(M))
        mass = vol * Pt.sum()
        if not (mass > 0.0 and np.isfinite(mass)):
            return st, float("nan")
        post = Pt / mass
        w = vol * post
        m0, m1 = (w * X0).sum(), (w * X1).sum()
        d0, d1 = X0 - m0, X1 - m1
        C = np.array([[(w * d0 * d0).sum(), (w * d0 * d1).sum()], [0.0, (w * d1 * d1).sum()]])
        C[1, 0] = C[0, 1]
        S = np.diag(C + self.Wnom)
        if not (np.all(np.isfinite(S)) and np.all(S > 0.0)):
            return st, float("nan")
        M2 = np.diag(2.0 * self.span * np.sqrt(S) / np.asarray(self.N, float))
        c2 = np.array([m0, m1])
        Pn = self.regrid(c, M, post, c2, M2)
        mass2 = abs(np.linalg.det(M2)) * Pn.sum()
        if not (mass2 > 0.0 and np.isfinite(mass2)):
            return st, float("nan")
        lognorm = -0.5 * np.linalg.slogdet(2 * np.pi * np.linalg.inv(self.Ri))[1]
        return State(c2, M2, st.t, Pn / mass2), float(s + lognorm + math.log(mass))

    def regrid(self, c, M, P, c2, M2):
        """Tensor cubic Lagrange interpolation of P (grid c, M) at the nodes of
        (c2, M2), in old index coordinates, zero outside the old grid."""
        N0, N1 = self.N
        Mi = np.linalg.inv(M)
        X0 = c2[0] + M2[0, 0] * self.u0[:, None] + M2[0, 1] * self.u1[None, :]
        X1 = c2[1] + M2[1, 0] * self.u0[:, None] + M2[1, 1] * self.u1[None, :]
        nu0 = (Mi[0, 0] * (X0 - c[0]) + Mi[0, 1] * (X1 - c[1]) + N0 // 2).ravel()
        nu1 = (Mi[1, 0] * (X0 - c[0]) + Mi[1, 1] * (X1 - c[1]) + N1 // 2).ravel()
        inside = (nu0 >= 0) & (nu0 <= N0 - 1) & (nu1 >= 0) & (nu1 <= N1 - 1)
        # zero-padded copy: taps -1 and N read zero
        Pp = np.zeros((N0 + 3, N1 + 3))
        Pp[1:N0 + 1, 1:N1 + 1] = P
        i0 = np.floor(np.clip(nu0, 0, N0 - 1)).astype(np.int64)
        i1 = np.floor(np.clip(nu1, 0, N1 - 1)).astype(np.int64)
        t0, t1 = nu0 - i0, nu1 - i1

        def weights(t):
            tp, tm, t2 = t + 1.0, t - 1.0, t - 2.0
            return [-t * tm * t2 / 6.0, tp * tm * t2 / 2.0, -tp * t * t2 / 2.0, tp * t * tm / 6.0]

        w0, w1 = weights(t0), weights(t1)
        out = np.zeros(nu0.shape)
        for a in range(4):
            row = np.zeros(nu0.shape)
            ra = i0 + a       # padded row of tap i0 - 1 + a
            for b in range(4):
                row += w1[b] * Pp[ra, i1 + b]
            out += w0[a] * row
        out[~inside] = 0.0
        return out.reshape(N0, N1)
