"""Quantities of the linear SDE dx = A x dt + Q dw (Sec. I, eq. dynam), FP64.

D = Q Q^T is the diffusion matrix of the Fokker-Planck equation (eq. fokker).
The moving grid follows x' = A x (Sec. II.B), so a grid matrix M evolves as
M(t) = e^{At} M(0) and the diffusion seen in the grid's index coordinates is
D_y(t) = M(t)^-1 D M(t)^-T.
"""
from __future__ import annotations

import numpy as np
import scipy.integrate
import scipy.linalg


def expm(A: np.ndarray) -> np.ndarray:
    return scipy.linalg.expm(A)


def W_integral(A: np.ndarray, D: np.ndarray, T: float) -> np.ndarray:
    """W(T) = int_0^T e^{-As} D e^{-A^T s} ds, by adaptive quadrature of the integrand."""
    if T == 0.0:
        return np.zeros_like(D)

    def f(s):
        E = scipy.linalg.expm(-A * s)
        return E @ D @ E.T

    val, _ = scipy.integrate.quad_vec(f, 0.0, T, epsabs=1e-15, epsrel=1e-13)
    return 0.5 * (val + val.T)


def Dy(A: np.ndarray, D: np.ndarray, M0: np.ndarray, t: float) -> np.ndarray:
    """Diffusion in index coordinates at time t after the grid matrix was M0."""
    Mi = np.linalg.inv(scipy.linalg.expm(A * t) @ M0)
    return Mi @ D @ Mi.T
