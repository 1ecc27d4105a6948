"""Fourier spectral operators on an equidistant periodic grid (Sec. IV).

Everything is in *index units*: node j sits at u = j, the period is N, so the
wavenumber of DFT slot s is kappa_s = 2 pi k_s / N with k_s the signed frequency
(s for s < N/2, s - N otherwise; the Nyquist slot N/2 carries k = -N/2, the
ordering of fftshift(-N/2 : N/2-1) in Sec. V.A).  A physical step delta turns
these into the paper's c' = 2 pi i s / L and c'' = -(2 pi s / L)^2 with L = N delta.
"""
from __future__ import annotations

import numpy as np


def dft_matrix(N: int) -> np.ndarray:
    """F[s, j] = exp(-2 pi i j s / N) / N  (eq. fourtrsf, forward with 1/N)."""
    j = np.arange(N)
    return np.exp(-2j * np.pi * np.outer(j, j) / N) / N


def idft_matrix(N: int) -> np.ndarray:
    """Inverse of eq. fourtrsf: P_j = sum_s P^s exp(+2 pi i j s / N)."""
    j = np.arange(N)
    return np.exp(2j * np.pi * np.outer(j, j) / N)


def signed_freq(N: int) -> np.ndarray:
    """k_s for s = 0..N-1; slot N/2 is the Nyquist frequency -N/2."""
    s = np.arange(N)
    return np.where(s < N // 2, s, s - N)


def kappa(N: int) -> np.ndarray:
    return 2.0 * np.pi * signed_freq(N) / N


def kappa_first(N: int) -> np.ndarray:
    """Symbol of the first derivative divided by i: the sum in Sec. IV runs over
    0 < s < N/2 only, so the Nyquist slot (and slot 0) get 0."""
    k = kappa(N).copy()
    k[N // 2] = 0.0
    return k


def kappa_second(N: int) -> np.ndarray:
    """Minus the symbol of the second derivative (eq. secDer): kappa^2, with the
    Nyquist term -(pi N / L)^2 (= -pi^2 in index units) kept."""
    return kappa(N) ** 2


def diff_matrices(N: int):
    """Dense real D1, D2 with D1 = F^-1 diag(i kappa1) F, D2 = F^-1 diag(-kappa^2) F.
    By design D2 != D1 @ D1 (the Nyquist mode)."""
    F = dft_matrix(N)
    Fi = idft_matrix(N)
    D1 = Fi @ np.diag(1j * kappa_first(N)) @ F
    D2 = Fi @ np.diag(-kappa_second(N)) @ F
    assert np.max(np.abs(D1.imag)) < 1e-9 and np.max(np.abs(D2.imag)) < 1e-9
    return D1.real.copy(), D2.real.copy()


def interpolant_basis(N: int, u: np.ndarray) -> np.ndarray:
    """Phi[m, s]: value at index position u_m of the s-th term of eq. interFreq,
    p(u) = P^0 + sum_{0<s<N/2} (P^s e^{2 pi i s u / N} + P^{N-s} e^{-2 pi i s u / N})
           + P^{N/2} cos(pi u)."""
    u = np.asarray(u, float)
    k = signed_freq(N)
    Phi = np.exp(2j * np.pi * np.outer(u, k) / N)
    Phi[:, N // 2] = np.cos(np.pi * u)
    return Phi


def interpolation_matrix(N: int, u: np.ndarray) -> np.ndarray:
    """W[m, j] such that p(u_m) = sum_j W[m, j] P_j for the trigonometric
    interpolant of the samples P_j (DFT then eq. interFreq)."""
    W = interpolant_basis(N, u) @ dft_matrix(N)
    assert np.max(np.abs(W.imag)) < 1e-9
    return W.real.copy()


def apply_along(mat: np.ndarray, q: np.ndarray, axis: int) -> np.ndarray:
    """(mat applied along one axis of q): out[..., i, ...] = sum_j mat[i, j] q[..., j, ...]."""
    return np.moveaxis(np.tensordot(mat, q, axes=([1], [axis])), 0, axis)


def dft_nd(P: np.ndarray) -> np.ndarray:
    out = P.astype(complex)
    for a, n in enumerate(P.shape):
        out = apply_along(dft_matrix(n), out, a)
    return out


def idft_nd(S: np.ndarray) -> np.ndarray:
    out = S
    for a, n in enumerate(S.shape):
        out = apply_along(idft_matrix(n), out, a)
    return out


def symbol(shape, W: np.ndarray) -> np.ndarray:
    """sigma(kappa) = sum_a W_aa kappa_a^2 + 2 sum_{a<b} W_ab kappa1_a kappa1_b on the
    full mode grid: the Fourier symbol of -sum_ab W_ab d_a d_b, with squares keeping
    the Nyquist term and mixed derivatives built from first-derivative symbols."""
    nx = len(shape)
    grids2 = np.meshgrid(*[kappa_second(n) for n in shape], indexing="ij")
    grids1 = np.meshgrid(*[kappa_first(n) for n in shape], indexing="ij")
    sig = np.zeros(shape)
    for a in range(nx):
        sig += W[a, a] * grids2[a]
        for b in range(a + 1, nx):
            sig += 2.0 * W[a, b] * grids1[a] * grids1[b]
    return sig
