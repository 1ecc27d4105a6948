"""Chebyshev interpolation and differentiation (Sec. IV.B, the alternative for
non-periodic functions; nodes, matrices and quadrature from Trefethen's
Spectral Methods in MATLAB, the paper's reference for Sec. IV).

A grid axis with N points uses the N interior points of the (N+2)-point
Chebyshev-Gauss-Lobatto set on [-1, 1]; the two end points carry the zero
boundary condition.  Nodes are in ascending order: v_k = -cos(k pi / n), n = N+1,
k = 0..n; the density lives on k = 1..N.
"""
from __future__ import annotations

import functools

import numpy as np


def cgl_nodes(N: int) -> np.ndarray:
    """All n+1 = N+2 nodes, ascending, including the boundary points -1 and +1."""
    n = N + 1
    return -np.cos(np.arange(n + 1) * np.pi / n)


def interior_nodes(N: int) -> np.ndarray:
    return cgl_nodes(N)[1:-1]


@functools.lru_cache(maxsize=None)
def _full_d1(N: int) -> np.ndarray:
    """Differentiation matrix of the polynomial interpolant on all N+2 nodes:
    off-diagonal (c_i / c_j) (-1)^(i+j) / (v_i - v_j), c = 2 at the end points and 1
    elsewhere; the diagonal makes every row sum to zero (constants have zero
    derivative)."""
    v = cgl_nodes(N)
    n1 = len(v)
    c = np.ones(n1)
    c[0] = c[-1] = 2.0
    D = np.zeros((n1, n1))
    for i in range(n1):
        for j in range(n1):
            if i != j:
                D[i, j] = (c[i] / c[j]) * (-1.0) ** (i + j) / (v[i] - v[j])
    D[np.diag_indices(n1)] = -D.sum(axis=1)
    return D


def diff_matrices(N: int):
    """Interior D1, D2 (N x N) for functions that vanish at both end points:
    D2 is the square of the full first-derivative matrix, then both are
    restricted to the interior rows and columns."""
    D = _full_d1(N)
    D2 = D @ D
    return D[1:-1, 1:-1].copy(), D2[1:-1, 1:-1].copy()


@functools.lru_cache(maxsize=None)
def d2_spectral_radius(N: int) -> float:
    _, D2 = diff_matrices(N)
    return float(np.max(np.abs(np.linalg.eigvals(D2))))


@functools.lru_cache(maxsize=None)
def d2_row_sum_bound(N: int) -> float:
    """max_i sum_j |D2_ij|: an upper bound of the spectral radius of the interior
    second-derivative matrix (Gershgorin), about 1.5 times the radius itself."""
    _, D2 = diff_matrices(N)
    return float(np.max(np.sum(np.abs(D2), axis=1)))


@functools.lru_cache(maxsize=None)
def cc_weights(N: int) -> np.ndarray:
    """Clenshaw-Curtis weights on all N+2 nodes, found from their defining
    property: the rule integrates T_m exactly on [-1, 1] for m = 0..n."""
    v = cgl_nodes(N)
    n = N + 1
    m = np.arange(n + 1)
    V = np.cos(np.outer(m, np.arccos(np.clip(v, -1, 1))))   # V[m, k] = T_m(v_k)
    even = m % 2 == 0
    rhs = np.zeros(n + 1)
    rhs[even] = 2.0 / (1.0 - m[even].astype(float) ** 2)
    return np.linalg.solve(V, rhs)


def lagrange_matrix(nodes: np.ndarray, x: np.ndarray) -> np.ndarray:
    """L[m, k] = prod_{i != k} (x_m - nodes_i) / (nodes_k - nodes_i)."""
    x = np.asarray(x, float)
    L = np.ones((len(x), len(nodes)))
    for k in range(len(nodes)):
        for i in range(len(nodes)):
            if i != k:
                L[:, k] *= (x - nodes[i]) / (nodes[k] - nodes[i])
    return L


def poly_interp_matrix(N: int, u: np.ndarray) -> np.ndarray:
    """W[m, j]: value at u_m of the degree-(N+1) interpolant through the N interior
    samples and the two zero boundary values (zero outside [-1, 1])."""
    u = np.asarray(u, float)
    W = lagrange_matrix(cgl_nodes(N), u)[:, 1:-1]
    W[np.abs(u) > 1.0] = 0.0
    return W
