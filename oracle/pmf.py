"""The point-mass filter cycle, step by step, in FP64 (oracle).

State: grid centre c, grid matrix M (its columns are the physical step vectors
of the index axes), time t and the point-mass weights P on N_0 x ... grid
points (C order, last axis fastest).

Fourier grid: node j sits at x_j = c + M (j - N/2) (Sec. III.A equidistant PMD).
Chebyshev grid: x = c + M u with u_a the interior Chebyshev-Gauss-Lobatto nodes
of [-1, 1] (Sec. IV.B), so M's columns are the half-widths.

Cycle: predict(T) is the time update of Sec. I.B solved on the moving grid
(Sec. II.B, Sec. V); update(z) is the Bayes rule of Sec. I.A followed by the
normalisation of Sec. III.A, a new grid design and re-interpolation.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, replace

import numpy as np

from . import chebyshev as cheb
from . import fourier as fou
from . import linear as lin

FOURIER, CHEBYSHEV = 0, 1
INT_EXACT, INT_RK4, INT_EULER, INT_FDM, INT_SINE = 0, 1, 2, 3, 4
INTERP_AUTO, INTERP_LAGRANGE = 0, 1
H_LINEAR, H_CUBIC1, H_NORM, H_TERRAIN = 0, 1, 2, 3

STATUS_OK = 0
STATUS_DEGENERATE = 4
STATUS_BOUNDARY = 64
BOUNDARY_TOL = 1e-4
RK4_STABLE_STEP = 2.5   # h * lambda_max kept at or below this (RK4 is stable to 2.78)
FDM_STABLE_STEP = 1.0   # h * sum_a Dy_aa kept at or below this (explicit scheme of eq. FDM)


@dataclass
class State:
    c: np.ndarray
    M: np.ndarray
    t: float
    P: np.ndarray

    def copy(self) -> "State":
        return State(self.c.copy(), self.M.copy(), float(self.t), self.P.copy())


# ---------------------------------------------------------------------------
# grid geometry

def axis_coords(model, a: int) -> np.ndarray:
    """Computational coordinate of each index along axis a."""
    n = model.N[a]
    if model.grid == FOURIER:
        return np.arange(n) - n // 2
    return cheb.interior_nodes(n)


def nodes(model, c: np.ndarray, M: np.ndarray) -> np.ndarray:
    """Physical positions, shape N + (nx,)."""
    us = np.meshgrid(*[axis_coords(model, a) for a in range(model.nx)], indexing="ij")
    U = np.stack(us, axis=-1).astype(float)
    return c + U @ M.T


def quadrature_weights(model, M: np.ndarray) -> np.ndarray:
    """Integration weight of each node.  Fourier: the cell volume |det M| of the
    equidistant PMD (eq. PDF_pm).  Chebyshev: tensor Clenshaw-Curtis weights of the
    interior nodes times |det M| (dx = |det M| du)."""
    vol = abs(np.linalg.det(M))
    if model.grid == FOURIER:
        return np.full(tuple(model.N), vol)
    w = np.ones(())
    for a in range(model.nx):
        w = np.multiply.outer(w, cheb.cc_weights(model.N[a])[1:-1])
    return vol * w


def moments(model, state: State):
    """Mean and covariance of the point-mass density, two-pass in physical units."""
    X = nodes(model, state.c, state.M)
    q = quadrature_weights(model, state.M) * state.P
    mass = q.sum()
    m = np.tensordot(q, X, axes=(tuple(range(model.nx)), tuple(range(model.nx)))) / mass
    Y = (X - m).reshape(-1, model.nx)
    qf = q.reshape(-1)
    C = (Y * qf[:, None]).T @ Y / mass
    return m, 0.5 * (C + C.T)


def boundary_fraction(model, state: State) -> float:
    """Share of the mass on the outermost layer of nodes."""
    q = quadrature_weights(model, state.M) * state.P
    mask = np.zeros(q.shape, bool)
    for a in range(model.nx):
        idx = [slice(None)] * model.nx
        idx[a] = 0
        mask[tuple(idx)] = True
        idx[a] = -1
        mask[tuple(idx)] = True
    tot = q.sum()
    return float(np.abs(q[mask]).sum() / tot) if tot != 0 else float("inf")


def design_grid(model, mean: np.ndarray, cov: np.ndarray):
    """Axis-aligned grid covering +-span sigmas of the density *after* the next
    nominal interval, pulled back to the present: S = cov + W(t_nominal).
    Fourier step 2h/N (period 2h), Chebyshev half-width h.  Returns (c, M) or
    None when a half-width is not a positive finite number."""
    S = cov + lin.W_integral(model.A, model.D, model.t_nominal)
    d = np.diag(S)
    if not np.all(np.isfinite(d)) or np.any(d <= 0.0):
        return None
    h = model.span_sigmas * np.sqrt(d)
    if model.grid == FOURIER:
        M = np.diag(2.0 * h / np.asarray(model.N, float))
    else:
        M = np.diag(h)
    return np.array(mean, float).copy(), M


# ---------------------------------------------------------------------------
# densities and likelihoods

def _gauss_logpdf(x: np.ndarray, mean: np.ndarray, cov: np.ndarray) -> np.ndarray:
    n = len(mean)
    r = x - mean
    Ci = np.linalg.inv(cov)
    quad = np.einsum("...i,ij,...j->...", r, Ci, r)
    _, logdet = np.linalg.slogdet(cov)
    return -0.5 * quad - 0.5 * (n * math.log(2 * math.pi) + logdet)


def _gm_logpdf(x, w, means, covs) -> np.ndarray:
    terms = np.stack([math.log(w[g]) + _gauss_logpdf(x, means[g], covs[g])
                      for g in range(len(w))], axis=0)
    mx = terms.max(axis=0)
    return mx + np.log(np.exp(terms - mx).sum(axis=0))


def prior_moments(prior):
    w = np.asarray(prior.w, float) / np.sum(prior.w)
    m = np.einsum("g,gi->i", w, prior.mean)
    C = np.zeros((len(m), len(m)))
    for g in range(len(w)):
        d = prior.mean[g] - m
        C += w[g] * (prior.cov[g] + np.outer(d, d))
    return m, C


def measurement(model, X: np.ndarray) -> np.ndarray:
    """h(x) of eq. meas at every node, shape N + (nz,)."""
    if model.meas_kind == H_LINEAR:
        return X @ np.asarray(model.H, float).T
    if model.meas_kind == H_CUBIC1:
        x1 = X[..., 0]
        return (model.hparam[0] * x1 + model.hparam[1] * x1 ** 3)[..., None]
    if model.meas_kind == H_NORM:
        return np.sqrt(np.sum(X * X, axis=-1))[..., None]
    if model.meas_kind == H_TERRAIN:
        # the terrain map of Sec. VI as an analytic function of the state:
        # sum over components m of a_m cos(w_m . x + phi_m)
        out = np.zeros(X.shape[:-1])
        for row in np.asarray(model.terrain, float):
            a, phi, w = row[0], row[1], row[2:2 + X.shape[-1]]
            out = out + a * np.cos(X @ w + phi)
        return out[..., None]
    raise ValueError(model.meas_kind)


def loglik_field(model, X: np.ndarray, z: np.ndarray) -> np.ndarray:
    """log p(z | x) = log p_v(z - h(x)) at every node (Gaussian-mixture noise)."""
    r = np.asarray(z, float) - measurement(model, X)
    w = np.asarray(model.noise_w, float) / np.sum(model.noise_w)
    return _gm_logpdf(r, w, np.asarray(model.noise_mean, float),
                      np.asarray(model.noise_cov, float))


# ---------------------------------------------------------------------------
# create

def create(model, prior) -> State:
    """Grid designed from the prior's moments; weights = prior PDF at the nodes,
    normalised (Sec. III.A)."""
    m, C = prior_moments(prior)
    g = design_grid(model, m, C)
    if g is None:
        raise ValueError("prior covariance gives a degenerate grid")
    c, M = g
    X = nodes(model, c, M)
    w = np.asarray(prior.w, float) / np.sum(prior.w)
    P = np.exp(_gm_logpdf(X, w, np.asarray(prior.mean, float), np.asarray(prior.cov, float)))
    P = P / (quadrature_weights(model, M) * P).sum()
    return State(c, M, 0.0, P)


# ---------------------------------------------------------------------------
# predict

def _rho(model, a: int) -> float:
    """Largest |wavenumber| per axis in index units: pi for Fourier (the Nyquist
    mode); for Chebyshev the square root of the row-sum bound of the interior
    second-derivative matrix (a bound of its spectral radius that needs no
    eigen-solver; the two largest eigenvalues nearly coincide)."""
    if model.grid == FOURIER:
        return math.pi
    return math.sqrt(cheb.d2_row_sum_bound(model.N[a]))


def lambda_bound(model, Dy: np.ndarray) -> float:
    """Upper bound of the decay rate 1/2 |sum_ab Dy_ab k_a k_b| over |k_a| <= rho_a."""
    r = np.array([_rho(model, a) for a in range(model.nx)])
    return 0.5 * float(np.sum(np.abs(Dy) * np.outer(r, r)))


def substeps(model, state: State, T: float) -> int:
    """l = max(l_min, ceil(T * lambda_max / 2.5)) for RK4, with lambda_max the bound
    at t = 0, T/2, T; for the finite-difference scheme l = max(l_min,
    ceil(T * max_t sum_a Dy_aa(t))) over the same times (its step matrix keeps
    its eigenvalues in (-1, 1] for h sum_a Dy_aa <= 1); exact and Euler use l_min."""
    l_min = max(1, int(model.substeps))
    if T <= 0.0:
        return l_min
    if model.integrator == INT_FDM:
        lam = max(float(np.trace(lin.Dy(model.A, model.D, state.M, t))) for t in (0.0, 0.5 * T, T))
        return max(l_min, int(math.ceil(T * lam / FDM_STABLE_STEP)))
    if model.integrator != INT_RK4:
        return l_min
    lam = max(lambda_bound(model, lin.Dy(model.A, model.D, state.M, t))
              for t in (0.0, 0.5 * T, T))
    return max(l_min, int(math.ceil(T * lam / RK4_STABLE_STEP)))


def second_difference(n: int) -> np.ndarray:
    """tridiag(1, -2, 1) on n interior nodes with zero values beyond both ends."""
    return -2.0 * np.eye(n) + np.eye(n, k=1) + np.eye(n, k=-1)


def fdm_step_matrix(n: int, a_t: float, b_t: float) -> np.ndarray:
    """The 1-D step matrix of eq. fdiff: b_t on the diagonal, a_t beside it."""
    return b_t * np.eye(n) + a_t * (np.eye(n, k=1) + np.eye(n, k=-1))


def sine_matrix(n: int) -> np.ndarray:
    """S[i, l] = sin((i + 1)(l + 1) pi / (n + 1)): the sine modes of n interior
    nodes with zeros beyond both ends (S S = (n + 1)/2 I)."""
    j = np.arange(1, n + 1)
    return np.sin(np.outer(j, j) * np.pi / (n + 1))


def _operators(model):
    ops = []
    for a in range(model.nx):
        if model.grid == FOURIER:
            ops.append(fou.diff_matrices(model.N[a]))
        else:
            ops.append(cheb.diff_matrices(model.N[a]))
    return ops


def diffusion_apply(q: np.ndarray, Dy: np.ndarray, ops) -> np.ndarray:
    """1/2 sum_ab Dy_ab d_a d_b q in index coordinates: squares use the second-
    derivative matrix, mixed terms the product of first-derivative matrices
    (Sec. IV derivatives, the diffusion term of eq. easyFPE)."""
    nx = q.ndim
    out = np.zeros_like(q)
    d1q = [fou.apply_along(ops[b][0], q, b) for b in range(nx)]
    for a in range(nx):
        out += 0.5 * Dy[a, a] * fou.apply_along(ops[a][1], q, a)
        for b in range(a + 1, nx):
            out += Dy[a, b] * fou.apply_along(ops[a][0], d1q[b], a)
    return out


def predict(model, state: State, T: float):
    """Time update over T on the moving grid.  Along x' = A x the density obeys
    dp/dt = -tr(A) p + 1/2 div(D grad p) (eq. easyFPE with D = Q Q^T); in index
    coordinates the diffusion is D_y(t) = M(t)^-1 D M(t)^-T.  The scalar trace term
    commutes with the diffusion operator and is applied exactly as e^{-tr(A) T}.
    Returns (new state, substeps used)."""
    A, D = np.asarray(model.A, float), model.D
    M0 = state.M
    l = substeps(model, state, T)
    P = state.P
    if T > 0.0:
        if model.integrator == INT_RK4:
            ops = _operators(model)
            h = T / l
            for n in range(l):
                t0 = n * h
                Da = lin.Dy(A, D, M0, t0)
                Db = lin.Dy(A, D, M0, t0 + 0.5 * h)
                Dc = lin.Dy(A, D, M0, t0 + h)
                k1 = diffusion_apply(P, Da, ops)
                k2 = diffusion_apply(P + 0.5 * h * k1, Db, ops)
                k3 = diffusion_apply(P + 0.5 * h * k2, Db, ops)
                k4 = diffusion_apply(P + h * k3, Dc, ops)
                P = P + (h / 6.0) * (k1 + 2.0 * k2 + 2.0 * k3 + k4)
        elif model.grid != FOURIER:
            raise ValueError("Chebyshev grids support the RK4 integrator only")
        elif model.integrator == INT_EXACT:
            Wy = np.linalg.inv(M0) @ lin.W_integral(A, D, T) @ np.linalg.inv(M0).T
            S = fou.dft_nd(P) * np.exp(-0.5 * fou.symbol(P.shape, Wy))
            P = fou.idft_nd(S).real
        elif model.integrator == INT_FDM:
            # explicit finite differences of eq. FDM on the moving grid, in index
            # coordinates: P <- P + h (-tr(A) P + 1/2 sum_a Dy_aa(t_n) (P_{j+1} - 2 P_j + P_{j-1})_a),
            # n = 0..l-1, zero beyond the grid (the step matrix of eq. fdiff per axis)
            if np.any(A != np.diag(np.diag(A))) or np.any(D != np.diag(np.diag(D))):
                raise ValueError("the finite-difference scheme needs diagonal A and D")
            h = T / l
            trA = float(np.trace(A))
            L2 = [second_difference(model.N[a]) for a in range(model.nx)]
            for n in range(l):
                Dy = lin.Dy(A, D, M0, n * h)
                rhs = -trA * P
                for a in range(model.nx):
                    rhs = rhs + 0.5 * Dy[a, a] * fou.apply_along(L2[a], P, a)
                P = P + h * rhs
        elif model.integrator == INT_SINE:
            # sine-series variant of the spectral update: expand P in the sine modes
            # of the grid with zeros beyond both ends (exact Dirichlet boundary); mode
            # l_a has the second-derivative symbol -(l_a pi / (N_a + 1))^2 in index
            # units and decays exactly by exp(-1/2 sum_a Wy_aa k_a^2)
            if np.any(A != np.diag(np.diag(A))) or np.any(D != np.diag(np.diag(D))):
                raise ValueError("the sine-series variant needs diagonal A and D")
            Wy = np.linalg.inv(M0) @ lin.W_integral(A, D, T) @ np.linalg.inv(M0).T
            coef = P
            for a in range(model.nx):
                n = model.N[a]
                coef = fou.apply_along(sine_matrix(n) * (2.0 / (n + 1)), coef, a)
            g = np.ones(P.shape)
            for a in range(model.nx):
                n = model.N[a]
                k = np.arange(1, n + 1) * np.pi / (n + 1)
                shape = [1] * model.nx
                shape[a] = n
                g = g * np.exp(-0.5 * Wy[a, a] * k ** 2).reshape(shape)
            P = g * coef
            for a in range(model.nx):
                P = fou.apply_along(sine_matrix(model.N[a]), P, a)
        elif model.integrator == INT_EULER:
            # implicit diffusion per substep (Sec. V.A): P_{n+1} = P_n / (1 - q/2 dt c''_n),
            # with c'' = -kappa^2 <= 0 and the diffusion taken at t_n, n = 0..l-1.
            h = T / l
            S = fou.dft_nd(P)
            for n in range(l):
                S = S / (1.0 + 0.5 * h * fou.symbol(P.shape, lin.Dy(A, D, M0, n * h)))
            P = fou.idft_nd(S).real
        else:
            raise ValueError(model.integrator)
        if model.integrator != INT_FDM:   # the explicit scheme carries its own trace term
            P = P * math.exp(-np.trace(A) * T)
    Phi = lin.expm(A * T)
    return State(Phi @ state.c, Phi @ M0, state.t + T, P), l


# ---------------------------------------------------------------------------
# re-interpolation

def _lagrange_weights(t: np.ndarray, pts: np.ndarray) -> np.ndarray:
    """Cubic Lagrange basis through the 4 abscissae pts[m, 0:4], evaluated at t[m]."""
    out = np.ones(pts.shape)
    for k in range(4):
        for i in range(4):
            if i != k:
                out[..., k] *= (t - pts[..., i]) / (pts[..., k] - pts[..., i])
    return out


def lagrange_stencil(model, a: int, ua: np.ndarray):
    """The four taps of the cubic Lagrange stencil along axis a at old
    computational coordinates ua: two nodes on either side of ua, shifted inwards
    at the ends of the node set.  Returns (density index of each tap, clipped to
    the grid; abscissa of each tap; whether the tap is a grid node, a tap beyond
    or on the grid's end being a zero value; whether ua lies in the grid).
    Fourier: the nodes are the indices 0..N-1 and the taps -1 and N are zero.
    Chebyshev: the nodes are the N + 2 Chebyshev-Gauss-Lobatto points, whose two
    end points +-1 carry the zero boundary values."""
    n = model.N[a]
    if model.grid == FOURIER:
        inside = (ua >= 0.0) & (ua <= n - 1)
        i0 = np.floor(np.clip(ua, 0.0, n - 1)).astype(int)
        idx = i0[:, None] + np.arange(-1, 3)[None, :]
        return np.clip(idx, 0, n - 1), idx.astype(float), (idx >= 0) & (idx <= n - 1), inside
    inside = np.abs(ua) <= 1.0
    v = cheb.cgl_nodes(n)                                    # n + 2 nodes
    nn = n + 1
    k0 = np.clip(np.searchsorted(v, ua, side="right") - 1, 0, nn - 1)
    ks = np.clip(k0 - 1, 0, nn - 3)
    kidx = ks[:, None] + np.arange(4)[None, :]
    return np.clip(kidx - 1, 0, n - 1), v[kidx], (kidx >= 1) & (kidx <= n), inside


def _separable(M: np.ndarray) -> bool:
    return bool(np.all(M[~np.eye(M.shape[0], dtype=bool)] == 0.0))


def interpolate(model, state: State, c_new: np.ndarray, M_new: np.ndarray) -> np.ndarray:
    """Values of the old density's interpolant at the new nodes, zero outside the
    old grid.  Trigonometric interpolant of eq. interFreq (Fourier) or the
    Chebyshev polynomial (Chebyshev) per axis when the old grid is axis-aligned
    (M_new is axis-aligned by design); otherwise tensor cubic Lagrange
    interpolation in the old grid's computational coordinates."""
    nx = model.nx
    c_old, M_old, P = state.c, state.M, state.P
    Xn = nodes(model, c_new, M_new)
    U = (Xn - c_old) @ np.linalg.inv(M_old).T      # old computational coordinates
    if model.grid == FOURIER:
        U = U + np.array([n // 2 for n in model.N], float)   # old index coordinates
    if model.interp == INTERP_AUTO and _separable(M_old):
        out = P
        for a in range(nx):
            idx = [0] * nx
            idx[a] = slice(None)
            ua = U[tuple(idx) + (a,)]
            n = model.N[a]
            if model.grid == FOURIER:
                W = fou.interpolation_matrix(n, ua)
                W[(ua < 0.0) | (ua > n - 1)] = 0.0
            else:
                W = cheb.poly_interp_matrix(n, ua)
            out = fou.apply_along(W, out, a)
        return out
    # tensor cubic Lagrange
    shape = tuple(model.N)
    flatU = U.reshape(-1, nx)
    npts = flatU.shape[0]
    inside = np.ones(npts, bool)
    taps_idx, taps_w = [], []
    for a in range(nx):
        ua = flatU[:, a]
        arr_idx, pts, valid, ins = lagrange_stencil(model, a, ua)
        inside &= ins
        taps_idx.append(arr_idx)
        taps_w.append(np.where(valid, _lagrange_weights(ua, pts), 0.0))
    out = np.zeros(npts)
    for combo in np.ndindex(*([4] * nx)):
        wt = np.ones(npts)
        ids = []
        for a in range(nx):
            wt = wt * taps_w[a][:, combo[a]]
            ids.append(taps_idx[a][:, combo[a]])
        out += wt * P[tuple(ids)]
    out[~inside] = 0.0
    return out.reshape(shape)


# ---------------------------------------------------------------------------
# update

def update(model, state: State, z):
    """Bayes rule (eq. filt) at the current nodes, normalisation, grid redesign
    and re-interpolation.  Returns (new state, log p(z | past), status,
    posterior mean, posterior covariance).  On a zero / non-finite normaliser the
    state is returned unchanged with STATUS_DEGENERATE."""
    X = nodes(model, state.c, state.M)
    L = loglik_field(model, X, z)
    s = float(np.max(L))
    if not np.isfinite(s):
        return state, float("nan"), STATUS_DEGENERATE, None, None
    Pt = state.P * np.exp(L - s)
    mass = float((quadrature_weights(model, state.M) * Pt).sum())
    if not np.isfinite(mass) or mass <= 0.0:
        return state, float("nan"), STATUS_DEGENERATE, None, None
    post = State(state.c, state.M, state.t, Pt / mass)
    loglik = s + math.log(mass)
    m, C = moments(model, post)
    status = STATUS_OK
    if boundary_fraction(model, post) > BOUNDARY_TOL:
        status |= STATUS_BOUNDARY
    g = design_grid(model, m, C)
    if g is None:
        return state, float("nan"), STATUS_DEGENERATE, None, None
    c2, M2 = g
    Pn = interpolate(model, post, c2, M2)
    mass2 = float((quadrature_weights(model, M2) * Pn).sum())
    if not np.isfinite(mass2) or mass2 <= 0.0:
        return state, float("nan"), STATUS_DEGENERATE, None, None
    return State(c2, M2, state.t, Pn / mass2), loglik, status, m, C
