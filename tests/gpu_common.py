"""Helpers shared by the GPU parity tests: run the HIP path through the C ABI and
the oracle side by side on the same seeded inputs."""
from __future__ import annotations

import sys

import numpy as np

import oracle
import workloads as W
from oracle import pmf as opmf


def note(msg: str) -> None:
    print(msg, flush=True)
    sys.stdout.flush()


def l1(model, M, a, b) -> float:
    q = oracle.quadrature_weights(model, np.asarray(M))
    return float(np.sum(q * np.abs(np.asarray(a, float) - np.asarray(b, float))))


# Designed-grid bars for FP32 densities (reading R19).  A measurement update
# designs the new grid from the posterior's FP64 moment sums of FP32 values.  If
# the posterior carries an L1 error e (mass-normalised), the mean moves by at most
# e * R and the variance along an axis by at most e * R^2, R the largest distance
# of a node from the mean: R = N/2 cells = span * sigma (span = 8 sigmas, sigma
# the predictive spread the grid is designed for).  So the centre moves by at most
# e N / 2 cells and a step M_ii = 2 span sqrt(S_ii) / N by at most a relative
# (span^2 / 2) e = 32 e.  With e at the FP32 bar (1e-5) these are the bars below.
# The deviations are printed by every check; FP32 rounding noise spread evenly
# over the grid weighs most in the outer cells, which sets them.
FP32_L1 = 1e-5
FP32_M_RTOL = 32 * FP32_L1   # designed step, relative


def fp32_c_cells(model) -> float:
    """Designed-centre bar in cells: e N / 2 with e the FP32 L1 bar."""
    return FP32_L1 * max(model.N[:model.nx]) / 2


def cell_size(model, M) -> float:
    """Length of one cell along the widest axis: the grid step (Fourier) or the
    half-width times 2/N (Chebyshev, mean node spacing)."""
    M = np.asarray(M, float)
    if model.grid == oracle.pmf.FOURIER:
        return float(np.abs(M).max())
    return float(2.0 * np.abs(M).max() / max(model.N[:model.nx]))


def grid_deviation(model, c, M, st):
    """(relative deviation of M, deviation of c in cells) of a GPU grid from the
    oracle's."""
    c, M = np.asarray(c, float), np.asarray(M, float)
    scale = np.abs(st.M).max()
    return float(np.abs(M - st.M).max() / scale), float(np.abs(c - st.c).max() / cell_size(model, st.M))


EDGE_CLAMP = 1e-6   # index units (Fourier) / computational units (Chebyshev)


def map_onto(model, c, M, P, c_new, M_new):
    """The density (c, M, P) evaluated at the nodes of (c_new, M_new) with the
    oracle's interpolant (trigonometric / Chebyshev-polynomial per axis for an
    axis-aligned grid, else tensor cubic Lagrange), zero outside the source grid,
    except that a node outside by less than EDGE_CLAMP counts as on the edge.
    Comparing two grids that differ by rounding must not hinge on which side of
    an edge a node falls: the regridded densities of the method carry the
    ringing of the trigonometric interpolant out to the grid edges (about 1e-5
    of the peak for an under-resolved posterior), so the zero-outside rule there
    would turn a 1e-8 grid shift into a 1e-5 difference."""
    from oracle import chebyshev as cheb, fourier as fou
    nx = model.nx
    c, M, P = np.asarray(c, float), np.asarray(M, float), np.asarray(P, float)
    Xn = oracle.nodes(model, np.asarray(c_new, float), np.asarray(M_new, float))
    U = (Xn - c) @ np.linalg.inv(M).T
    if model.grid == opmf.FOURIER:
        U = U + np.array([n // 2 for n in model.N[:nx]], float)
        lo, hi = np.zeros(nx), np.array([n - 1 for n in model.N[:nx]], float)
    else:
        lo, hi = -np.ones(nx), np.ones(nx)
    near_lo = (U < lo) & (U >= lo - EDGE_CLAMP)
    near_hi = (U > hi) & (U <= hi + EDGE_CLAMP)
    U = np.where(near_lo, lo, np.where(near_hi, hi, U))
    if model.interp == opmf.INTERP_AUTO and opmf._separable(M):
        out = P
        for a in range(nx):
            idx = [0] * nx
            idx[a] = slice(None)
            ua = U[tuple(idx) + (a,)]
            n = model.N[a]
            if model.grid == opmf.FOURIER:
                Wm = fou.interpolation_matrix(n, ua)
                Wm[(ua < 0.0) | (ua > n - 1)] = 0.0
            else:
                Wm = cheb.poly_interp_matrix(n, ua)
            out = fou.apply_along(Wm, out, a)
        return out
    flatU = U.reshape(-1, nx)
    npts = flatU.shape[0]
    inside = np.ones(npts, bool)
    taps_idx, taps_w = [], []
    for a in range(nx):
        ua = flatU[:, a]
        arr_idx, pts, valid, ins = opmf.lagrange_stencil(model, a, ua)
        inside &= ins
        taps_idx.append(arr_idx)
        taps_w.append(np.where(valid, opmf._lagrange_weights(ua, pts), 0.0))
    out = np.zeros(npts)
    for combo in np.ndindex(*([4] * nx)):
        wt = np.ones(npts)
        ids = []
        for a in range(nx):
            wt = wt * taps_w[a][:, combo[a]]
            ids.append(taps_idx[a][:, combo[a]])
        out += wt * P[tuple(ids)]
    out[~inside] = 0.0
    return out.reshape(tuple(model.N[:nx]))


def errs_vs_oracle(model, c, M, P, st):
    """(L1, largest pointwise error relative to the oracle's peak) of a GPU density
    (c, M, P) against the oracle state st.  When the two grids differ by more than
    1e-12 (FP32 moments move the designed grid), the GPU density is first mapped
    onto the oracle's grid with the oracle's interpolant (map_onto), so the
    figures measure the density, not the grid shift; the grid deviation is
    checked separately."""
    c, M = np.asarray(c, float), np.asarray(M, float)
    scale = np.abs(st.M).max()
    if np.abs(M - st.M).max() <= 1e-12 * scale and np.abs(c - st.c).max() <= 1e-12 * (scale + np.abs(st.c).max()):
        mapped = np.asarray(P, float).reshape(st.P.shape)
    else:
        mapped = map_onto(model, c, M, np.asarray(P, float).reshape(st.P.shape), st.c, st.M)
    err_l1 = l1(model, st.M, mapped, st.P)
    peak = float(np.abs(st.P).max())
    err_max = float(np.abs(mapped - st.P).max() / peak) if peak > 0 else 0.0
    return err_l1, err_max


EPS32 = 2.0 ** -24


def update_amplification(model, st_pred, z) -> float:
    """How much an update magnifies an absolute error spread evenly over the
    predictive density: A = max(P) * sum_j q_j l_j / sum_j q_j P_j l_j (l the
    likelihood at the nodes).  Rounding noise of eta times the predictive's peak
    at every node becomes an L1 error of eta * A in the posterior; A is about 1
    for a measurement near the predictive's mean and grows like the inverse of
    the predictive density where the measurement falls (a 3-sigma outlier in
    one dimension: ~e^4.5)."""
    X = oracle.nodes(model, st_pred.c, st_pred.M)
    L = opmf.loglik_field(model, X, np.atleast_1d(np.asarray(z, float)))
    w = np.exp(L - L.max())
    q = oracle.quadrature_weights(model, st_pred.M)
    P = st_pred.P
    den = float((q * P * w).sum())
    return float(P.max() * (q * w).sum() / den) if den > 0 else float("inf")


def fp32_free_tol(A_sum: float) -> float:
    """FP32 bar of a free-running comparison after updates whose amplifications
    sum to A_sum: each update adds at most 2 eps32 A_k of L1 error."""
    return max(FP32_L1, 2.0 * EPS32 * A_sum)


def fp32_update_tol(A: float) -> float:
    """FP32 bar of a measurement update with amplification A: the 1e-5 bar, or the
    predictive's FP32 rounding noise (2 eps32 of its peak per node, one FFT round
    trip) magnified by the update, whichever is larger."""
    return max(FP32_L1, 2.0 * EPS32 * A)


def l1_vs_oracle(model, c, M, P, st) -> float:
    return errs_vs_oracle(model, c, M, P, st)[0]


def check_density(model, c, M, P, st, tol, what="", designed=False):
    """Assert the GPU density against the oracle: L1 <= tol and every point within
    tol of the oracle's peak; grid equal to rounding (both sides moved the grid
    with the same FP64 plan), or, for grids designed from FP32 densities, within
    the bars that an L1 error tol allows (step 32 tol relative, centre tol N/2
    cells).  Returns (L1, max pointwise error, M deviation, c deviation)."""
    dM, dc = grid_deviation(model, c, M, st)
    if designed:
        mb, cb = 32.0 * tol, tol * max(model.N[:model.nx]) / 2
        assert dM <= mb, f"grid M deviates {dM:.2e} relative > {mb:.1e} {what}"
        assert dc <= cb, f"grid c deviates {dc:.2e} cells > {cb:.1e} {what}"
    else:
        assert dM <= 1e-11, f"grid M deviates {dM:.2e} relative {what}"
        assert dc <= 1e-9, f"grid c deviates {dc:.2e} cells {what}"
    e1, em = errs_vs_oracle(model, c, M, P, st)
    assert e1 <= tol, f"L1 {e1:.3e} > {tol:.1e} {what}"
    assert em <= tol, f"pointwise error {em:.3e} of the peak > {tol:.1e} {what}"
    return e1, em, dM, dc


class Pair:
    """One GPU filter and its oracle twin."""

    def __init__(self, B, ctx, model, prior):
        self.B = B
        self.model = model
        self.f = B.pmf_create(ctx, model, prior)
        self.st = oracle.create(model, prior)

    def close(self):
        self.B.pmf_destroy(self.f)

    def gpu_state(self):
        _, c, M, t, P = self.B.pmf_get_state(self.f)
        return c, M, t, P

    def predict(self, T):
        self.B.pmf_predict(self.f, T)
        self.st, l = oracle.predict(self.model, self.st, T)
        return l

    def update(self, z):
        ll = self.B.pmf_update(self.f, z, want_loglik=True)
        self.amp = update_amplification(self.model, self.st, z)
        self.st, ll_o, status, m, C = oracle.update(self.model, self.st, z)
        return ll, ll_o, status

    def inject_oracle_state(self):
        """Lockstep: give the GPU the oracle's grid and density."""
        self.B.pmf_set_state(self.f, self.st.c, self.st.M, self.st.t, self.st.P, self.model.grid,
                             self.model.precision)

    def compare(self, tol_l1, designed=False, what=""):
        """L1 and pointwise error against the oracle (see check_density); returns L1."""
        c, M, t, P = self.gpu_state()
        self.last = check_density(self.model, c, M, P, self.st, tol_l1, what=what, designed=designed)
        return self.last[0]


def run_free(B, ctx, sc, K, tol, ll_tol=1e-9, what="", report=False):
    """Free-running: GPU and oracle each carry their own state through K cycles,
    compared after every op.  FP64: grids equal to rounding, substep counts equal.
    FP32: the designed grids differ by rounding of the moments (bars from the L1
    bar), the RK4 substep count, a ceiling of a rate computed from the grid, may
    differ by one where that rate sits at an integer, and the bar accumulates:
    every update adds the FP32 noise it magnifies (fp32_update_tol of its
    amplification), and an error an update leaves behind is carried forward, not
    magnified again (the accumulation bar, fp32_free_tol)."""
    fp32 = sc.model.precision == W.FP32
    p = Pair(B, ctx, sc.model, sc.prior)
    worst = [0.0, 0.0, 0.0, 0.0]
    amp_sum = 0.0
    try:
        p.compare(tol, designed=fp32, what=f"{what} create")
        for k in range(K):
            bar = fp32_free_tol(amp_sum) if fp32 else tol
            l_o = p.predict(sc.T)
            l_g = B.pmf_last_substeps(p.f)
            if fp32:
                assert abs(l_g - l_o) <= 1, f"{what} substeps {l_g} vs {l_o} at cycle {k}"
            else:
                assert l_g == l_o, f"{what} substeps differ at cycle {k}"
            p.compare(bar, designed=fp32, what=f"{what} predict {k}")
            ll, ll_o, status = p.update(sc.z[k])
            if fp32:
                amp_sum += p.amp
                bar = fp32_free_tol(amp_sum)
            if np.isnan(ll_o):
                assert np.isnan(ll), (what, k, ll)      # both reject the update
            else:
                assert abs(ll - ll_o) <= ll_tol * max(1.0, abs(ll_o)), (what, k, ll, ll_o)
            p.compare(bar, designed=fp32, what=f"{what} update {k}")
            worst = [max(a, b) for a, b in zip(worst, p.last)]
            if report:
                note(f"  {what} cycle {k}: L1 {p.last[0]:.2e}  max {p.last[1]:.2e}  "
                     f"dM {p.last[2]:.1e}  dc {p.last[3]:.1e} cells  A {p.amp:.0f}  bar {bar:.1e}")
        mean, cov, st = B.pmf_moments(p.f, sc.model.nx)
        m_o, C_o = oracle.moments(sc.model, p.st)
        np.testing.assert_allclose(mean, m_o, atol=1e-9 if tol < 1e-8 else 1e-4)
        np.testing.assert_allclose(cov, C_o, atol=1e-9 if tol < 1e-8 else 1e-4)
        note(f"  {what}: worst over {K} cycles: L1 {worst[0]:.2e}  pointwise {worst[1]:.2e}  "
             f"grid dM {worst[2]:.1e}  dc {worst[3]:.1e} cells" + (f"  summed A {amp_sum:.0f}" if fp32 else ""))
    finally:
        p.close()
    return worst


def run_lockstep(B, ctx, sc, K, tol, what=""):
    """Lockstep: before each op the GPU is given the oracle's state, so each op's
    own error is measured; an update's bar is scaled by its amplification."""
    p = Pair(B, ctx, sc.model, sc.prior)
    worst = [0.0, 0.0, 0.0, 0.0]
    try:
        for k in range(K):
            p.inject_oracle_state()
            p.predict(sc.T)
            p.compare(tol, what=f"{what} predict {k}")
            worst = [max(a, b) for a, b in zip(worst, p.last)]
            p.inject_oracle_state()
            ll, ll_o, status = p.update(sc.z[k])
            assert abs(ll - ll_o) <= 1e-4 * max(1.0, abs(ll_o)), (what, k, ll, ll_o)
            p.compare(max(tol, fp32_update_tol(p.amp)), designed=True, what=f"{what} update {k} (A {p.amp:.0f})")
            worst = [max(a, b) for a, b in zip(worst, p.last)]
        note(f"  {what}: worst over {K} lockstep cycles: L1 {worst[0]:.2e}  pointwise {worst[1]:.2e}  "
             f"grid dM {worst[2]:.1e}  dc {worst[3]:.1e} cells")
    finally:
        p.close()
    return worst


def kalman_density(model, c, M, mean, cov):
    """The Gaussian N(mean, cov) at the nodes of grid (c, M), normalised with the
    grid's quadrature (the exact posterior of a linear-Gaussian model as a grid
    density)."""
    from scipy.stats import multivariate_normal
    X = oracle.nodes(model, c, M)
    P = multivariate_normal(mean, cov).pdf(X.reshape(-1, model.nx)).reshape(tuple(model.N[:model.nx]))
    q = oracle.quadrature_weights(model, M)
    return P / (q * P).sum()


def kalman_filter(sc, K):
    """Exact Kalman filter of a linear-Gaussian scenario (Gaussian prior, z = H x +
    v): posterior (mean, cov) after each of K cycles.  Discretisation x' = e^{AT} x
    + w, w ~ N(0, e^{AT} W(T) e^{A^T T}) with W(T) the oracle's integral."""
    from oracle import linear as lin
    m = sc.model
    nx, nz = m.nx, m.nz
    A = np.asarray(m.A, float)[:nx, :nx]
    Phi = lin.expm(A * sc.T)
    Qd = Phi @ lin.W_integral(A, np.asarray(m.D, float)[:nx, :nx], sc.T) @ Phi.T
    H = np.asarray(m.H, float)[:nz, :nx]
    R = np.asarray(m.noise_cov, float)[0][:nz, :nz]
    mu = np.asarray(sc.prior.mean, float)[0][:nx]
    P = np.asarray(sc.prior.cov, float)[0][:nx, :nx]
    out = []
    for k in range(K):
        mu, P = Phi @ mu, Phi @ P @ Phi.T + Qd
        S = H @ P @ H.T + R
        G = P @ H.T @ np.linalg.inv(S)
        mu = mu + G @ (np.asarray(sc.z[k], float)[:nz] - H @ mu)
        P = (np.eye(nx) - G @ H) @ P
        out.append((mu.copy(), 0.5 * (P + P.T)))
    return out


def oracle_trajectory(args):
    """(c, M, t, P, loglik, update amplification, L1 against the exact Kalman
    posterior or None) of the oracle after each of K predict + update cycles of
    one scenario from its prior.  Pure CPU; runs in a worker process."""
    sc, K, exact = args
    st = oracle.create(sc.model, sc.prior)
    kf = kalman_filter(sc, K) if exact else None
    out = []
    for k in range(K):
        st, _ = oracle.predict(sc.model, st, sc.T)
        amp = update_amplification(sc.model, st, sc.z[k])
        st, ll, status, _, _ = oracle.update(sc.model, st, sc.z[k])
        e_kf = None
        if exact:
            ex = kalman_density(sc.model, st.c, st.M, *kf[k])
            e_kf = l1(sc.model, st.M, st.P, ex)
        out.append((st.c.copy(), st.M.copy(), st.t, st.P.copy(), ll, amp, e_kf))
    return out


def oracle_one_step(args):
    """The oracle's predict + update of step k from the given state: (c, M, t, P,
    loglik, update amplification).  Pure CPU; runs in a worker process."""
    sc, k, c, M, t, P = args
    st = oracle.State(np.asarray(c, float), np.asarray(M, float), t, np.asarray(P, float))
    st, _ = oracle.predict(sc.model, st, sc.T)
    amp = update_amplification(sc.model, st, sc.z[k])
    st, ll, status, _, _ = oracle.update(sc.model, st, sc.z[k])
    return st.c, st.M, st.t, st.P, ll, amp


def oracle_trajectories(scs, K, workers=8, exact=False):
    """oracle_trajectory of every scenario, over fresh worker processes (spawned:
    nothing of this process's GPU state is inherited)."""
    import multiprocessing
    with multiprocessing.get_context("spawn").Pool(min(workers, len(scs))) as pool:
        return pool.map(oracle_trajectory, [(sc, K, exact) for sc in scs])
