"""Helpers shared by the GPU parity tests: run the HIP path through the C ABI and
the oracle side by side on the same seeded inputs."""
from __future__ import annotations

import sys

import numpy as np

import oracle
from oracle import pmf as opmf


def note(msg: str) -> None:
    print(msg, flush=True)
    sys.stdout.flush()


def l1(model, M, a, b) -> float:
    q = oracle.quadrature_weights(model, np.asarray(M))
    return float(np.sum(q * np.abs(np.asarray(a, float) - np.asarray(b, float))))


def l1_vs_oracle(model, c, M, P, st) -> float:
    """L1 of a GPU density (c, M, P) against the oracle state st.  When the two
    grids differ by more than 1e-12 (FP32 moments move the designed grid by
    ~1e-6), the GPU density is first mapped onto the oracle's grid with the
    oracle's own interpolant, so the figure measures the density, not the grid
    shift; the grid deviation is checked separately."""
    c, M = np.asarray(c, float), np.asarray(M, float)
    scale = np.abs(st.M).max()
    if np.abs(M - st.M).max() <= 1e-12 * scale and np.abs(c - st.c).max() <= 1e-12 * (scale + np.abs(st.c).max()):
        return l1(model, st.M, P, st.P)
    mapped = oracle.interpolate(model, oracle.State(c, M, st.t, np.asarray(P, float)), st.c, st.M)
    return l1(model, st.M, mapped, st.P)


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
        self.st, ll_o, status, m, C = oracle.update(self.model, self.st, z)
        return ll, ll_o, status

    def inject_oracle_state(self):
        """Lockstep: give the GPU the oracle's grid and density."""
        self.B.pmf_set_state(self.f, self.st.c, self.st.M, self.st.t, self.st.P, self.model.grid,
                             self.model.precision)

    def compare(self, tol_l1, grid_rtol=1e-11, what=""):
        c, M, t, P = self.gpu_state()
        scale = np.max(np.abs(self.st.M))
        np.testing.assert_allclose(M, self.st.M, rtol=0, atol=grid_rtol * scale, err_msg=f"grid M {what}")
        np.testing.assert_allclose(c, self.st.c, rtol=0, atol=grid_rtol * (1 + np.abs(self.st.c).max()) + grid_rtol * scale * 10,
                                   err_msg=f"grid c {what}")
        err = l1_vs_oracle(self.model, c, M, P, self.st)
        assert err <= tol_l1, f"L1 {err:.3e} > {tol_l1:.1e} {what}"
        return err


def run_free(B, ctx, sc, K, tol, ll_tol=1e-9, what=""):
    p = Pair(B, ctx, sc.model, sc.prior)
    try:
        p.compare(tol, what=f"{what} create")
        for k in range(K):
            l_o = p.predict(sc.T)
            assert B.pmf_last_substeps(p.f) == l_o, f"{what} substeps differ at cycle {k}"
            p.compare(tol, what=f"{what} predict {k}")
            ll, ll_o, status = p.update(sc.z[k])
            if np.isnan(ll_o):
                assert np.isnan(ll), (what, k, ll)      # both reject the update
            else:
                assert abs(ll - ll_o) <= ll_tol * max(1.0, abs(ll_o)), (what, k, ll, ll_o)
            p.compare(tol, what=f"{what} update {k}")
        mean, cov, st = B.pmf_moments(p.f, sc.model.nx)
        m_o, C_o = oracle.moments(sc.model, p.st)
        np.testing.assert_allclose(mean, m_o, atol=1e-9 if tol < 1e-8 else 1e-4)
        np.testing.assert_allclose(cov, C_o, atol=1e-9 if tol < 1e-8 else 1e-4)
    finally:
        p.close()


def run_lockstep(B, ctx, sc, K, tol, what=""):
    p = Pair(B, ctx, sc.model, sc.prior)
    try:
        for k in range(K):
            p.inject_oracle_state()
            p.predict(sc.T)
            p.compare(tol, grid_rtol=1e-11, what=f"{what} predict {k}")
            p.inject_oracle_state()
            ll, ll_o, status = p.update(sc.z[k])
            assert abs(ll - ll_o) <= 1e-4 * max(1.0, abs(ll_o)), (what, k, ll, ll_o)
            p.compare(tol, grid_rtol=1e-4, what=f"{what} update {k}")
    finally:
        p.close()
