"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module only *draws* inputs: model parameters, priors, true trajectories and
measurements.  It contains none of the filter's arithmetic (no Fokker-Planck
solve, no Bayes update, no grid design); both the CPU oracle and the GPU
library consume the arrays it returns.

Model (Sec. I, eqs. dynam/meas): dx = A x dt + Q dw with E[dw dw^T] = I dt, so the
diffusion matrix of the Fokker-Planck equation is D = Q Q^T; z_k = h(x_k) + v_k
with v_k a Gaussian mixture (Sec. VI, eq. ex1_PDF gives a two-component one).

Every generator is keyed by ``SeedSequence([241207240, cfg, index])``.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace
from typing import List, Optional, Sequence

import numpy as np
import scipy.linalg

SEED_ROOT = 241207240

# grid kinds, integrators, interpolation modes, measurement kinds, precisions
FOURIER, CHEBYSHEV = 0, 1
INT_EXACT, INT_RK4, INT_EULER, INT_FDM, INT_SINE = 0, 1, 2, 3, 4
INTERP_AUTO, INTERP_LAGRANGE = 0, 1
H_LINEAR, H_CUBIC1, H_NORM, H_TERRAIN = 0, 1, 2, 3
FP64, FP32 = 0, 1


@dataclass
class ModelSpec:
    """Plain description of one filter; mirrors ``pmf_model`` in include/pmf.h."""
    nx: int
    A: np.ndarray                 # (nx, nx)
    Q: np.ndarray                 # (nx, nx) noise gain; D = Q Q^T
    N: tuple                      # points per axis, len nx
    grid: int = FOURIER
    span_sigmas: float = 8.0
    t_nominal: float = 0.05
    integrator: int = INT_EXACT
    substeps: int = 1             # minimum number of substeps l
    precision: int = FP64
    interp: int = INTERP_AUTO
    meas_kind: int = H_LINEAR
    nz: int = 1
    H: np.ndarray = field(default_factory=lambda: np.zeros((1, 1)))
    hparam: np.ndarray = field(default_factory=lambda: np.zeros(4))
    noise_w: np.ndarray = field(default_factory=lambda: np.ones(1))
    noise_mean: np.ndarray = field(default_factory=lambda: np.zeros((1, 1)))
    noise_cov: np.ndarray = field(default_factory=lambda: np.eye(1))
    # H_TERRAIN: rows (a_m, phi_m, w_m[0..nx)), h(x) = sum_m a_m cos(w_m . x + phi_m)
    terrain: np.ndarray = field(default_factory=lambda: np.zeros((0, 2)))

    @property
    def D(self) -> np.ndarray:
        return self.Q @ self.Q.T

    def with_(self, **kw) -> "ModelSpec":
        return replace(self, **kw)


@dataclass
class PriorSpec:
    w: np.ndarray                 # (G,)
    mean: np.ndarray              # (G, nx)
    cov: np.ndarray               # (G, nx, nx)


@dataclass
class Scenario:
    model: ModelSpec
    prior: PriorSpec
    T: float                      # interval between measurements
    truth: np.ndarray             # (K+1, nx); truth[0] drawn from the prior
    z: np.ndarray                 # (K, nz); z[k-1] measures truth[k]


def rng_for(cfg: int, index: int = 0) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([SEED_ROOT, cfg, index]))


# ---------------------------------------------------------------------------
# data simulation (exact discretisation of the linear SDE, used only to draw
# the truth; the filter never sees these matrices)

def _discretise(A: np.ndarray, D: np.ndarray, T: float):
    n = A.shape[0]
    blk = np.zeros((2 * n, 2 * n))
    blk[:n, :n] = -A
    blk[:n, n:] = D
    blk[n:, n:] = A.T
    E = scipy.linalg.expm(blk * T)
    F = E[n:, n:].T
    Qd = F @ E[:n, n:]
    return F, 0.5 * (Qd + Qd.T)


def _draw_gm(rng, w, mean, cov):
    g = rng.choice(len(w), p=np.asarray(w) / np.sum(w))
    return rng.multivariate_normal(mean[g], cov[g])


def _h(model: ModelSpec, x: np.ndarray) -> np.ndarray:
    if model.meas_kind == H_LINEAR:
        return model.H @ x
    if model.meas_kind == H_CUBIC1:
        return np.array([model.hparam[0] * x[0] + model.hparam[1] * x[0] ** 3])
    if model.meas_kind == H_NORM:
        return np.array([np.sqrt(np.sum(x * x))])
    if model.meas_kind == H_TERRAIN:
        t = np.asarray(model.terrain, float)
        return np.array([np.sum(t[:, 0] * np.cos(t[:, 2:] @ x + t[:, 1]))])
    raise ValueError(model.meas_kind)


def simulate(model: ModelSpec, prior: PriorSpec, T: float, K: int,
             rng: np.random.Generator) -> Scenario:
    F, Qd = _discretise(model.A, model.D, T)
    x = _draw_gm(rng, prior.w, prior.mean, prior.cov)
    truth = [x]
    zs = []
    for _ in range(K):
        x = F @ x + rng.multivariate_normal(np.zeros(model.nx), Qd)
        v = _draw_gm(rng, model.noise_w, model.noise_mean, model.noise_cov)
        zs.append(_h(model, x) + v)
        truth.append(x)
    return Scenario(model, prior, T, np.array(truth), np.array(zs).reshape(K, model.nz))


def gaussian_noise(R: np.ndarray) -> dict:
    R = np.atleast_2d(np.asarray(R, float))
    nz = R.shape[0]
    return dict(noise_w=np.ones(1), noise_mean=np.zeros((1, nz)), noise_cov=R[None].copy())


def gaussian_prior(mean, cov) -> PriorSpec:
    mean = np.atleast_1d(np.asarray(mean, float))
    cov = np.atleast_2d(np.asarray(cov, float))
    return PriorSpec(np.ones(1), mean[None].copy(), cov[None].copy())


def random_stable_A(rng, nx: int, lo: float, hi: float, max_cond: float = 10.0) -> np.ndarray:
    """A = V diag(lam) V^-1 with Gaussian V (redrawn until cond(V) <= max_cond)."""
    lam = rng.uniform(lo, hi, size=nx)
    while True:
        V = rng.standard_normal((nx, nx))
        if np.linalg.cond(V) <= max_cond:
            break
    return V @ np.diag(lam) @ np.linalg.inv(V)


# ---------------------------------------------------------------------------
# the five workload shapes

def config1(K: int = 100, N: int = 64, precision: int = FP64) -> Scenario:
    """1-D linear SDE A=-0.5, Q=1, prior N(0,1), z = x + v, v ~ N(0, 0.1^2), N=64."""
    T = 0.1  # ten substeps of 0.01 between measurements
    model = ModelSpec(nx=1, A=np.array([[-0.5]]), Q=np.array([[1.0]]), N=(N,),
                      t_nominal=T, integrator=INT_RK4, substeps=10, precision=precision,
                      meas_kind=H_LINEAR, nz=1, H=np.array([[1.0]]),
                      **gaussian_noise([[0.1 ** 2]]))
    prior = gaussian_prior([0.0], [[1.0]])
    return simulate(model, prior, T, K, rng_for(1))


def config2(K: int = 500, N: int = 128, precision: int = FP64,
            integrator: int = INT_RK4) -> Scenario:
    """2-D nearly-constant-velocity model with a cubic measurement of x1."""
    T = 0.05
    model = ModelSpec(nx=2, A=np.array([[0.0, 1.0], [0.0, 0.0]]),
                      Q=np.diag([0.1, 0.5]), N=(N, N), t_nominal=T,
                      integrator=integrator, substeps=1, precision=precision,
                      meas_kind=H_CUBIC1, nz=1, hparam=np.array([1.0, 0.05, 0.0, 0.0]),
                      **gaussian_noise([[0.2 ** 2]]))
    prior = gaussian_prior([0.0, 1.0], np.diag([1.0, 0.25]))
    return simulate(model, prior, T, K, rng_for(2))


def config3(K: int = 200, N: int = 64, precision: int = FP32) -> Scenario:
    """3-D stable linear SDE on a Chebyshev grid, range measurement ||x||."""
    rng = rng_for(3)
    A = random_stable_A(rng, 3, -1.0, -0.1)
    Q = np.tril(rng.uniform(0.0, 0.5, size=(3, 3)))
    T = 0.05
    G = 3
    means = rng.standard_normal((G, 3))
    covs = np.array([np.diag(rng.uniform(0.1, 0.3, size=3) ** 2) for _ in range(G)])
    prior = PriorSpec(np.ones(G) / G, means, covs)
    model = ModelSpec(nx=3, A=A, Q=Q, N=(N, N, N), grid=CHEBYSHEV, t_nominal=T,
                      integrator=INT_RK4, substeps=1, precision=precision,
                      meas_kind=H_NORM, nz=1, **gaussian_noise([[0.1 ** 2]]))
    return simulate(model, prior, T, K, rng)


def synthetic_terrain(rng: np.random.Generator, centre, n: int = 6, wavelengths=(150.0, 900.0),
                      amplitudes=(2.0, 8.0)) -> np.ndarray:
    """A smooth terrain map over the horizontal position (state components 0 and 2
    of the coordinated-turn state): n cosines with random directions, wavelengths
    and amplitudes, in the terrain-function form of ModelSpec.terrain.  Stands in
    for the SRTM table of the paper's experiment (not available)."""
    rows = []
    for _ in range(n):
        lam = rng.uniform(*wavelengths)
        th = rng.uniform(0.0, 2.0 * np.pi)
        k = 2.0 * np.pi / lam
        a = rng.uniform(*amplitudes)
        phi = rng.uniform(0.0, 2.0 * np.pi)
        wx, wy = k * np.cos(th), k * np.sin(th)
        # phase referred to the region's centre keeps the FP64 argument small
        rows.append([a, phi - wx * centre[0] - wy * centre[1], wx, 0.0, wy, 0.0])
    return np.array(rows)


CT_TURN_RATE = np.pi / 6.0          # 30 degrees per second
CT_PRIOR_MEAN = np.array([36569.0, 50.0, 55581.0, 50.0])
CT_PRIOR_COV = np.diag([90.0, 160.0, 5.0, 5.0])


def config6(K: int = 20, N: int = 34, precision: int = FP64, mc: int = 0,
            integrator: int = INT_EXACT) -> Scenario:
    """4-D coordinated turn with known turn rate (Sec. VI): state (p_x, v_x, p_y,
    v_y), D = diag(0, 1, 0, 1), T_s = 1, the paper's prior, a synthetic terrain
    measurement of the horizontal position with the two-component noise
    0.5 N(0, 1) + 0.5 N(20, 1); N_pa points per axis.  The terrain is the same for
    every Monte-Carlo run; mc selects the truth and measurement draws."""
    al = CT_TURN_RATE
    A = np.array([[0.0, 1.0, 0.0, 0.0], [0.0, 0.0, 0.0, -al], [0.0, 0.0, 0.0, 1.0], [0.0, al, 0.0, 0.0]])
    Q = np.diag([0.0, 1.0, 0.0, 1.0])
    terr = synthetic_terrain(rng_for(7, 0), (CT_PRIOR_MEAN[0], CT_PRIOR_MEAN[2]))
    model = ModelSpec(nx=4, A=A, Q=Q, N=(N,) * 4, t_nominal=1.0, integrator=integrator, substeps=1,
                      precision=precision, meas_kind=H_TERRAIN, nz=1, terrain=terr,
                      noise_w=np.array([0.5, 0.5]), noise_mean=np.array([[0.0], [20.0]]),
                      noise_cov=np.array([[[1.0]], [[1.0]]]))
    prior = gaussian_prior(CT_PRIOR_MEAN, CT_PRIOR_COV)
    return simulate(model, prior, 1.0, K, rng_for(7, 1 + mc))


BATCH_SIZES = (32, 48, 64, 96, 128)


def batched_filter(index: int, K: int = 100, sizes: Sequence[int] = BATCH_SIZES,
                   integrator: int = INT_EXACT, precision: int = FP32) -> Scenario:
    """One of the independent 2-D filters of the batched workload."""
    rng = rng_for(4, index)
    A = random_stable_A(rng, 2, -1.0, 0.0)
    Q = np.diag(rng.uniform(0.05, 1.0, size=2))
    N = int(sizes[rng.integers(len(sizes))])
    T = 0.05
    # prior and noise widths (0.3) keep the first posterior resolved on the prior's
    # +-8 sigma grid even at N = 32
    model = ModelSpec(nx=2, A=A, Q=Q, N=(N, N), t_nominal=T, integrator=integrator,
                      substeps=1, precision=precision, meas_kind=H_LINEAR, nz=2,
                      H=np.eye(2), **gaussian_noise(0.3 ** 2 * np.eye(2)))
    prior = gaussian_prior([0.0, 0.0], 0.3 ** 2 * np.eye(2))
    return simulate(model, prior, T, K, rng)


def batched_workload(n_filters: int = 4096, K: int = 100, **kw) -> List[Scenario]:
    return [batched_filter(i, K=K, **kw) for i in range(n_filters)]


SERVE_1D = (64, 96, 128, 192, 256)
SERVE_2D = (32, 48, 64, 96, 128)
SERVE_3D = (32, 48, 64)


def serving_track(index: int, K: int = 4) -> Scenario:
    """One live track of the serving mix: 50% 1-D, 40% 2-D, 10% 3-D."""
    rng = rng_for(5, index)
    u = rng.uniform()
    nx = 1 if u < 0.5 else (2 if u < 0.9 else 3)
    sizes = {1: SERVE_1D, 2: SERVE_2D, 3: SERVE_3D}[nx]
    N = int(sizes[rng.integers(len(sizes))])
    A = random_stable_A(rng, nx, -1.0, 0.0)
    Q = np.diag(rng.uniform(0.05, 1.0, size=nx))
    T = 0.05
    model = ModelSpec(nx=nx, A=A, Q=Q, N=(N,) * nx, t_nominal=T, integrator=INT_EXACT,
                      substeps=1, precision=FP32, meas_kind=H_LINEAR, nz=nx,
                      H=np.eye(nx), **gaussian_noise(0.3 ** 2 * np.eye(nx)))
    prior = gaussian_prior(np.zeros(nx), 0.3 ** 2 * np.eye(nx))
    return simulate(model, prior, T, K, rng)


def poisson_arrivals(rate: float, n: int, seed_index: int = 0) -> np.ndarray:
    """Arrival times (seconds) of n requests of a Poisson process."""
    rng = rng_for(6, seed_index)
    return np.cumsum(rng.exponential(1.0 / rate, size=n))


def gm_measurement_noise() -> dict:
    """Two-component noise of Sec. VI, eq. ex1_PDF: 0.5 N(0,1) + 0.5 N(20,1)."""
    return dict(noise_w=np.array([0.5, 0.5]), noise_mean=np.array([[0.0], [20.0]]),
                noise_cov=np.array([[[1.0]], [[1.0]]]))


def random_density(rng: np.random.Generator, shape: Sequence[int]) -> np.ndarray:
    return rng.uniform(0.0, 1.0, size=tuple(shape))
