"""Four-dimensional filters (the coordinated-turn workload of Sec. VI) on the
HIP path vs the FP64 oracle through the C ABI: linear-Gaussian 4-D cycles with
the exact and RK4 integrators, the coordinated turn with the synthetic terrain
measurement and two-component noise at N_pa = 16 (free running), and at the
paper's N_pa = 34 (radix-17 FFT passes, 34^4 = 1,336,336 points) in lockstep.
Bars as in the other parity tests: L1 <= 1e-10 (FP64), <= 1e-5 per cycle (FP32)."""
import numpy as np
import pytest

import workloads as W
from gpu_common import note, run_free, run_lockstep

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    from paper_2412_07240_amd import binding
    binding.lib()
    return binding


@pytest.fixture(scope="module")
def ctx(B):
    c = B.pmf_ctx_create(0)
    yield c
    B.pmf_ctx_destroy(c)


def _linear_4d(N, integrator, K=2):
    rng = W.rng_for(8, 0)
    A = W.random_stable_A(rng, 4, -0.8, -0.1)
    Q = np.diag(rng.uniform(0.3, 0.8, size=4))
    m = W.ModelSpec(nx=4, A=A, Q=Q, N=N, t_nominal=0.1, integrator=integrator, substeps=1,
                    precision=W.FP64, meas_kind=W.H_LINEAR, nz=2,
                    H=np.array([[1.0, 0.0, 0.5, 0.0], [0.0, 1.0, 0.0, -0.3]]),
                    **W.gaussian_noise(np.diag([0.3, 0.2])))
    prior = W.gaussian_prior(np.zeros(4), np.diag([0.5, 0.4, 0.6, 0.3]))
    return W.simulate(m, prior, 0.1, K, rng)


def test_linear_4d_exact(B, ctx):
    note("case: 4-D linear-Gaussian N=(16,12,16,12), exact integrator, FP64, 2 cycles")
    run_free(B, ctx, _linear_4d((16, 12, 16, 12), W.INT_EXACT), 2, 1e-10, what="lin4d-exact")


def test_linear_4d_rk4(B, ctx):
    note("case: 4-D linear-Gaussian N=(12,10,12,10), RK4, FP64, 2 cycles")
    run_free(B, ctx, _linear_4d((12, 10, 12, 10), W.INT_RK4), 2, 1e-10, what="lin4d-rk4")


def test_coordinated_turn_terrain_n16(B, ctx):
    note("case: coordinated turn + terrain + mixture noise, N_pa=16, FP64, 3 cycles")
    run_free(B, ctx, W.config6(K=3, N=16), 3, 1e-10, what="ct16")


def test_coordinated_turn_terrain_n34_fp32(B, ctx):
    note("case: coordinated turn + terrain, N_pa=34 (34^4 points, radix 17), FP32 lockstep, 1 cycle")
    run_lockstep(B, ctx, W.config6(K=1, N=34, precision=W.FP32), 1, 1e-5, what="ct34-fp32")
