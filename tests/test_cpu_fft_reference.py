"""The CPU-FFT timing reference (oracle/cpu_fft.py) computes the oracle's cycle:
same densities, grids and log-likelihoods to FP64 rounding on the batched
workload's filters; its W(T) equals the oracle's quadrature."""
import numpy as np

import oracle
import workloads as W
from oracle import cpu_fft, linear


def test_van_loan_w_matches_quadrature():
    rng = np.random.default_rng(3)
    for _ in range(4):
        A = W.random_stable_A(rng, 2, -1.0, 0.0)
        Q = np.diag(rng.uniform(0.05, 1.0, size=2))
        D = Q @ Q.T
        for T in (0.05, 0.7):
            np.testing.assert_allclose(cpu_fft.w_integral(A, D, T), linear.W_integral(A, D, T),
                                       rtol=1e-11, atol=1e-14)


def test_cycle_matches_the_oracle():
    scs = W.batched_workload(5, K=3)
    for sc in scs:
        f = cpu_fft.Filter(sc.model, sc.T)
        st_o = oracle.create(sc.model, sc.prior)
        st_c = st_o.copy()
        for k in range(3):
            st_o, _ = oracle.predict(sc.model, st_o, sc.T)
            st_c = f.predict(st_c)
            np.testing.assert_allclose(st_c.M, st_o.M, rtol=1e-11)
            q = abs(np.linalg.det(st_o.M))
            assert q * np.abs(st_c.P - st_o.P).sum() < 1e-12
            st_o, ll_o, status, _, _ = oracle.update(sc.model, st_o, sc.z[k])
            st_c, ll_c = f.update(st_c, sc.z[k])
            np.testing.assert_allclose(st_c.M, st_o.M, rtol=1e-11)
            np.testing.assert_allclose(st_c.c, st_o.c, atol=1e-11 * np.abs(st_o.M).max())
            q = abs(np.linalg.det(st_o.M))
            assert q * np.abs(st_c.P - st_o.P).sum() < 1e-11, (sc.model.N, k)
            assert abs(ll_c - ll_o) < 1e-9 * max(1.0, abs(ll_o))
