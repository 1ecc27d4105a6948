"""What FP32 interpolation weights cost.

The fused kernel evaluates the cubic Lagrange weights of the re-interpolation in
FP32 from FP64 old-grid coordinates (the fractional coordinate rounded to FP32,
the four weights in FP32 arithmetic); everything that sets the coordinates stays
FP64.  This measures that reading in isolation on the oracle: the same update
(same predicted state, measurement, designed grid) with FP64 weights and with
weights rounded as the kernel rounds them, every other step in FP64.  The
difference is held to a tenth of the FP32 density bar (L1 and pointwise 1e-5 of
the peak), so the FP32 weights are not what the FP32 bar is spent on."""
import numpy as np

import oracle
import oracle.pmf as OP
import workloads as W


def _fma32(a, b, c):
    """float32 fused multiply-add: the exact a b + c rounded once (the product of two
    float32 values is exact in float64, and so is its sum with c at these magnitudes
    up to one float64 rounding, far below float32's)."""
    return (a.astype(np.float64) * b.astype(np.float64) + c.astype(np.float64)).astype(np.float32)


def _fp32_weights(t, pts):
    """Cubic Lagrange weights at t through the unit-spaced taps pts = i0 - 1 .. i0 + 2,
    evaluated as the kernel does: s = float32(t - i0), then in float32 with fused
    multiply-adds, from u = 1 - s and p = s u:
    w0 = p (-(1 + u) / 6), w1 = (1 + p / 2) u, w2 = (1 + p / 2) s, w3 = p (-(1 + s) / 6)."""
    f = np.float32
    i0 = pts[..., 1]
    s = (t - i0).astype(f)
    u = (f(1.0) - s).astype(f)
    p = (s * u).astype(f)
    h = _fma32(p, f(0.5), f(1.0))
    w0 = (p * _fma32(u, f(-1.0 / 6.0), f(-1.0 / 6.0))).astype(f)
    w1 = (h * u).astype(f)
    w2 = (h * s).astype(f)
    w3 = (p * _fma32(s, f(-1.0 / 6.0), f(-1.0 / 6.0))).astype(f)
    return np.stack([w0, w1, w2, w3], axis=-1).astype(np.float64)


def _cell(model, M):
    return abs(np.linalg.det(M))


def test_fp32_lagrange_weights_cost(monkeypatch):
    worst_l1 = worst_pt = 0.0
    for idx in range(10):
        sc = W.batched_filter(idx, K=3)
        m = sc.model
        st = oracle.create(m, sc.prior)
        for k in range(3):
            pred, _ = oracle.predict(m, st, sc.T)
            ref, ll_ref, *_ = oracle.update(m, pred, sc.z[k])
            with monkeypatch.context() as mp:
                mp.setattr(OP, "_lagrange_weights", _fp32_weights)
                alt, ll_alt, *_ = oracle.update(m, pred, sc.z[k])
            assert np.array_equal(ref.c, alt.c) and np.array_equal(ref.M, alt.M)
            peak = np.abs(ref.P).max()
            l1 = _cell(m, ref.M) * np.abs(ref.P - alt.P).sum()
            pt = np.abs(ref.P - alt.P).max() / peak
            worst_l1, worst_pt = max(worst_l1, l1), max(worst_pt, pt)
            assert l1 <= 1e-6 and pt <= 1e-6, (idx, k, m.N, l1, pt)
            assert abs(ll_ref - ll_alt) <= 1e-12 * max(1.0, abs(ll_ref))
            st = ref
    print(f"FP32 weights vs FP64 weights: worst L1 {worst_l1:.2e}, worst pointwise {worst_pt:.2e} of the peak")
