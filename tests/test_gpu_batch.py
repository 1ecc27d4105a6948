"""The fused batched step (a planning kernel and one persistent launch per step)
against the FP64 oracle and against the generic path.

Bar (FP32 densities): L1 <= 1e-5 and every point within 1e-5 of the peak, per
filter per step, vs the oracle started from the same state; designed grids
within the bars derived in gpu_common (step 1e-5 relative, centre 1e-4 cells);
log-likelihood to 1e-4 relative."""
import dataclasses

import numpy as np
import pytest

import oracle
import workloads as W
from gpu_common import (EPS32, check_density, fp32_free_tol, fp32_update_tol, oracle_one_step, l1, l1_vs_oracle, note, oracle_trajectories,
                        update_amplification)

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


def make(B, ctx, scs):
    return [B.pmf_create(ctx, sc.model, sc.prior) for sc in scs]


def zmat(scs, k):
    nz = max(sc.model.nz for sc in scs)
    z = np.zeros((len(scs), nz))
    for i, sc in enumerate(scs):
        z[i, :sc.model.nz] = sc.z[k]
    return z


def check_against_oracle(B, fs, scs, before, lls, what):
    """before[i] = (c, M, t, P) of filter i ahead of the step.  Returns the worst
    (L1, pointwise error, grid M deviation, grid c deviation in cells)."""
    worst = [0.0, 0.0, 0.0, 0.0]
    for i, (f, sc) in enumerate(zip(fs, scs)):
        c, M, t, P = before[i]
        st = oracle.State(np.array(c), np.array(M), t, np.asarray(P, float))
        st, _ = oracle.predict(sc.model, st, sc.T)
        amp = update_amplification(sc.model, st, sc.z[k_of(what)])
        st, ll_o, status, _, _ = oracle.update(sc.model, st, sc.z[k_of(what)])
        _, c2, M2, t2, P2 = B.pmf_get_state(f)
        assert abs(t2 - st.t) <= 1e-12 * max(1.0, abs(st.t)), f"{what} filter {i}: time {t2} vs {st.t}"
        e1, em, dM, dc = check_density(sc.model, c2, M2, P2, st, fp32_update_tol(amp),
                                       what=f"{what} filter {i} N={sc.model.N} A {amp:.0f}", designed=True)
        for q, v in enumerate((e1, em, dM, dc)):
            worst[q] = max(worst[q], v)
        if np.isnan(ll_o):
            assert np.isnan(lls[i]), (what, i, lls[i])     # both reject; predicted state kept
        else:
            assert abs(lls[i] - ll_o) <= 1e-4 * max(1.0, abs(ll_o)), (what, i, lls[i], ll_o)
    return worst


_K = {}


def k_of(what):
    return _K[what]


def test_batch_lockstep_mixed_sizes(B, ctx):
    scs = W.batched_workload(40, K=3)
    note(f"case: batch of 40 mixed-size 2-D filters, sizes {sorted(set(sc.model.N[0] for sc in scs))}")
    fs = make(B, ctx, scs)
    try:
        for k in range(3):
            before = [B.pmf_get_state(f)[1:] for f in fs]
            lls = B.pmf_batch_step(ctx, fs, scs[0].T, zmat(scs, k), want_loglik=True)
            what = f"lockstep step {k}"
            _K[what] = k
            worst = check_against_oracle(B, fs, scs, before, lls, what)
            note(f"  step {k}: worst L1 {worst[0]:.2e}  pointwise {worst[1]:.2e}  "
                 f"grid dM {worst[2]:.1e}  dc {worst[3]:.1e} cells")
    finally:
        for f in fs:
            B.pmf_destroy(f)


RECT = ((128, 32), (32, 128), (96, 48), (48, 128), (64, 96), (128, 64), (32, 48))


def test_batch_rectangular_grids_lockstep(B, ctx):
    """Rectangular N0 x N1 grids in one batch with square ones: three steps, each
    against the oracle's step from the same pre-step state (the FP32 bars of the
    mixed-size test); counts per shape leave ragged last groups."""
    scs = []
    for i in range(30):
        sc = W.batched_filter(200 + i, K=3)
        n0, n1 = RECT[i % len(RECT)] if i < 26 else (sc.model.N[0], sc.model.N[0])
        scs.append(dataclasses.replace(sc, model=sc.model.with_(N=(n0, n1))))
    note(f"case: batch of 30 2-D filters, rectangular shapes {RECT} and 4 square")
    fs = make(B, ctx, scs)
    try:
        for k in range(3):
            before = [B.pmf_get_state(f)[1:] for f in fs]
            lls = B.pmf_batch_step(ctx, fs, scs[0].T, zmat(scs, k), want_loglik=True)
            what = f"rectangular step {k}"
            _K[what] = k
            worst = check_against_oracle(B, fs, scs, before, lls, what)
            note(f"  step {k}: worst L1 {worst[0]:.2e}  pointwise {worst[1]:.2e}  "
                 f"grid dM {worst[2]:.1e}  dc {worst[3]:.1e} cells")
    finally:
        for f in fs:
            B.pmf_destroy(f)


def test_batch_step_beyond_the_fused_substep_limit_leaves_the_filter(B, ctx):
    """An RK4 filter whose clamp needs more substeps than the fused form holds (64)
    at run time: the batched cycle leaves its grid, time and density as they were
    (the density up to the FP32 round trip of the transforms), flags PMF_E_INVALID,
    and the same filter then steps on the generic path like its twin."""
    A = np.array([[-0.2, 0.1], [0.05, -0.3]])
    m = W.ModelSpec(nx=2, A=A, Q=np.diag([0.5, 0.5]), N=(32, 32), t_nominal=0.05, integrator=W.INT_RK4,
                    substeps=1, precision=W.FP32, meas_kind=W.H_LINEAR, nz=2, H=np.eye(2),
                    **W.gaussian_noise(0.3 ** 2 * np.eye(2)))
    prior = W.gaussian_prior([0.0, 0.0], 0.3 ** 2 * np.eye(2))
    T = 1.0
    assert oracle.substeps(m, oracle.create(m, prior), T) > 64   # the case's premise
    note("case: RK4 filter needing more than 64 substeps in a batched step (32^2, T = 1)")
    f = B.pmf_create(ctx, m, prior)
    g = B.pmf_create(ctx, m, prior)
    try:
        _, c0, M0, t0, P0 = B.pmf_get_state(f)
        z = np.array([[0.1, -0.05]])
        B.pmf_batch_step(ctx, [f], T, z)
        st = B.lib().pmf_sync_status(f, None)
        assert st & B.PMF_E_INVALID and not st & B.PMF_E_DEGENERATE, st
        _, c1, M1, t1, P1 = B.pmf_get_state(f)
        assert np.array_equal(c1, c0) and np.array_equal(M1, M0) and t1 == t0
        d = np.abs(P1 - P0).max() / np.abs(P0).max()
        note(f"  state kept: density within {d:.1e} of the peak (FFT round trip)")
        assert d <= 1e-5
        # the generic path takes it, as it takes the twin
        for h in (f, g):
            B.pmf_predict(h, T)
        lf = B.pmf_update(f, z[0], want_loglik=True)
        lg = B.pmf_update(g, z[0], want_loglik=True)
        assert np.isfinite(lf) and abs(lf - lg) <= 1e-4 * max(1.0, abs(lg)), (lf, lg)
    finally:
        B.pmf_destroy(f)
        B.pmf_destroy(g)


@pytest.mark.timeout(900)
def test_batch_50_steps_free_running_and_per_step(B, ctx):
    """40 mixed-size filters carried through 50 batched steps with no
    resynchronisation.  Two checks after every step:
      * per step: the GPU's step against the oracle's step from the same
        pre-step state (each step's own error), bar fp32_update_tol of that
        update's amplification;
      * free-running: the GPU's state against the oracle's own 50-step run from
        the same prior.  FP32 rounding moves the GPU's trajectory away from the
        oracle's mostly at outlier measurements (an update magnifies absolute
        errors of the predictive by up to its amplification A) and the filter
        carries such a difference for many steps, so the bar is the stability
        bound max(accumulation bar, 2 A_k (e_{k-1} + 2 eps32)), e_{k-1} the
        difference measured after the previous step (the predict does not grow
        an L1 difference; the update at most magnifies it by its amplification,
        twice for the normalisation).
    The models are linear-Gaussian, so the oracle's own L1 against the exact
    Kalman posterior is printed beside the free-running difference."""
    import multiprocessing
    K, n = 50, 40
    scs = W.batched_workload(n, K=K)
    note(f"case: batch of {n} mixed-size 2-D filters, {K} steps: per-step and free-running vs the oracle")
    trajs = oracle_trajectories(scs, K, exact=True)
    note("  oracle runs done")
    fs = make(B, ctx, scs)
    fa = B.FilterArray(fs)
    worst_step = [0.0, 0.0, 0.0, 0.0]
    worst_free = [0.0, 0.0, 0.0, 0.0]
    amp_sum = np.zeros(n)
    e_prev = np.zeros(n)
    pool = multiprocessing.get_context("spawn").Pool(8)
    try:
        for k in range(K):
            before = [B.pmf_get_state(f)[1:] for f in fs]
            lls = B.pmf_batch_step(ctx, fa, scs[0].T, zmat(scs, k), want_loglik=True)
            one = pool.map(oracle_one_step, [(sc, k, *before[i]) for i, sc in enumerate(scs)])
            ws, wf = [0.0, 0.0, 0.0, 0.0], [0.0, 0.0, 0.0, 0.0]
            e_kf_max = 0.0
            for i, (f, sc) in enumerate(zip(fs, scs)):
                _, c2, M2, t2, P2 = B.pmf_get_state(f)
                c1, M1, t1, P1, ll1, amp1 = one[i]
                r = check_density(sc.model, c2, M2, P2, oracle.State(c1, M1, t1, P1), fp32_update_tol(amp1),
                                  what=f"step {k} filter {i} N={sc.model.N} A {amp1:.0f}", designed=True)
                ws = [max(a, b) for a, b in zip(ws, r)]
                if not np.isnan(ll1):
                    assert abs(lls[i] - ll1) <= 1e-4 * max(1.0, abs(ll1)), (k, i, lls[i], ll1)
                c_o, M_o, t_o, P_o, ll_o, amp, e_kf = trajs[i][k]
                amp_sum[i] += amp
                bar = max(fp32_free_tol(amp_sum[i]), 2.0 * amp * (e_prev[i] + 2.0 * EPS32))
                rf = check_density(sc.model, c2, M2, P2, oracle.State(c_o, M_o, t_o, P_o), bar,
                                   what=f"free step {k} filter {i} N={sc.model.N} A {amp:.0f} prev {e_prev[i]:.1e}",
                                   designed=True)
                e_prev[i] = rf[0]
                wf = [max(a, b) for a, b in zip(wf, rf)]
                e_kf_max = max(e_kf_max, e_kf)
            worst_step = [max(a, b) for a, b in zip(worst_step, ws)]
            worst_free = [max(a, b) for a, b in zip(worst_free, wf)]
            note(f"  step {k}: per-step L1 {ws[0]:.2e} pointwise {ws[1]:.2e} dM {ws[2]:.1e} dc {ws[3]:.1e}; "
                 f"free-running L1 {wf[0]:.2e} pointwise {wf[1]:.2e} dM {wf[2]:.1e} dc {wf[3]:.1e}; "
                 f"oracle vs exact posterior up to {e_kf_max:.1e}")
        note(f"  over {K} steps: per-step worst L1 {worst_step[0]:.2e} pointwise {worst_step[1]:.2e} "
             f"dM {worst_step[2]:.1e} dc {worst_step[3]:.1e}; free-running worst L1 {worst_free[0]:.2e} "
             f"pointwise {worst_free[1]:.2e} dM {worst_free[2]:.1e} dc {worst_free[3]:.1e}")
    finally:
        pool.close()
        pool.join()
        for f in fs:
            B.pmf_destroy(f)


@pytest.mark.parametrize("nf", [12, 1])
def test_batch_matches_generic_fp32_path(B, ctx, nf):
    scs = W.batched_workload(nf, K=5)
    note(f"case: batch vs separate predict+update calls, {nf} filter(s), 5 steps")
    fa = make(B, ctx, scs)
    fb = make(B, ctx, scs)
    try:
        for k in range(5):
            B.pmf_batch_step(ctx, fa, scs[0].T, zmat(scs, k))
            for f, sc in zip(fb, scs):
                B.pmf_predict(f, sc.T)
                B.pmf_update(f, sc.z[k])
        for f, g, sc in zip(fa, fb, scs):
            _, c1, M1, _, P1 = B.pmf_get_state(f)
            _, c2, M2, _, P2 = B.pmf_get_state(g)
            np.testing.assert_allclose(M1, M2, rtol=1e-4)
            ref = oracle.State(c2, M2, 0.0, np.asarray(P2, float))
            assert l1_vs_oracle(sc.model, c1, M1, P1, ref) <= 1e-5
    finally:
        for f in fa + fb:
            B.pmf_destroy(f)


def test_batch_1d_filters_trig_regrid(B, ctx):
    note("case: batch of 1-D filters N in 64..256 (trigonometric re-interpolation)")
    scs = [W.serving_track(i, K=3) for i in range(60)]
    scs = [sc for sc in scs if sc.model.nx == 1][:10]
    assert len(scs) >= 5
    fs = make(B, ctx, scs)
    try:
        for k in range(3):
            before = [B.pmf_get_state(f)[1:] for f in fs]
            lls = B.pmf_batch_step(ctx, fs, scs[0].T, zmat(scs, k), want_loglik=True)
            what = f"1d step {k}"
            _K[what] = k
            check_against_oracle(B, fs, scs, before, lls, what)
    finally:
        for f in fs:
            B.pmf_destroy(f)


def test_batch_full_size_sampled(B, ctx):
    """The benchmark's launch: 4096 filters, N uniform in {32..128}^2.  Sampled
    filters are checked against the oracle from their pre-step state."""
    n = 4096
    note(f"case: full batch {n} filters, 2 steps, 12 sampled filters checked")
    scs = W.batched_workload(n, K=2)
    fs = make(B, ctx, scs)
    rng = np.random.default_rng(5)
    sample = sorted(rng.choice(n, size=12, replace=False).tolist())
    # make sure the largest grid is in the sample
    big = [i for i, sc in enumerate(scs) if sc.model.N[0] == 128][0]
    if big not in sample:
        sample[0] = big
    try:
        B.pmf_batch_step(ctx, fs, scs[0].T, zmat(scs, 0))          # warm: launch set-up cached
        before = [B.pmf_get_state(fs[i])[1:] for i in sample]
        lls = B.pmf_batch_step(ctx, fs, scs[0].T, zmat(scs, 1), want_loglik=True)
        assert np.all(np.isfinite(lls))
        what = "full step 1"
        _K[what] = 1
        worst = check_against_oracle(B, [fs[i] for i in sample], [scs[i] for i in sample], before,
                                     [lls[i] for i in sample], what)
        note(f"  worst L1 {worst[0]:.2e}  pointwise {worst[1]:.2e}  grid dM {worst[2]:.1e}  dc {worst[3]:.1e} cells")
    finally:
        for f in fs:
            B.pmf_destroy(f)


def _corner_state(sc, k, far=False):
    """A state whose next regrid reads the old grid's corner: the old grid is the
    new one (as the oracle designs it) moved back by e^{-AT} and shifted by half a
    cell along both index axes, so new node (0, 0) sits at old index (1/2, 1/2)
    and its cubic stencil takes taps from row -1 and column -1 (far: shifted the
    other way, new node (N-1, N-1) at old index (N-3/2, N-3/2), taps from row N
    and column N)."""
    import scipy.linalg
    import scipy.stats
    m = sc.model
    st = oracle.create(m, sc.prior)
    Phi_inv = scipy.linalg.expm(-np.asarray(m.A, float) * sc.T)
    for _ in range(2):
        s1, _ = oracle.predict(m, st, sc.T)
        s2, *_ = oracle.update(m, s1, sc.z[k])
        M0 = Phi_inv @ s2.M
        c0 = Phi_inv @ (s2.c + (0.5 if far else -0.5) * s2.M @ np.ones(2))
        X = oracle.nodes(m, c0, M0)
        P = sum(w * scipy.stats.multivariate_normal(mu, C).pdf(X)
                for w, mu, C in zip(sc.prior.w, sc.prior.mean, sc.prior.cov))
        st = oracle.State(c0, M0, 0.0, P / (oracle.quadrature_weights(m, M0) * P).sum())
    # where new node (0, 0) falls on the moved old grid
    s1, _ = oracle.predict(m, st, sc.T)
    s2, *_ = oracle.update(m, s1, sc.z[k])
    N = np.asarray(m.N)
    j = (N - 1) if far else np.zeros(2, int)
    x = s2.c + s2.M @ (j - N // 2).astype(float)
    nu = np.linalg.solve(s1.M, x - s1.c) + N // 2
    lo = (N - 2) if far else np.zeros(2)
    assert np.all(nu > lo + 0.05) and np.all(nu < lo + 0.95), nu
    return st


@pytest.mark.parametrize("far", [False, True], ids=["near", "far"])
def test_batch_regrid_reads_corner_taps(B, ctx, far):
    """Regression: the stencil of new node (0, 0) reads old row -1 and column -1
    (far corner: node (N-1, N-1), old row N and column N), which must read as zero
    (guard rows, row pads, or clamped rows of weight zero; not whatever the memory
    held)."""
    scs = W.batched_workload(20, K=1)
    note(f"case: 20 filters set up so that a corner node regrids from the old grid's "
         f"{'far' if far else 'near'} corner cell, sizes {sorted(set(sc.model.N[0] for sc in scs))}")
    fs = make(B, ctx, scs)
    try:
        before = []
        for f, sc in zip(fs, scs):
            st = _corner_state(sc, 0, far)
            B.pmf_set_state(f, st.c, st.M, st.t, st.P, sc.model.grid, sc.model.precision)
            before.append(B.pmf_get_state(f)[1:])
        lls = B.pmf_batch_step(ctx, fs, scs[0].T, zmat(scs, 0), want_loglik=True)
        what = "corner regrid"
        _K[what] = 0
        check_against_oracle(B, fs, scs, before, lls, what)
    finally:
        for f in fs:
            B.pmf_destroy(f)


def _slow_path_scenarios():
    """2-D FP32 filters that take the fused kernel's general branches: RK4 and
    implicit-Euler gains from per-stage coefficient tables, a cubic and a range
    measurement and a two-component mixture noise (log-likelihood per node
    instead of the linear-Gaussian quadratic)."""
    out = []
    for i, N in enumerate((32, 48, 64, 96, 32, 48)):
        rng = W.rng_for(9, i)
        A = W.random_stable_A(rng, 2, -1.0, -0.1)
        Q = np.diag(rng.uniform(0.2, 0.6, size=2))
        kind = i % 3
        if kind == 0:      # RK4 gain, cubic measurement of x1
            meas = dict(meas_kind=W.H_CUBIC1, nz=1, hparam=np.array([1.0, 0.05, 0.0, 0.0]),
                        **W.gaussian_noise([[0.3 ** 2]]))
            integ = W.INT_RK4
        elif kind == 1:    # Euler gain, linear measurement with mixture noise
            meas = dict(meas_kind=W.H_LINEAR, nz=1, H=np.array([[1.0, 0.5]]),
                        noise_w=np.array([0.6, 0.4]), noise_mean=np.array([[0.0], [0.8]]),
                        noise_cov=np.array([[[0.3 ** 2]], [[0.4 ** 2]]]))
            integ = W.INT_EULER
        else:              # exact gain, range measurement
            meas = dict(meas_kind=W.H_NORM, nz=1, **W.gaussian_noise([[0.3 ** 2]]))
            integ = W.INT_EXACT
        m = W.ModelSpec(nx=2, A=A, Q=Q, N=(N, N), t_nominal=0.05, integrator=integ, substeps=1,
                        precision=W.FP32, **meas)
        prior = W.gaussian_prior(np.array([1.5, -1.0]), np.diag([0.4, 0.3]))
        out.append(W.simulate(m, prior, 0.05, 2, rng))
    return out


def test_batch_general_branches_lockstep(B, ctx):
    scs = _slow_path_scenarios()
    note("case: batch of RK4 / Euler / exact gains with cubic, range and mixture-noise "
         "measurements, sizes 32..96, lockstep, 2 steps")
    fs = make(B, ctx, scs)
    try:
        for k in range(2):
            before = [B.pmf_get_state(f)[1:] for f in fs]
            lls = B.pmf_batch_step(ctx, fs, scs[0].T, zmat(scs, k), want_loglik=True)
            what = f"general step {k}"
            _K[what] = k
            check_against_oracle(B, fs, scs, before, lls, what)
    finally:
        for f in fs:
            B.pmf_destroy(f)


def test_batch_replays_are_deterministic(B, ctx):
    note("case: two identical batches give bitwise equal densities")
    scs = W.batched_workload(24, K=3)
    outs = []
    for _ in range(2):
        fs = make(B, ctx, scs)
        for k in range(3):
            B.pmf_batch_step(ctx, fs, scs[0].T, zmat(scs, k))
        outs.append([B.pmf_get_state(f)[4] for f in fs])
        for f in fs:
            B.pmf_destroy(f)
    for a, b in zip(*outs):
        assert np.array_equal(a, b)


def test_batch_steps_back_to_back_equal_synchronised_steps(B, ctx):
    """More steps than the library's z staging slots, submitted back to back from
    one host buffer that the caller overwrites between calls: bitwise equal to
    the same steps with the host waiting for each (a slot reused too early would
    feed a later step's z to an earlier one)."""
    K = 20
    note(f"case: {K} batched steps back to back vs waited for, 24 mixed-size filters")
    scs = W.batched_workload(24, K=K)
    outs = []
    for wait in (True, False):
        fs = make(B, ctx, scs)
        fa = B.FilterArray(fs)
        zbuf = np.zeros((len(scs), 2))
        try:
            for k in range(K):
                zbuf[:] = zmat(scs, k)
                B.pmf_batch_step(ctx, fa, scs[0].T, zbuf)
                if wait:
                    B.pmf_stream_sync()
            B.pmf_stream_sync()
            outs.append([B.pmf_get_state(f) for f in fs])
        finally:
            for f in fs:
                B.pmf_destroy(f)
    for i, (a, b) in enumerate(zip(*outs)):
        assert np.all(np.isfinite(a[4])), f"filter {i}"
        for q in (1, 2, 4):
            assert np.array_equal(a[q], b[q]), f"filter {i} field {q}"


def test_batch_rejects_bad_calls(B, ctx):
    note("case: batch refuses a filter listed twice (not adjacent), T <= 0 and non-finite z")
    scs = W.batched_workload(3, K=1)
    fs = make(B, ctx, scs)
    try:
        for args in (([fs[0], fs[1], fs[0]], 0.05, zmat([scs[0], scs[1], scs[0]], 0)),
                     (fs, 0.0, zmat(scs, 0)),
                     (fs, 0.05, np.full((3, 2), np.nan))):
            with pytest.raises(B.PmfError) as e:
                B.pmf_batch_step(ctx, *args)
            assert e.value.status == B.PMF_E_INVALID
        # an empty batch (through the C call: the binding needs a z row per filter)
        zz = np.zeros(2)
        st = B.lib().pmf_batch_step(ctx, (B.C.c_void_p * 1)(), 0, 0.05,
                                    zz.ctypes.data_as(B.C.POINTER(B.C.c_double)), None, None)
        assert st == B.PMF_E_INVALID
        # the filters are untouched and still step normally
        lls = B.pmf_batch_step(ctx, fs, 0.05, zmat(scs, 0), want_loglik=True)
        assert np.all(np.isfinite(lls))
        # the same set again (the cached path) with a non-finite z: refused, and the
        # next step runs normally
        with pytest.raises(B.PmfError) as e:
            B.pmf_batch_step(ctx, fs, 0.05, np.full((3, 2), np.inf))
        assert e.value.status == B.PMF_E_INVALID
        lls = B.pmf_batch_step(ctx, fs, 0.05, zmat(scs, 0), want_loglik=True)
        assert np.all(np.isfinite(lls))
    finally:
        for f in fs:
            B.pmf_destroy(f)


def test_batch_rejects_unsupported_filters(B, ctx):
    note("case: batch rejects FP64 / 3-D filters before running")
    sc = W.config2(K=1, N=32)                       # FP64
    f = B.pmf_create(ctx, sc.model, sc.prior)
    try:
        with pytest.raises(B.PmfError) as e:
            B.pmf_batch_step(ctx, [f], sc.T, sc.z[:1])
        assert e.value.status == B.PMF_E_INVALID
    finally:
        B.pmf_destroy(f)
