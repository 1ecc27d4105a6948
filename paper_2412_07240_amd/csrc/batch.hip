// Batched predict + update: one fused launch per step.
//
// A workgroup takes one group of same-size filters (groups in launch order,
// largest grids first) and runs their whole cycle with the densities resident in
// LDS:
//   load -> row r2c FFT (N/2-point complex FFT + split) -> column FFT ->
//   per-mode gain -> inverse column FFT -> row c2r (merge + N/2-point inverse) ->
//   likelihood (FP64 log-likelihood, FP32 exp) with FP64 moment sums ->
//   normaliser, log-likelihood, grid design -> interpolation onto the new grid
//   (cubic Lagrange for 2-D, trigonometric for 1-D) -> FP64 renormalisation ->
//   store.
// HBM traffic per filter: the density read once and written once.
#include <algorithm>
#include <cstdio>
#include <string>
#include <map>
#include <mutex>
#include <cstdint>
#include <cstring>
#include <vector>

#include "api_internal.h"

namespace pmf {

constexpr int FUSED_THREADS = 1024;
constexpr int FUSED_LMAX = 64;
constexpr int PLAN_THREADS = 16;   // planning kernel workgroup

constexpr int GMAX = 16;            // filters of one size packed into a workgroup
// complex LDS entries per buffer (2 buffers): with the static LDS (10,160 B) and
// the twiddle tables (3,088 B) the workgroup takes the whole 160 KiB
constexpr int CPLX_BUDGET = 9412;

// Complex entries per row of a spectrum: N1/2 + 1 (2-D rows hold the real DC
// and Nyquist entries packed into entry 0 and leave the last unused: the odd
// stride keeps the row transforms free of LDS bank conflicts).
constexpr int spec_pitch(int n1) { return n1 / 2 + 1; }

// complex LDS entries of one buffer for a group of G filters: the spectra, or
// the 2-D posterior, whichever is larger.  The posterior has super-rows of
// n1 + 1 floats (the last a zero pad) after one zero float; with guard, a zero
// super-row set above and below it as well (row -1 and row n0 of every filter)
constexpr int group_cplx(int n0, int n1, int G, bool guard = false) {
    const int spec = n0 * G * spec_pitch(n1);
    const int post = n0 > 1 ? ((n0 + (guard ? 2 : 0)) * G * (n1 + 1) + 2) / 2 : 0;
    return spec > post ? spec : post;
}
// guard rows when they fit the budget; otherwise the stencil clamps its rows
constexpr bool group_guard(int n0, int n1, int G) { return n0 > 1 && group_cplx(n0, n1, G, true) <= CPLX_BUDGET; }

struct FConst {
    KModel m;
    PredictArgs pa;
};

// one filter of a batch
struct BItem {
    float* P[2];
    DevDesc* d;
    const FConst* k;
    double* coef;  // stage coefficient table (RK4 / Euler)
    int idx;       // row of z / loglik
    int n0, n1;    // rows (1 for nx = 1) and row length
    int nx;
};

// a group of G filters with the same grid size, processed by one workgroup
struct GItem {
    int first, G, n0, n1, nx, seg, type, pad;
};

// per-filter plan for one step, written by k_batch_plan
struct FPlan {
    double c[2], M[4], Mi[4], vol;   // grid after the move (2x2 row-major)
    double gc[3];                    // exact integrator: W_y packed 00, 11, 01
    double h, etr, tnew;             // substep, e^{-tr A T}, the filter's time after the step
    double q0, qb[2], qQ[3];         // linear-Gaussian log l = q0 + qb.u - 1/2 u^T Q u
    double Wnom[2], span;
    double pscale;                   // pending scale of the stored density
    int l, bad, fast, integ, interp, nx, par;
    int status;                      // the descriptor's status word before the step
};

// per-filter working state in LDS
struct FState {
    FPlan p;
    const float* pin;
    float* pout;
    DevDesc* d;             // the filter's descriptor, model and row of z, fetched
    const KModel* km;       // once per group (no pointer chase later)
    const double* zrow;
    int idx;
    double s, loglik;
    double amap[4], bmap[2];
    double gnc[2], gnM[4], gnvol;
    double pscale2;
    int ok, bits;
};

// ---------------------------------------------------------------- small helpers

__device__ inline float2 f2add(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ inline float2 f2sub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ inline float2 f2mul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ inline float2 f2conj(float2 a) { return make_float2(a.x, -a.y); }
__device__ inline float2 f2si(float2 a, int s) { return make_float2(-s * a.y, s * a.x); }   // * (s i)
__device__ inline float2 f2scale(float2 a, float f) { return make_float2(a.x * f, a.y * f); }

__device__ inline void fdft2(float2* a) {
    float2 t = a[0];
    a[0] = f2add(t, a[1]);
    a[1] = f2sub(t, a[1]);
}
__device__ inline void fdft3(float2* a, int s) {
    const float h = 0.86602540378443864676f;
    float2 t = f2add(a[1], a[2]), d = f2sub(a[1], a[2]);
    float2 m = f2sub(a[0], f2scale(t, 0.5f));
    a[0] = f2add(a[0], t);
    float2 rot = f2scale(f2si(d, s), h);
    a[1] = f2add(m, rot);
    a[2] = f2sub(m, rot);
}
__device__ inline void fdft4(float2* a, int s) {
    float2 t0 = f2add(a[0], a[2]), t1 = f2sub(a[0], a[2]);
    float2 t2 = f2add(a[1], a[3]), t3 = f2si(f2sub(a[1], a[3]), s);
    a[0] = f2add(t0, t2);
    a[2] = f2sub(t0, t2);
    a[1] = f2add(t1, t3);
    a[3] = f2sub(t1, t3);
}
__device__ inline void fdft8(float2* a, int s) {
    float2 e[4] = {a[0], a[2], a[4], a[6]};
    float2 o[4] = {a[1], a[3], a[5], a[7]};
    fdft4(e, s);
    fdft4(o, s);
    const float r = 0.70710678118654752440f;
    const float2 w1 = make_float2(r, s * r), w3 = make_float2(-r, s * r);
    float2 o1 = f2mul(o[1], w1), o2 = f2si(o[2], s), o3 = f2mul(o[3], w3);
    a[0] = f2add(e[0], o[0]);
    a[4] = f2sub(e[0], o[0]);
    a[1] = f2add(e[1], o1);
    a[5] = f2sub(e[1], o1);
    a[2] = f2add(e[2], o2);
    a[6] = f2sub(e[2], o2);
    a[3] = f2add(e[3], o3);
    a[7] = f2sub(e[3], o3);
}
// 16 points as 4 x 4: four 4-point DFTs over n1 (x[4 n1 + n2]), twiddles
// W16^(n2 k1), four 4-point DFTs over n2; output k1 + 4 k2
__device__ inline void fdft16(float2* a, int s) {
    float2 y[4][4];
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) {
        float2 t[4] = {a[n2], a[n2 + 4], a[n2 + 8], a[n2 + 12]};
        fdft4(t, s);
#pragma unroll
        for (int k1 = 0; k1 < 4; ++k1) y[n2][k1] = t[k1];
    }
    const float c1 = 0.92387953251128675613f, s1 = 0.38268343236508977173f, r = 0.70710678118654752440f;
    y[1][1] = f2mul(y[1][1], make_float2(c1, s * s1));
    y[1][2] = f2mul(y[1][2], make_float2(r, s * r));
    y[1][3] = f2mul(y[1][3], make_float2(s1, s * c1));
    y[2][1] = f2mul(y[2][1], make_float2(r, s * r));
    y[2][2] = f2si(y[2][2], s);
    y[2][3] = f2mul(y[2][3], make_float2(-r, s * r));
    y[3][1] = f2mul(y[3][1], make_float2(s1, s * c1));
    y[3][2] = f2mul(y[3][2], make_float2(-r, s * r));
    y[3][3] = f2mul(y[3][3], make_float2(-c1, -s * s1));
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
        float2 t[4] = {y[0][k1], y[1][k1], y[2][k1], y[3][k1]};
        fdft4(t, s);
#pragma unroll
        for (int k2 = 0; k2 < 4; ++k2) a[k1 + 4 * k2] = t[k2];
    }
}

// 12 = 3 x 4: radix-3 transforms of the stride-4 subsequences, twiddles
// W12^(n2 k1), radix-4 transforms across them (x[n2 + 4 n1] -> X[k1 + 3 k2])
__device__ inline void fdft12(float2* a, int s) {
    float2 y[4][3];
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) {
        float2 t[3] = {a[n2], a[n2 + 4], a[n2 + 8]};
        fdft3(t, s);
#pragma unroll
        for (int k1 = 0; k1 < 3; ++k1) y[n2][k1] = t[k1];
    }
    const float c = 0.86602540378443864676f;   // cos 30 degrees
    y[1][1] = f2mul(y[1][1], make_float2(c, s * 0.5f));
    y[1][2] = f2mul(y[1][2], make_float2(0.5f, s * c));
    y[2][1] = f2mul(y[2][1], make_float2(0.5f, s * c));
    y[2][2] = f2mul(y[2][2], make_float2(-0.5f, s * c));
    y[3][1] = f2si(y[3][1], s);
    y[3][2] = make_float2(-y[3][2].x, -y[3][2].y);
#pragma unroll
    for (int k1 = 0; k1 < 3; ++k1) {
        float2 t[4] = {y[0][k1], y[1][k1], y[2][k1], y[3][k1]};
        fdft4(t, s);
#pragma unroll
        for (int k2 = 0; k2 < 4; ++k2) a[k1 + 3 * k2] = t[k2];
    }
}


// ---------------------------------------------------------------- segmented reductions
// Threads map onto points as (tr, g, j): TPR = G * seg threads per "super-row",
// seg = next power of two >= n1.  Every filter's threads form aligned segments of
// sw = min(seg, 64) lanes, so a filter's partials are reduced in a fixed order:
// shuffles inside the segment part (cseg_sum / cseg_max below), then slots in LDS
// summed by one thread per value.

// ---------------------------------------------------------------- planning (one thread per filter)

// RK4 substep clamp on the moved grid (rarely used in batched steps: out of line)
__device__ __noinline__ int plan_substeps(const PredictArgs& a, const double* Mi, int n, int l) {
    double lam = 0.0;
    for (int q = 0; q < 3; ++q) {
        double E[MSQ], t1[MSQ], Dy[MSQ];
        if (q == 0) {
            mat_copy(E, a.D);
        } else {
            const double* Eq = (q == 1) ? a.emh : a.emT;
            mat_mul(t1, Eq, a.D, n);
            mat_mul_bt(E, t1, Eq, n);
        }
        sandwich_inv(Dy, Mi, E, n);
        double lb = 0.0;
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) lb += fabs(Dy[i * MS + j]) * a.rho[i] * a.rho[j];
        lam = fmax(lam, 0.5 * lb);
    }
    const double need = ceil(a.T * lam / RK4_STABLE_STEP);
    if (need > (double)l) l = need > (double)FUSED_LMAX ? FUSED_LMAX + 1 : (int)need;
    return l;
}

// D_y at the RK4 stage times / Euler substep starts, packed 00, 11, 01
__device__ __noinline__ void plan_stage_coefs(const PredictArgs& a, const double* Mi, int n, int l, double h,
                                              double* coef) {
    const int cnt = (a.integ == PMF_INT_RK4) ? 2 * l + 1 : l;
    const double dt = (a.integ == PMF_INT_RK4) ? 0.5 * h : h;
    double Estep[MSQ], Ek[MSQ], t1[MSQ], E[MSQ], Dy[MSQ], nxt[MSQ];
    expm3(Estep, a.A, -dt, n);
    mat_eye(Ek, n);
    for (int k = 0; k < cnt; ++k) {
        mat_mul(t1, Ek, a.D, n);
        mat_mul_bt(E, t1, Ek, n);
        sandwich_inv(Dy, Mi, E, n);
        coef[3 * k + 0] = Dy[0];
        coef[3 * k + 1] = Dy[MS + 1];
        coef[3 * k + 2] = Dy[1];
        mat_mul(nxt, Ek, Estep, n);
        mat_copy(Ek, nxt);
    }
}

// One filter's plan.  Every operand is loaded before the first branch on any of
// them (the model, the grid, the constants of the interval and the row of z), so
// that the loads go out together: one memory round trip after the item's own.
template <int NX>
__device__ void plan_one(const BItem& I, const double* __restrict__ zs, int nzmax, double* __restrict__ zd,
                         FPlan& __restrict__ Pout) {
    constexpr int n = NX;   // compile-time: the small matrix loops unroll into registers
    const PredictArgs& a = I.k->pa;
    const KModel& m = I.k->m;
    const DevDesc& d = *I.d;

    // ---- loads
    Grid g;
    mat_zero(g.M);
    mat_zero(g.Mi);
    double Phi[MSQ], W[MSQ];
    mat_zero(Phi);
    mat_zero(W);
    for (int i = 0; i < MS; ++i) g.c[i] = i < n ? d.g.c[i] : 0.0;
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            g.M[i * MS + j] = d.g.M[i * MS + j];
            g.Mi[i * MS + j] = d.g.Mi[i * MS + j];
            Phi[i * MS + j] = a.Phi[i * MS + j];
            W[i * MS + j] = a.W[i * MS + j];
        }
    const int par = d.par, status0 = d.status;
    const double pscale = d.pscale, t0 = d.t;
    const int integ = a.integ, lmin = a.lmin;
    const double T = a.T, etr = a.etr;
    const double Wn0 = m.Wnom[0], Wn1 = m.Wnom[MS + 1], span = m.span;
    const int interp = m.interp, meas = m.meas, ncomp = m.ncomp, nz = m.nz;
    const double lw0 = m.lw[0];
    // measurement rows past nz are loaded from valid addresses and weighted zero
    double z[3], H[3][NX], nmean[3], Ri[9];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        z[i] = zs[i < nzmax ? i : 0];
        nmean[i] = m.nmean[0][i];
#pragma unroll
        for (int k = 0; k < n; ++k) H[i][k] = m.H[i * MS + k];
#pragma unroll
        for (int k = 0; k < 3; ++k) Ri[i * 3 + k] = m.nRi[0][i * MS + k];
    }

    // ---- the plan, built in registers
    FPlan P;
    int l = lmin;
    P.bad = 0;
    // exact integrator: W_y = M^-1 W M^-T on the current grid
    if (n == 2) {
        const double m00 = g.Mi[0], m01 = g.Mi[1], m10 = g.Mi[MS], m11 = g.Mi[MS + 1];
        const double t00 = m00 * W[0] + m01 * W[MS], t01 = m00 * W[1] + m01 * W[MS + 1];
        const double t10 = m10 * W[0] + m11 * W[MS], t11 = m10 * W[1] + m11 * W[MS + 1];
        P.gc[0] = t00 * m00 + t01 * m01;
        P.gc[1] = t10 * m10 + t11 * m11;
        P.gc[2] = t00 * m10 + t01 * m11;
    } else {
        P.gc[0] = g.Mi[0] * W[0] * g.Mi[0];
        P.gc[1] = 0.0;
        P.gc[2] = 0.0;
    }
    if (integ != PMF_INT_EXACT) {
        // RK4 / Euler: stage coefficients into the filter's table (out of line)
        double Mi[MSQ];
        mat_copy(Mi, g.Mi);
        if (integ == PMF_INT_RK4 && T > 0.0) l = plan_substeps(a, Mi, n, l);
        if (l > FUSED_LMAX) {
            l = FUSED_LMAX;
            P.bad = 1;
        }
        plan_stage_coefs(a, Mi, n, l, T / l, I.coef);
    }
    P.l = l;
    P.h = T / l;
    P.etr = etr;
    P.tnew = t0 + T;
    P.status = status0;
    if (P.bad) {
        // more substeps than the fused form holds: the cycle leaves the filter as it
        // was (unit gain, no grid move or time step; the update is rejected) and
        // flags PMF_E_INVALID, so that the caller can run it on the generic path
        P.gc[0] = P.gc[1] = P.gc[2] = 0.0;
        P.etr = 1.0;
        P.tnew = t0;
        mat_eye(Phi, n);
    }
    // grid follows x' = A x
    double c2[MS], M2[MSQ];
    mat_zero(M2);
    mat_vec(c2, Phi, g.c, n);
    mat_mul(M2, Phi, g.M, n);
    for (int i = 0; i < n; ++i) g.c[i] = c2[i];
    mat_copy(g.M, M2);
    grid_finish(g, n);
    P.c[0] = g.c[0];
    P.c[1] = n > 1 ? g.c[1] : 0.0;
    P.M[0] = g.M[0];
    P.M[1] = g.M[1];
    P.M[2] = g.M[MS];
    P.M[3] = g.M[MS + 1];
    P.Mi[0] = g.Mi[0];
    P.Mi[1] = g.Mi[1];
    P.Mi[2] = g.Mi[MS];
    P.Mi[3] = g.Mi[MS + 1];
    P.vol = g.vol;
    P.Wnom[0] = Wn0;
    P.Wnom[1] = Wn1;
    P.span = span;
    P.integ = P.bad ? PMF_INT_EXACT : integ;
    P.interp = interp;
    P.nx = n;
    P.par = par;
    P.pscale = pscale;
    // linear-Gaussian measurement: log l as a quadratic in index coordinates,
    // r0 = z - mean - H c, G = H M (rows past nz zero)
    P.fast = (meas == PMF_H_LINEAR && ncomp == 1) ? 1 : 0;
    double r0[3], G[3][NX], Rir0[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const bool on = i < nz;
        double hc = 0.0;
#pragma unroll
        for (int k = 0; k < n; ++k) hc += H[i][k] * g.c[k];
        r0[i] = on ? z[i] - nmean[i] - hc : 0.0;
#pragma unroll
        for (int b = 0; b < n; ++b) {
            double s = 0.0;
#pragma unroll
            for (int k = 0; k < n; ++k) s += H[i][k] * g.M[k * MS + b];
            G[i][b] = on ? s : 0.0;
        }
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < 3; ++k) s += (i < nz && k < nz ? Ri[i * 3 + k] : 0.0) * r0[k];
        Rir0[i] = s;
    }
    double rr = 0.0;
#pragma unroll
    for (int i = 0; i < 3; ++i) rr += r0[i] * Rir0[i];
    double qb[2] = {0.0, 0.0}, Qf[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int a2 = 0; a2 < n; ++a2) {
        double s = 0.0;
#pragma unroll
        for (int i = 0; i < 3; ++i) s += G[i][a2] * Rir0[i];
        qb[a2] = s;
#pragma unroll
        for (int b = 0; b < n; ++b) {
            double t = 0.0;
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int k = 0; k < 3; ++k) t += G[i][a2] * (i < nz && k < nz ? Ri[i * 3 + k] : 0.0) * G[k][b];
            Qf[a2 * 2 + b] = t;
        }
    }
    P.q0 = P.fast ? lw0 - 0.5 * rr : 0.0;
    P.qb[0] = P.fast ? qb[0] : 0.0;
    P.qb[1] = P.fast ? qb[1] : 0.0;
    P.qQ[0] = P.fast ? Qf[0] : 0.0;
    P.qQ[1] = P.fast ? Qf[3] : 0.0;
    P.qQ[2] = P.fast ? Qf[1] : 0.0;
    Pout = P;
    if (zd)
        for (int q = 0; q < 3; ++q)
            if (q < nzmax) zd[q] = z[q];
}

// One thread per filter.  zsrc: the step's measurements, one row of nzmax per item in item
// order (possibly in mapped host memory), so that its load needs no field of the
// item; zdst (optional): device copy of them, same order, for the fused kernel.
// Narrow workgroups spread the filters' latency-bound round trips over every
// compute unit.
__global__ void __launch_bounds__(PLAN_THREADS) k_batch_plan(const BItem* __restrict__ items, FPlan* __restrict__ plans, int n,
                             const double* __restrict__ zsrc, double* __restrict__ zdst, int nzmax) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const BItem I = items[i];
    const double* zs = zsrc + (size_t)i * nzmax;
    double* zd = zdst ? zdst + (size_t)i * nzmax : nullptr;
    if (I.nx == 2)
        plan_one<2>(I, zs, nzmax, zd, plans[i]);
    else
        plan_one<1>(I, zs, nzmax, zd, plans[i]);
}


// general measurement models: log p(z | x) at index coordinates u (FP64)
__device__ __noinline__ double floglik_general(const KModel& m, const FPlan& P, double u0, double u1,
                                               const double* z) {
    double x[2];
    x[0] = P.c[0] + P.M[0] * u0 + P.M[1] * u1;
    x[1] = P.c[1] + P.M[2] * u0 + P.M[3] * u1;
    double hx[3] = {0, 0, 0};
    if (m.meas == PMF_H_LINEAR) {
        for (int i = 0; i < m.nz; ++i) hx[i] = m.H[i * MS] * x[0] + (m.nx > 1 ? m.H[i * MS + 1] * x[1] : 0.0);
    } else if (m.meas == PMF_H_CUBIC1) {
        hx[0] = m.hp[0] * x[0] + m.hp[1] * x[0] * x[0] * x[0];
    } else {
        hx[0] = sqrt(x[0] * x[0] + (m.nx > 1 ? x[1] * x[1] : 0.0));
    }
    double best = -INFINITY, terms[MAXMIX];
    for (int g = 0; g < m.ncomp; ++g) {
        double r[3];
        for (int i = 0; i < m.nz; ++i) r[i] = z[i] - hx[i] - m.nmean[g][i];
        double q = 0.0;
        for (int i = 0; i < m.nz; ++i)
            for (int k = 0; k < m.nz; ++k) q += r[i] * m.nRi[g][i * MS + k] * r[k];
        terms[g] = m.lw[g] - 0.5 * q;
        best = fmax(best, terms[g]);
    }
    if (m.ncomp == 1) return terms[0];
    double acc = 0.0;
    for (int g = 0; g < m.ncomp; ++g) acc += exp(terms[g] - best);
    return best + log(acc);
}

__device__ inline double floglik(const FPlan& P, const KModel& m, double u0, double u1, const double* z) {
    if (P.fast) return P.q0 + P.qb[0] * u0 + P.qb[1] * u1 -
                       0.5 * (P.qQ[0] * u0 * u0 + P.qQ[1] * u1 * u1 + 2.0 * P.qQ[2] * u0 * u1);
    return floglik_general(m, P, u0, u1, z);
}

// al + u0 (be + ga u0), one rounding order everywhere it is evaluated
__device__ __forceinline__ double qpoly(double al, double be, double ga, double u0) {
    return fma(u0, fma(ga, u0, be), al);
}

// trigonometric interpolant of the n samples Po[0..n) at index position nu (1-D)
__device__ __noinline__ float trig_interp_1d(const float* Po, int n, double nu) {
    const double fl = floor(nu);
    if (nu == fl) return Po[(int)fl];
    double sa, ca, spn, cpn;
    sincospi(nu / n, &sa, &ca);
    sincospi(nu, &spn, &cpn);
    double acc = 0.0;
    for (int q = 0; q < n; ++q) {
        double sb, cb;
        sincospi((double)q / n, &sb, &cb);
        const double num = ca * cb + sa * sb;
        const double den = sa * cb - ca * sb;
        acc += ((q & 1) ? -spn : spn) * num / (n * den) * (double)Po[q];
    }
    return (float)acc;
}

// cubic Lagrange weights through nodes -1, 0, 1, 2 at t in [0, 1] (nine
// operations).  With s = 1 - t and p = t s, the weights factor as
// w0 = -p (1 + s) / 6, w1 = (1 + p / 2) s, w2 = (1 + p / 2) t, w3 = -p (1 + t) / 6
// (from (t + 1)(2 - t) = 2 + p).  At t = 0 they are exactly (0, 1, 0, 0) and at
// t = 1 exactly (0, 0, 1, 0)
__device__ inline void cubic_weights(float t, float* w) {
    const float s = 1.f - t;
    const float p = t * s;
    const float h = fmaf(p, 0.5f, 1.f);
    w[0] = p * fmaf(s, -1.f / 6.f, -1.f / 6.f);
    w[1] = h * s;
    w[2] = h * t;
    w[3] = p * fmaf(t, -1.f / 6.f, -1.f / 6.f);
}

typedef __attribute__((address_space(3))) const float lcfloat;

// LDS bases of the four rows of a 16-tap stencil, for a posterior whose rows are
// RSO floats apart: row a of the stencil at offset off starts at base + off + a RSO
// (a = 0..3; base is the top-left tap of the stencil at offset 0).
// Each row's four taps are read as two ds_read2 pairs.  Rows 0 and 1 share one base
// when their offsets fit the 8-bit read2 offset field; the other bases are hidden
// from the compiler by an empty asm, once per thread before the loop over points,
// since it would otherwise rebuild a base for every pair of taps whose offset does
// not fit (four or six address adds per point instead of one or three).
template <int RSO>
struct StencilRows {
    static constexpr bool PAIRED = RSO + 3 <= 255;
    lcfloat* b[4];
    __device__ __forceinline__ explicit StencilRows(lcfloat* base) {
        const unsigned a0 = (unsigned)(size_t)base;
        unsigned a1 = a0 + 4u * RSO, a2 = a0 + 8u * RSO, a3 = a0 + 12u * RSO;
        if constexpr (PAIRED) {
            asm("" : "+v"(a2));
        } else {
            asm("" : "+v"(a1), "+v"(a2), "+v"(a3));
        }
        b[0] = base;
        b[1] = (lcfloat*)(size_t)a1;
        b[2] = (lcfloat*)(size_t)a2;
        b[3] = (lcfloat*)(size_t)a3;
    }
    // sum_a w0[a] sum_b w1[b] P[a][b] over the stencil at offset off
    __device__ __forceinline__ float apply(unsigned off, const float* w0, const float* w1) const {
        float rs[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            lcfloat* row = PAIRED ? (a < 2 ? b[0] + off + a * RSO : b[2] + off + (a - 2) * RSO) : b[a] + off;
            rs[a] = w1[0] * row[0] + w1[1] * row[1] + w1[2] * row[2] + w1[3] * row[3];
        }
        return w0[0] * rs[0] + w0[1] * rs[1] + w0[2] * rs[2] + w0[3] * rs[3];
    }
};

// ---------------------------------------------------------------- the fused kernel
// Specialised at compile time per group type (N0 x N1 grid, G filters side by
// side): every loop bound, divisor and radix plan is a constant.

// Radices of an n-point FFT, first pass first: the power-of-two part 2^e in as
// few passes as possible (8s, with one 16 when e = 1 mod 3 and e >= 4, two 16s
// when e = 2 mod 3 and e >= 8), the first pass (no twiddles) taking the largest
// radix, then 3s.
constexpr int radix_at(int n, int i) {
    int e = 0;
    while (n % 2 == 0) {
        n /= 2;
        ++e;
    }
    int r[16] = {};
    int k = 0;
    if (e % 3 == 1 && e >= 4) {
        r[k++] = 16;
        e -= 4;
    } else if (e % 3 == 2 && e >= 8) {
        r[k++] = 16;
        r[k++] = 16;
        e -= 8;
    }
    while (e >= 3) {
        r[k++] = 8;
        e -= 3;
    }
    if (e == 2) r[k++] = 4;
    if (e == 1) r[k++] = 2;
    // a trailing 4 and a factor 3 merge into one radix-12 pass (96 = 8 x 12);
    // with 8s only, a pair 8 x 8 becomes 16 x 4 first (192 = 16 x 12)
    if (n % 3 == 0 && k >= 2 && r[k - 1] == 8 && r[k - 2] == 8) {
        r[k - 2] = 16;
        r[k - 1] = 4;
    }
    if (n % 3 == 0 && k >= 1 && r[k - 1] == 4) {
        r[k - 1] = 12;
        n /= 3;
    }
    while (n % 3 == 0) {
        r[k++] = 3;
        n /= 3;
    }
    return i < k ? r[i] : 0;
}
// The radix plan of schedule variant alt: 0 the plan above, 1 the same radices in
// reverse order (the Stockham passes take any order)
constexpr int radix_at_v(int n, int i, int alt) {
    if (alt == 0) return radix_at(n, i);
    int k = 0;
    while (radix_at(n, k) != 0) ++k;
    return i < k ? radix_at(n, k - 1 - i) : 0;
}
constexpr bool plan_has_alt(int n) {
    int k = 0;
    while (radix_at(n, k) != 0) ++k;
    for (int i = 0; i < k; ++i)
        if (radix_at_v(n, i, 1) != radix_at(n, i)) return true;
    return false;
}
constexpr int num_passes(int n) {
    int k = 0;
    while (radix_at(n, k) != 0) ++k;
    return k;
}
constexpr int plan_product(int n) {
    int p = 1;
    for (int k = 0; radix_at(n, k) != 0; ++k) p *= radix_at(n, k);
    return p;
}
constexpr int pow2_ceil(int v) {
    int p = 1;
    while (p < v) p <<= 1;
    return p;
}

template <int R> __device__ inline void fdft(float2* v, int sign) {
    if constexpr (R == 16) fdft16(v, sign);
    if constexpr (R == 12) fdft12(v, sign);
    if constexpr (R == 2) fdft2(v);
    if constexpr (R == 3) fdft3(v, sign);
    if constexpr (R == 4) fdft4(v, sign);
    if constexpr (R == 8) fdft8(v, sign);
}

// one Stockham pass; LF: consecutive threads take consecutive lines.  GAP > 0
// (with LS = 1): the lines come in runs of GAP with one skipped slot after each
// run, i.e. line l starts at l + l / GAP
template <int R, int N, int NS, int NL, int LS, int ES, int SIGN, bool LF, int GAP = 0>
__device__ inline void cpass(const float2* __restrict__ in, float2* __restrict__ out, const float2* __restrict__ tw) {
    constexpr int NB = N / R;
    constexpr int TOT = NL * NB;
    constexpr int TWS = N / (NS * R);
#pragma unroll 1
    for (int w0 = 0; w0 < TOT; w0 += FUSED_THREADS) {
        const int w = w0 + (int)threadIdx.x;
        if (TOT % FUSED_THREADS == 0 || w < TOT) {
            int line, j;
            if constexpr (LF) {
                j = w / NL;
                line = w - j * NL;
            } else {
                line = w / NB;
                j = w - line * NB;
            }
            const int lo = GAP ? line + line / GAP : line * LS;
            const float2* src = in + lo;
            float2* dst = out + lo;
            float2 v[R];
#pragma unroll
            for (int r = 0; r < R; ++r) v[r] = src[(j + r * NB) * ES];
            const int q = j / NS;
            const int k = j - q * NS;
            if (NS > 1 && k) {
#pragma unroll
                for (int r = 1; r < R; ++r) {
                    float2 t = tw[k * r * TWS];
                    if (SIGN > 0) t.y = -t.y;
                    v[r] = f2mul(v[r], t);
                }
            }
            fdft<R>(v, SIGN);
            const int base = q * NS * R + k;
#pragma unroll
            for (int r = 0; r < R; ++r) dst[(base + r * NS) * ES] = v[r];
        }
    }
}

template <int N, int NL, int LS, int ES, int SIGN, bool LF, int GAP = 0, int ALT = 0, int P = 0, int NS = 1>
__device__ inline float2* cfft(float2* in, float2* out, const float2* tw) {
    static_assert(GAP == 0 || LS == 1, "gapped lines are unit-stride");
    static_assert(plan_product(N) == N, "the radix plan multiplies out to the transform length");
    if constexpr (P == num_passes(N)) {
        return in;
    } else {
        constexpr int R = radix_at_v(N, P, ALT);
        cpass<R, N, NS, NL, LS, ES, SIGN, LF, GAP>(in, out, tw);
        __syncthreads();
        return cfft<N, NL, LS, ES, SIGN, LF, GAP, ALT, P + 1, NS * R>(out, in, tw);
    }
}

// segmented reductions with compile-time mapping (the mapping is described above)
template <int G, int SEGW, int NV>
__device__ inline void cseg_sum(double* v, double* slots) {
    constexpr int SW = SEGW < 64 ? SEGW : 64;
    constexpr int TPR = G * SEGW;
    constexpr int RPS = FUSED_THREADS / TPR;
    constexpr int PER_ROW = TPR / SW, PER_SEG = SEGW / SW;
    constexpr int NSLOT = FUSED_THREADS / SW;
    if constexpr (NV == 1) {
#pragma unroll
        for (int o = SW >> 1; o > 0; o >>= 1) v[0] += __shfl_xor(v[0], o);
        if ((threadIdx.x & (SW - 1)) == 0 && (int)threadIdx.x < RPS * TPR) slots[(threadIdx.x / SW) * 8] = v[0];
    } else {
        // reduce-scatter of up to 8 values over the SW-lane part: three halving
        // exchanges leave value q in the lanes whose bits SW/2, SW/4, SW/8 spell q,
        // the remaining butterflies sum it over those lanes (10 shuffles, not 6 NV)
        static_assert(NV <= 8, "at most 8 values");
        double w[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) w[q] = q < NV ? v[q] : 0.0;
        const int lane = threadIdx.x & (SW - 1);
        int q = 0;
#pragma unroll
        for (int half = 4, o = SW >> 1; half >= 1; half >>= 1, o >>= 1) {
            const bool hi = (lane & o) != 0;
#pragma unroll
            for (int k = 0; k < half; ++k) {
                const double mine = hi ? w[half + k] : w[k];
                const double give = hi ? w[k] : w[half + k];
                w[k] = mine + __shfl_xor(give, o);
            }
            q += hi ? half : 0;
        }
#pragma unroll
        for (int o = SW >> 4; o > 0; o >>= 1) w[0] += __shfl_xor(w[0], o);
        if ((lane & (SW / 8 - 1)) == 0 && q < NV && (int)threadIdx.x < RPS * TPR)
            slots[(threadIdx.x / SW) * 8 + q] = w[0];
    }
    __syncthreads();
    // one thread per (filter, value) sums that filter's slots in a fixed order
    double* res = slots + NSLOT * 8;
    if ((int)threadIdx.x < G * NV) {
        const int g = threadIdx.x / NV, q = threadIdx.x - g * NV;
        double acc = 0.0;
#pragma unroll
        for (int tr = 0; tr < RPS; ++tr)
#pragma unroll
            for (int h = 0; h < PER_SEG; ++h) acc += slots[(tr * PER_ROW + g * PER_SEG + h) * 8 + q];
        res[g * 8 + q] = acc;
    }
    __syncthreads();
    if ((int)threadIdx.x < G)
        for (int q = 0; q < NV; ++q) v[q] = res[threadIdx.x * 8 + q];
}

template <int G, int SEGW>
__device__ inline double cseg_max(double v, double* slots) {
    constexpr int SW = SEGW < 64 ? SEGW : 64;
    constexpr int TPR = G * SEGW;
    constexpr int RPS = FUSED_THREADS / TPR;
#pragma unroll
    for (int o = SW >> 1; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    if ((threadIdx.x & (SW - 1)) == 0 && (int)threadIdx.x < RPS * TPR) slots[(threadIdx.x / SW) * 8] = v;
    __syncthreads();
    if ((int)threadIdx.x < G) {
        const int g = threadIdx.x;
        constexpr int PER_ROW = TPR / SW, PER_SEG = SEGW / SW;
        double r = -INFINITY;
        for (int tr = 0; tr < RPS; ++tr)
            for (int h = 0; h < PER_SEG; ++h) r = fmax(r, slots[(tr * PER_ROW + g * PER_SEG + h) * 8]);
        v = r;
    }
    __syncthreads();
    return v;
}

// thread 0..G-1: normaliser, moments and the new grid of filter tid (FP64, 2x2 scalars)
__device__ void filter_design(FState& F, const double* acc, int NX, int n0, int n1) {
    const FPlan& P = F.p;
    const double S0 = acc[0];
    const double mass = P.vol * S0;
    const double half0 = (double)(n0 / 2), half1 = (double)(n1 / 2);
    F.ok = !P.bad && isfinite(F.s) && isfinite(mass) && mass > 0.0;
    F.bits = 0;
    if (!F.ok) return;
    F.loglik = F.s + log(mass);
    const double iS0 = 1.0 / S0;
    const double ub0 = acc[1] * iS0, ub1 = acc[2] * iS0;
    const double C00 = acc[3] * iS0 - ub0 * ub0;
    const double C11 = acc[4] * iS0 - ub1 * ub1;
    const double C01 = acc[5] * iS0 - ub0 * ub1;
    if (acc[6] * iS0 > BOUNDARY_TOL) F.bits = PMF_W_BOUNDARY;
    double mean0, mean1, cov00, cov11;
    if (NX == 2) {
        mean0 = P.c[0] + P.M[0] * ub0 + P.M[1] * ub1;
        mean1 = P.c[1] + P.M[2] * ub0 + P.M[3] * ub1;
        cov00 = P.M[0] * P.M[0] * C00 + 2.0 * P.M[0] * P.M[1] * C01 + P.M[1] * P.M[1] * C11;
        cov11 = P.M[2] * P.M[2] * C00 + 2.0 * P.M[2] * P.M[3] * C01 + P.M[3] * P.M[3] * C11;
    } else {
        mean0 = P.c[0] + P.M[0] * ub0;
        mean1 = 0.0;
        cov00 = P.M[0] * P.M[0] * C00;
        cov11 = 1.0;
    }
    const double v0 = cov00 + P.Wnom[0];
    const double v1 = (NX == 2) ? cov11 + P.Wnom[1] : 1.0;
    if (!(v0 > 0.0) || !(v1 > 0.0) || !isfinite(v0) || !isfinite(v1)) {
        F.ok = 0;
        return;
    }
    const double d0 = 2.0 * P.span * sqrt(v0) / (NX == 2 ? (double)n0 : (double)n1);
    const double d1 = (NX == 2) ? 2.0 * P.span * sqrt(v1) / (double)n1 : 1.0;
    F.gnc[0] = mean0;
    F.gnc[1] = mean1;
    F.gnM[0] = d0;
    F.gnM[1] = 0.0;
    F.gnM[2] = 0.0;
    F.gnM[3] = d1;
    F.gnvol = (NX == 2) ? d0 * d1 : d0;
    const bool aligned = (NX == 1) || (P.M[1] == 0.0 && P.M[2] == 0.0);
    // separable 2-D and Lagrange 1-D regrids are not fused: reject, flagged
    if ((NX == 2 && P.interp == PMF_INTERP_AUTO && aligned) || (NX == 1 && P.interp != PMF_INTERP_AUTO)) {
        F.ok = 0;
        F.bits = PMF_E_INVALID;
        return;
    }
    // new index coordinates -> old index coordinates: Mi (M' u' + c' - c) + N/2
    const double dc0 = mean0 - P.c[0], dc1 = mean1 - P.c[1];
    if (NX == 2) {
        F.amap[0] = P.Mi[0] * d0;
        F.amap[1] = P.Mi[1] * d1;
        F.amap[2] = P.Mi[2] * d0;
        F.amap[3] = P.Mi[3] * d1;
        F.bmap[0] = P.Mi[0] * dc0 + P.Mi[1] * dc1 + half0;
        F.bmap[1] = P.Mi[2] * dc0 + P.Mi[3] * dc1 + half1;
    } else {
        F.amap[0] = P.Mi[0] * d0;
        F.bmap[0] = P.Mi[0] * dc0 + half1;
    }
}

// thread 0..G-1: write back descriptor and log-likelihood of filter tid (stores
// only: the time and status word come with the plan)
template <int NX>
__device__ void filter_commit(const FState& F, double* ll_out) {
    const FPlan& P = F.p;
    DevDesc* d = F.d;
    Grid gg;
    mat_zero(gg.M);
    for (int q = 0; q < MS; ++q) gg.c[q] = 0.0;
    if (F.ok) {
        gg.c[0] = F.gnc[0];
        gg.c[1] = NX == 2 ? F.gnc[1] : 0.0;
        gg.M[0] = F.gnM[0];
        if (NX == 2) gg.M[MS + 1] = F.gnM[3];
    } else {
        gg.c[0] = P.c[0];
        gg.c[1] = P.c[1];
        gg.M[0] = P.M[0];
        if (NX == 2) {
            gg.M[1] = P.M[1];
            gg.M[MS] = P.M[2];
            gg.M[MS + 1] = P.M[3];
        }
    }
    grid_finish(gg, NX);
    // the batched grid is at most 2 x 2: only that block of the descriptor
    // changes (the rest is zero since the filter was created)
    d->g.c[0] = gg.c[0];
    d->g.c[1] = gg.c[1];
    d->g.M[0] = gg.M[0];
    d->g.M[1] = gg.M[1];
    d->g.M[MS] = gg.M[MS];
    d->g.M[MS + 1] = gg.M[MS + 1];
    d->g.Mi[0] = gg.Mi[0];
    d->g.Mi[1] = gg.Mi[1];
    d->g.Mi[MS] = gg.Mi[MS];
    d->g.Mi[MS + 1] = gg.Mi[MS + 1];
    d->g.vol = gg.vol;
    d->t = P.tnew;
    d->l = P.l;
    d->h = P.h;
    d->etr = P.etr;
    d->par = 1 - P.par;
    if (F.ok) {
        d->loglik = F.loglik;
        d->status = P.status | F.bits;
        d->pscale = F.pscale2;
        ll_out[F.idx] = F.loglik;
    } else {
        d->loglik = NAN;
        d->status = P.status | F.bits | (P.bad ? PMF_E_INVALID : PMF_E_DEGENERATE);
        d->pscale = 1.0;
        ll_out[F.idx] = NAN;
    }
}

// LDS of the fused kernel, at file scope so that the specialised group functions
// address it as LDS (ds_* instructions) rather than through generic pointers
extern __shared__ __align__(16) unsigned char pmf_fsm[];
__shared__ FState pmf_FS[GMAX];
__shared__ double pmf_slots[32 * 8 + GMAX * 8];
__shared__ GItem pmf_gi;   // the workgroup's group, written by thread 0 at the start

typedef __attribute__((address_space(1))) float gfloat;
// The interval's gain constants of one filter, read once per thread from its
// plan in LDS (the gain loops then keep them in registers).  Exact integrator:
// e0 = -gc0/2, e1 = -gc1/2, e2 = -gc2, so that the gain is exp(e0 a2 + e1 b2 +
// e2 a1 b1); RK4 / Euler: substep count and length.
struct GainC {
    int integ, l;
    float h, e0, e1, e2;
};
__device__ inline GainC gain_consts(const FPlan& P) {
    GainC c;
    c.integ = P.integ;
    c.l = P.l;
    c.h = (float)P.h;
    c.e0 = -0.5f * (float)P.gc[0];
    c.e1 = -0.5f * (float)P.gc[1];
    c.e2 = -(float)P.gc[2];
    return c;
}

// spectral gain of one mode over the interval: a2 = k0^2, a1 = k0 (first
// derivative symbol), b2 = k1^2, b1 = k1; exact, or the product over the RK4 /
// Euler substeps of their amplification factors (stage coefficients in cf)
__device__ inline float mode_gain(const GainC& c, const double* cf, float a2, float a1, float b2, float b1) {
    if (c.integ == PMF_INT_EXACT) return __expf(c.e0 * a2 + c.e1 * b2 + c.e2 * a1 * b1);
    const float hh = c.h;
    float g2 = 1.f;
    if (c.integ == PMF_INT_EULER) {
        for (int q = 0; q < c.l; ++q) {
            const float sig = (float)cf[3 * q] * a2 + (float)cf[3 * q + 1] * b2 + 2.f * (float)cf[3 * q + 2] * a1 * b1;
            g2 = g2 / (1.f + 0.5f * hh * sig);
        }
    } else {
        for (int q = 0; q < c.l; ++q) {
            const double* c3 = cf + 6 * q;
            const float la = -0.5f * ((float)c3[0] * a2 + (float)c3[1] * b2 + 2.f * (float)c3[2] * a1 * b1);
            const float lb = -0.5f * ((float)c3[3] * a2 + (float)c3[4] * b2 + 2.f * (float)c3[5] * a1 * b1);
            const float lc = -0.5f * ((float)c3[6] * a2 + (float)c3[7] * b2 + 2.f * (float)c3[8] * a1 * b1);
            const float y2 = 1.f + 0.5f * hh * la;
            const float y3 = 1.f + 0.5f * hh * lb * y2;
            const float y4 = 1.f + hh * lb * y3;
            g2 *= 1.f + hh / 6.f * (la + 2.f * lb * y2 + 2.f * lb * y3 + lc * y4);
        }
    }
    return g2;
}

typedef __attribute__((address_space(1))) const float cgfloat;
typedef __attribute__((address_space(1))) const unsigned long long cgu64;   // a complex pair

template <int N0, int N1, int NX, int G, int TYPE, int ALT>
__device__ __forceinline__ void process_group(const BItem* __restrict__ items, const FPlan* __restrict__ plans,
                                           const double* __restrict__ zall, int nzmax, double* __restrict__ ll_out,
                                           int bufcplx) {
    // the group's first item and size, uniform (scalar registers; no per-thread copy)
    struct {
        int first, count;
    } const GI = {__builtin_amdgcn_readfirstlane(pmf_gi.first), __builtin_amdgcn_readfirstlane(pmf_gi.G)};
    float2* bufA = reinterpret_cast<float2*>(pmf_fsm);
    float2* bufB = bufA + bufcplx;
    float2* twr = bufB + bufcplx;   // 128
    float2* twc = twr + 128;        // 128
    float2* twp = twc + 128;        // 130
    FState* FS = pmf_FS;
    double* slots = pmf_slots;
    // spectra and the predicted density: super-row L = r G + g (row r of filter g)
    // of PITCH complex = RP floats; the 2-D posterior: super-rows of RPO floats
    constexpr int H1 = N1 / 2, PITCH = spec_pitch(N1), SPITCH = G * PITCH, RP = 2 * PITCH, RS = G * RP;
    constexpr int RPO = NX == 2 ? N1 + 1 : RP, RSO = G * RPO;
    constexpr bool GUARD = group_guard(N0, N1, G);
    constexpr int SEGW = pow2_ceil(N1) < 32 ? 32 : pow2_ceil(N1);
    constexpr int TPR = G * SEGW, RPS = FUSED_THREADS / TPR;
    constexpr int NT = FUSED_THREADS;
    const int tid = threadIdx.x;
    const int Gact = GI.count;   // filters present (<= G)

    // plans into LDS, one 8-byte word per thread (one round trip for the group)
    constexpr int PW = sizeof(FPlan) / sizeof(double);
    static_assert(sizeof(FPlan) % sizeof(double) == 0, "FPlan is copied as doubles");
    for (int e = tid; e < G * PW; e += NT) {
        const int g = e / PW, w = e - g * PW;
        const int gg = g < Gact ? g : 0;
        reinterpret_cast<double*>(&FS[g].p)[w] = reinterpret_cast<const double*>(&plans[GI.first + gg])[w];
    }
    if (tid < G) {
        const int gg = tid < Gact ? tid : 0;
        const BItem& I = items[GI.first + gg];
        // the item's fields and the parity loaded independently (one round trip)
        float* const p0 = I.P[0];
        float* const p1 = I.P[1];
        DevDesc* const d = I.d;
        const FConst* const k = I.k;
        const int idx = I.idx;
        const int par = plans[GI.first + gg].par;
        FS[tid].pin = par ? p1 : p0;
        FS[tid].pout = par ? p0 : p1;
        FS[tid].d = d;
        FS[tid].km = &k->m;
        FS[tid].zrow = zall + (size_t)(GI.first + gg) * nzmax;
        FS[tid].idx = idx;
    }
    // twiddle tables of this group type (after both buffers)
    for (int i = tid; i < H1; i += NT) {
        float sn, cs;
        sincospif(-2.0f * i / H1, &sn, &cs);
        twr[i] = make_float2(cs, sn);
    }
    if (NX == 2)
        for (int i = tid; i < N0; i += NT) {
            float sn, cs;
            sincospif(-2.0f * i / N0, &sn, &cs);
            twc[i] = make_float2(cs, sn);
        }
    for (int i = tid; i <= H1; i += NT) {
        float sn, cs;
        sincospif(-2.0f * i / N1, &sn, &cs);
        twp[i] = make_float2(cs, sn);
    }
    __syncthreads();

    // ---- load: super-row L = r*G + g holds row r of filter g as complex pairs.
    // Every load of the thread is issued before the first wait: the addresses are
    // clamped to valid ones (an absent filter reads filter 0, a surplus element the
    // last one) and the values discarded afterwards.
    {
        constexpr int TOT = G * N0 * H1, NE = (TOT + NT - 1) / NT;
        unsigned long long ld[NE];
#pragma unroll
        for (int i = 0; i < NE; ++i) {
            const int e = min(tid + i * NT, TOT - 1);
            const int L = e / H1, k = e - L * H1;
            const int r = L / G, g = L - r * G;
            ld[i] = ((cgu64*)FS[g < Gact ? g : 0].pin)[r * H1 + k];
        }
#pragma unroll
        for (int i = 0; i < NE; ++i) {
            const int e = tid + i * NT;
            if (TOT % NT == 0 || e < TOT) {
                const int L = e / H1, k = e - L * H1;
                const int r = L / G, g = L - r * G;
                // absent filters read filter 0's (finite) values: scaled to zero
                const float sc = g < Gact ? (float)FS[g].p.pscale : 0.f;
                bufA[L * PITCH + k] = make_float2(__uint_as_float((unsigned int)ld[i]) * sc,
                                                  __uint_as_float((unsigned int)(ld[i] >> 32)) * sc);
            }
        }
    }
    __syncthreads();
    // ---- forward: rows (r2c), columns
    float2* cur = cfft<H1, N0 * G, PITCH, 1, -1, true>(bufA, bufB, twr);
    float2* oth = (cur == bufA) ? bufB : bufA;
    // Split of the N1/2-point transforms Z of the rows into the half spectra X of
    // the real rows: with E = (Z_s + conj Z_{H1-s}) / 2, O = (Z_s - conj Z_{H1-s}) / 2
    // and t = W^s O (W = e^{-2 pi i / N1}), X_s = E - i t and X_{H1-s} = conj E - i conj t,
    // so one thread makes both entries of a pair (s, H1 - s) from the same two loads.
    // The DC and Nyquist entries are real, X_0 = Re Z_0 + Im Z_0 and X_H1 = Re Z_0 - Im Z_0;
    // in 2-D they are stored packed as X_0 + i X_H1 in entry 0, so that the column
    // transforms run over H1 columns per filter (entry H1 is not used)
    constexpr int HP = H1 / 2 + 1;             // pairs (s, H1 - s), s = 0 .. H1/2, per row
#pragma unroll 1
    for (int e = tid; e < N0 * G * HP; e += NT) {
        const int L = e / HP, s = e - L * HP;
        const float2* zr = cur + L * PITCH;
        float2* xr = oth + L * PITCH;
        if (s == 0) {
            const float2 Z0 = zr[0];
            if constexpr (NX == 2) {
                xr[0] = make_float2(Z0.x + Z0.y, Z0.x - Z0.y);
            } else {
                xr[0] = make_float2(Z0.x + Z0.y, 0.f);
                xr[H1] = make_float2(Z0.x - Z0.y, 0.f);
            }
        } else {
            const float2 Zs = zr[s], Zc = f2conj(zr[H1 - s]);
            const float2 E = f2scale(f2add(Zs, Zc), 0.5f);
            const float2 t = f2mul(twp[s], f2scale(f2sub(Zs, Zc), 0.5f));
            xr[s] = make_float2(E.x + t.y, E.y - t.x);
            if (2 * s != H1) xr[H1 - s] = make_float2(E.x - t.y, -E.y - t.x);
        }
    }
    __syncthreads();
    cur = oth;
    oth = (cur == bufA) ? bufB : bufA;
    if constexpr (NX == 2) {
        cur = cfft<N0, G * H1, 1, SPITCH, -1, true, H1, ALT>(cur, oth, twc);
        oth = (cur == bufA) ? bufB : bufA;
    }
    // ---- per-mode gain with 1/(N0 N1) of the unnormalised transforms.  2-D: the
    // last wave takes the packed DC/Nyquist columns, the other waves the remaining
    // columns, a thread owning one column (filter g, frequency s1) and walking its
    // rows (no wave mixes the two kinds)
    {
        constexpr float inv = 1.0f / ((float)N0 * (float)N1);
        auto rowk = [](int s0, float& a2, float& a1) {
            const int kk = (s0 < N0 / 2) ? s0 : s0 - N0;
            const float kap = (6.283185307179586f / N0) * kk;
            a2 = kap * kap;
            a1 = (2 * s0 == N0) ? 0.f : kap;
        };
        if constexpr (NX == 2) {
            constexpr int CWN = H1 - 1;       // columns 1 .. H1-1 of each filter
            constexpr int NCOLN = G * CWN;
            constexpr int TN = NT - 64;
            constexpr int CPS = TN / NCOLN;   // rows walked in parallel per column
            static_assert(CPS >= 1, "a thread per column");
            if (tid < TN) {
                const int cth = tid % NCOLN, r0 = tid / NCOLN;
                if (r0 < CPS) {
                    const int g = cth / CWN, s1 = 1 + cth - g * CWN;
                    const GainC gc = gain_consts(FS[g].p);
                    const float scale = (float)FS[g].p.etr * inv;
                    const float kap1 = (6.283185307179586f / N1) * s1;
                    float2* colp = cur + g * PITCH + s1;
                    if (gc.integ == PMF_INT_EXACT) {
                        // exp(e0 a2 + e2 kap1 a1 + e1 kap1^2): the column's part once
                        const float cb = gc.e1 * (kap1 * kap1), cx = gc.e2 * kap1;
                        for (int s0 = r0; s0 < N0; s0 += CPS) {
                            float a2, a1;
                            rowk(s0, a2, a1);
                            float2* x = colp + s0 * SPITCH;
                            *x = f2scale(*x, __expf(fmaf(gc.e0, a2, fmaf(cx, a1, cb))) * scale);
                        }
                    } else {
                        const double* cf = items[GI.first + (g < Gact ? g : 0)].coef;
                        for (int s0 = r0; s0 < N0; s0 += CPS) {
                            float a2, a1;
                            rowk(s0, a2, a1);
                            float2* x = colp + s0 * SPITCH;
                            *x = f2scale(*x, mode_gain(gc, cf, a2, a1, kap1 * kap1, kap1) * scale);
                        }
                    }
                }
            } else {
                // packed column Z = A + i B, A and B the column spectra of the real
                // DC and Nyquist columns; their gains gd, gn are even in the row
                // frequency (no cross term: the first-derivative symbol of both is
                // zero), so Z'[k] = (gd + gn)/2 Z[k] + (gd - gn)/2 conj Z[N0 - k];
                // one (filter, pair k <-> N0 - k) per lane
                constexpr int PAIRS = N0 / 2 + 1;
                const float kn = 3.14159265358979f;   // |kappa_1| at the Nyquist index
                for (int e = tid - TN; e < G * PAIRS; e += 64) {
                    const int g = e / PAIRS, s0 = e - g * PAIRS;
                    const GainC gc = gain_consts(FS[g].p);
                    const double* cf = items[GI.first + (g < Gact ? g : 0)].coef;
                    const float scale = (float)FS[g].p.etr * inv;
                    const int m = s0 == 0 ? 0 : N0 - s0;
                    float a2, a1;
                    rowk(s0, a2, a1);
                    const float gd = mode_gain(gc, cf, a2, a1, 0.f, 0.f);
                    const float gn = mode_gain(gc, cf, a2, a1, kn * kn, 0.f);
                    const float pa = 0.5f * (gd + gn) * scale, pb = 0.5f * (gd - gn) * scale;
                    float2* x = cur + s0 * SPITCH + g * PITCH;
                    float2* y = cur + m * SPITCH + g * PITCH;
                    const float2 zk = *x, zm = *y;
                    *x = f2add(f2scale(zk, pa), f2scale(f2conj(zm), pb));
                    if (m != s0) *y = f2add(f2scale(zm, pa), f2scale(f2conj(zk), pb));
                }
            }
        } else {
            // 1-D: a thread per spectral entry (filter g, frequency s1)
            for (int cth = tid; cth < SPITCH; cth += NT) {
                const int g = cth / PITCH, s1 = cth - g * PITCH;
                const GainC gc = gain_consts(FS[g].p);
                const double* cf = items[GI.first + (g < Gact ? g : 0)].coef;
                const int kk1 = (s1 < H1) ? s1 : s1 - N1;
                const float kap1 = (6.283185307179586f / N1) * kk1;
                const float a1 = (s1 == H1) ? 0.f : kap1;
                float2* x = cur + cth;
                *x = f2scale(*x, mode_gain(gc, cf, kap1 * kap1, a1, 0.f, 0.f) * (float)FS[g].p.etr * inv);
            }
        }
    }
    __syncthreads();
    // ---- inverse: columns, rows (c2r)
    if constexpr (NX == 2) {
        cur = cfft<N0, G * H1, 1, SPITCH, +1, true, H1, ALT>(cur, oth, twc);
        oth = (cur == bufA) ? bufB : bufA;
    }
    // Merge of the half spectra X into the N1/2-point inverse inputs Z, per pair
    // (s, H1 - s): with A = X_s + conj X_{H1-s}, B = X_s - conj X_{H1-s} and
    // u = conj(W^s) B, Z_s = A + i u and Z_{H1-s} = conj A + i conj u.  Entry 0 (2-D:
    // the packed X_0 + i X_H1, both real) gives Z_0 = (X_0 + X_H1) + i (X_0 - X_H1).
#pragma unroll 1
    for (int e = tid; e < N0 * G * HP; e += NT) {
        const int L = e / HP, s = e - L * HP;
        const float2* xr = cur + L * PITCH;
        float2* zr = oth + L * PITCH;
        if (s == 0) {
            const float2 X0 = xr[0];
            if constexpr (NX == 2) {
                zr[0] = make_float2(X0.x + X0.y, X0.x - X0.y);
            } else {
                const float2 XH = f2conj(xr[H1]);
                const float2 A = f2add(X0, XH), Bv = f2sub(X0, XH);
                zr[0] = make_float2(A.x - Bv.y, A.y + Bv.x);
            }
        } else {
            const float2 Xs = xr[s], Xc = f2conj(xr[H1 - s]);
            const float2 A = f2add(Xs, Xc);
            const float2 u = f2mul(f2conj(twp[s]), f2sub(Xs, Xc));
            zr[s] = make_float2(A.x - u.y, A.y + u.x);
            if (2 * s != H1) zr[H1 - s] = make_float2(A.x + u.y, u.x - A.y);
        }
    }
    __syncthreads();
    cur = cfft<H1, N0 * G, PITCH, 1, +1, true>(oth, cur, twr);
    oth = (cur == bufA) ? bufB : bufA;
    const float* Pr = reinterpret_cast<const float*>(cur);   // predicted: (r, g, j) at r*RS + g*RP + j
    // posterior (2-D): super-rows of RPO = N1 + 1 floats after one float (and,
    // with GUARD, after the super-row set of row -1); that float, the last float
    // of every super-row and the guard rows -1 and N0 are zeroed here (positions
    // the likelihood pass does not write, so no barrier is needed): a stencil tap
    // one column left or right of a row, or one row above or below the grid,
    // reads zero
    constexpr int PO_OFF = NX == 2 ? (GUARD ? RSO + 1 : 1) : 0;
    float* Po = reinterpret_cast<float*>(oth) + PO_OFF;
    if constexpr (NX == 2) {
        for (int e = tid; e < PO_OFF; e += NT) Po[e - PO_OFF] = 0.f;
        if (GUARD)
            for (int e = tid; e < RSO; e += NT) Po[N0 * RSO + e] = 0.f;
        for (int e = tid; e < N0 * G; e += NT) Po[e * RPO + N1] = 0.f;
    }

    // ---- likelihood (FP64 Horner in u0 per thread), shift, multiply, FP64 sums
    const int tr = tid / TPR;
    const int tt = tid - tr * TPR;
    const int g = tt / SEGW;
    const int j = tt - g * SEGW;
    const bool act = tr < RPS && j < N1 && g < Gact;
    constexpr double half0 = (double)(N0 / 2), half1 = (double)(N1 / 2);
    const int gi = act ? g : 0;
    const double* zg = FS[gi].zrow;
    const KModel& mg = *FS[gi].km;
    const FPlan& Pg = FS[gi].p;
    // log l = alpha + beta u0 + gamma u0^2 along this thread's rows (fast path)
    const double uj = (double)j - half1;
    double al, be, ga;
    if (NX == 2) {
        al = Pg.q0 + Pg.qb[1] * uj - 0.5 * Pg.qQ[1] * uj * uj;
        be = Pg.qb[0] - Pg.qQ[2] * uj;
        ga = -0.5 * Pg.qQ[0];
    } else {
        al = Pg.q0;
        be = Pg.qb[0];
        ga = -0.5 * Pg.qQ[0];
    }
    double mx = -INFINITY;
    const double u0first = (NX == 2) ? (double)tr - half0 : uj;
    constexpr double du0 = (NX == 2) ? (double)RPS : 0.0;
    if (act) {
        if (Pg.fast && (NX == 1 || ga < 0.0)) {
            // a concave quadratic along this thread's rows u0 = u0first + k RPS:
            // its maximum over them sits at the row nearest the vertex (or a
            // neighbour, within rounding)
            const int cnt = (N0 - tr + RPS - 1) / RPS;
            int ks = 0;
            if (NX == 2) {
                const double kv = (-be / (2.0 * ga) - u0first) / du0;
                ks = kv <= 0.0 ? 0 : (kv >= (double)(cnt - 1) ? cnt - 1 : (int)rint(kv));
            }
            for (int k = ks - 1; k <= ks + 1; ++k)
                if (k >= 0 && k < cnt) mx = fmax(mx, qpoly(al, be, ga, u0first + (double)k * du0));
        } else {
            double u0 = u0first;
            for (int r = tr; r < N0; r += RPS, u0 += du0) {
                const double L = Pg.fast ? qpoly(al, be, ga, u0) : floglik_general(mg, Pg, u0, NX == 2 ? uj : 0.0, zg);
                mx = fmax(mx, L);
            }
        }
    }
    mx = cseg_max<G, SEGW>(mx, slots);
    if (tid < G) FS[tid].s = mx;
    __syncthreads();
    double acc[4] = {0, 0, 0, 0};   // sum w, sum w u0, sum w u0^2, boundary
    if (act) {
        const double sh = FS[g].s;
        const bool jedge = (j == 0 || j == N1 - 1);
        double u0 = u0first;
        const float* pr = Pr + tr * RS + g * RP + j;
        float* po = Po + tr * RSO + g * RPO + j;
        for (int r = tr; r < N0; r += RPS, u0 += du0, pr += RPS * RS, po += RPS * RSO) {
            const double L = Pg.fast ? qpoly(al, be, ga, u0) : floglik_general(mg, Pg, u0, NX == 2 ? uj : 0.0, zg);
            const float v = *pr * __expf((float)(L - sh));
            *po = v;
            const double w = (double)v;
            acc[0] += w;
            acc[1] += w * u0;
            acc[2] += w * u0 * u0;
            if (jedge) acc[3] += w;
        }
        if (NX == 2 && !jedge) {
            // rows 0 and N0-1 are on the boundary too
            if (tr == 0) acc[3] += (double)Po[g * RPO + j];
            if ((N0 - 1) % RPS == tr) acc[3] += (double)Po[(N0 - 1) * RSO + g * RPO + j];
        }
    }
    // per-thread sums -> the seven moment sums (u1 is constant per thread in 2-D)
    double red[7];
    if (NX == 2) {
        red[0] = acc[0];
        red[1] = acc[1];
        red[2] = uj * acc[0];
        red[3] = acc[2];
        red[4] = uj * uj * acc[0];
        red[5] = uj * acc[1];
        red[6] = acc[3];
    } else {
        red[0] = acc[0];
        red[1] = acc[1];
        red[2] = 0.0;
        red[3] = acc[2];
        red[4] = 0.0;
        red[5] = 0.0;
        red[6] = acc[3];
    }
    if (!act)
        for (int q = 0; q < 7; ++q) red[q] = 0.0;
    cseg_sum<G, SEGW, 7>(red, slots);
    if (tid < Gact) filter_design(FS[tid], red, NX, N0, N1);
    __syncthreads();

    // ---- interpolation of the unnormalised posterior onto the new grid, straight to
    // HBM: the stored values are normalised lazily, by the pending scale 1/(vol' sum)
    // of the new grid's sum, which absorbs the posterior's own normaliser too
    double macc[1] = {0.0};
    // rows shorter than their thread segment (N1 = 48, 96) are enumerated flat,
    // point p = r N1 + j over all RPS x SEGW threads of the filter, so that no
    // lane idles
    constexpr bool FLAT = NX == 2 && N1 < SEGW;
    if ((FLAT ? (tr < RPS && g < Gact) : act) && FS[g].ok) {
        const FState& F = FS[g];
        gfloat* Pout = (gfloat*)F.pout;
        const float* Pog = Po + g * RPO;
        if constexpr (NX == 2) {
            // the top-left tap (row -1, column -1) of node (0, 0)'s stencil (guard layouts only)
            const StencilRows<RSO> rows((lcfloat*)(Pog - (GUARD ? RSO + 1 : 0)));
            // the cubic interpolant of the posterior at old index coordinates (nu0, nu1)
            auto interp_at = [&](double nu0, double nu1) -> float {
                float val = 0.f;
                if (nu0 >= 0.0 && nu0 <= (double)(N0 - 1) && nu1 >= 0.0 && nu1 <= (double)(N1 - 1)) {
                    // stencil base at most N - 2: on the last node the weights are
                    // exactly (0, 0, 1, 0), the node's value as with base N - 1
                    const int i0 = min((int)nu0, N0 - 2), i1 = min((int)nu1, N1 - 2);   // floor: nu >= 0
                    float w0[4], w1[4];
                    cubic_weights((float)(nu0 - i0), w0);
                    cubic_weights((float)(nu1 - i1), w1);
                    // taps outside the grid are zero: columns -1 and N1 read the zero
                    // pad floats, rows -1 and N0 the zero guard rows (without GUARD
                    // they get weight zero and read rows 0 and N0 - 1 instead)
                    if constexpr (GUARD) {
                        val = rows.apply(__umul24(i0, RSO) + (unsigned)i1, w0, w1);
                    } else {
                        const float* q = Pog + __umul24(i0, RSO) + (i1 - 1);
                        const bool top = i0 == 0, bot = i0 == N0 - 2;
                        if (top) w0[0] = 0.f;
                        if (bot) w0[3] = 0.f;
                        const float* rows[4] = {top ? q : q - RSO, q, q + RSO, bot ? q + RSO : q + 2 * RSO};
#pragma unroll
                        for (int a = 0; a < 4; ++a) {
                            const float* row = rows[a];
                            val += w0[a] * (w1[0] * row[0] + w1[1] * row[1] + w1[2] * row[2] + w1[3] * row[3]);
                        }
                    }
                }
                return val;
            };
            if constexpr (FLAT) {
                constexpr int STEP = RPS * SEGW;
#pragma unroll 2
                for (int p = tr * SEGW + j; p < N0 * N1; p += STEP) {
                    const int r = p / N1, c = p - r * N1;
                    const double u0 = (double)r - half0, u1 = (double)c - half1;
                    const float val = interp_at(F.amap[0] * u0 + F.amap[1] * u1 + F.bmap[0],
                                                F.amap[2] * u0 + F.amap[3] * u1 + F.bmap[1]);
                    Pout[p] = val;
                    macc[0] += (double)val;
                }
            } else {
                // old index coordinates of new node (r, j), advanced by RPS rows per step
                double nu0 = F.amap[0] * ((double)tr - half0) + F.amap[1] * uj + F.bmap[0];
                double nu1 = F.amap[2] * ((double)tr - half0) + F.amap[3] * uj + F.bmap[1];
                const double dn0 = F.amap[0] * RPS, dn1 = F.amap[2] * RPS;
#pragma unroll 2
                for (int r = tr; r < N0; r += RPS, nu0 += dn0, nu1 += dn1) {
                    const float val = interp_at(nu0, nu1);
                    Pout[r * N1 + j] = val;
                    macc[0] += (double)val;
                }
            }
        } else {
            const double nu = F.amap[0] * uj + F.bmap[0];
            float val = 0.f;
            if (nu >= 0.0 && nu <= (double)(N1 - 1)) val = trig_interp_1d(Pog, N1, nu);
            Pout[j] = val;
            macc[0] += (double)val;
        }
    }
    cseg_sum<G, SEGW, 1>(macc, slots);
    if (tid < Gact) {
        FState& F = FS[tid];
        if (F.ok) {
            const double mass2 = F.gnvol * macc[0];
            if (!(mass2 > 0.0) || !isfinite(mass2)) F.ok = 0;
            else F.pscale2 = 1.0 / mass2;
        }
    }
    __syncthreads();
    // ---- rejected updates keep the predicted density and the moved grid
    if (act && !FS[g].ok) {
        gfloat* Pout = (gfloat*)FS[g].pout;
        for (int r = tr; r < N0; r += RPS) Pout[r * N1 + j] = Pr[r * RS + g * RP + j];
    }
    if (tid < Gact) filter_commit<NX>(FS[tid], ll_out);
    __syncthreads();
}

// group types served by the fused kernel
enum {
    GT_2D_128, GT_2D_96, GT_2D_64, GT_2D_48, GT_2D_32,
    GT_1D_256, GT_1D_192, GT_1D_128, GT_1D_96, GT_1D_64, GT_1D_48, GT_1D_32,
    // rectangular 2-D grids N0 x N1 (N0 != N1, both in 128, 96, 64, 48, 32):
    // GT_2R + 5 i0 + i1 with i the position in that list (the diagonal unused)
    GT_2R, GT_COUNT = GT_2R + 25
};
static_assert(GT_COUNT <= 40, "pmf_ctx::sched holds one entry per group type");

constexpr int size_index_c(int n) { return n == 128 ? 0 : n == 96 ? 1 : n == 64 ? 2 : n == 48 ? 3 : n == 32 ? 4 : -1; }
constexpr int rect_type(int n0, int n1) { return GT_2R + 5 * size_index_c(n0) + size_index_c(n1); }

template <int N0, int N1>
constexpr int group_g() {
    constexpr int seg = pow2_ceil(N1) < 32 ? 32 : pow2_ceil(N1);
    int G = 1;
    while (G < GMAX && group_cplx(N0, N1, 2 * G) <= CPLX_BUDGET && (2 * G) * seg <= FUSED_THREADS) G *= 2;
    return G;
}

// Schedule variants of a group type (2 bits): bit 0 halves the filters per
// workgroup (when more than one fits), bit 1 reverses the radix order of the
// column transforms (when that changes the plan).  The autotuner picks one per
// type; 0 is the default.
constexpr int SCHED_HALF_G = 1, SCHED_COL_ALT = 2, NSCHED = 4;
template <int N0, int N1>
constexpr int group_g_v(int v) {
    return (v & SCHED_HALF_G) && group_g<N0, N1>() > 1 ? group_g<N0, N1>() / 2 : group_g<N0, N1>();
}

__global__ void __launch_bounds__(FUSED_THREADS)
k_fused(const GItem* __restrict__ groups, const BItem* __restrict__ items, const FPlan* __restrict__ plans,
        const double* __restrict__ zall, int nzmax, double* __restrict__ ll_out, int bufcplx) {
    // One workgroup per group: the dispatcher hands the groups out in launch
    // order, largest grids first, as compute units free up.  Each group type's
    // function is inlined into its own branch, so no call saves and restores
    // registers through scratch memory (a persistent loop over claimed groups
    // needed the group functions out of line: inlined into the loop, the
    // compiler kept their loop-invariant addressing live across all of them)
    if (threadIdx.x == 0) pmf_gi = groups[blockIdx.x];
    __syncthreads();
    {
        const int type = __builtin_amdgcn_readfirstlane(pmf_gi.type);
        // group record type = base type * NSCHED + schedule variant
#define PMF_GROUP_V(T, N0, N1, NX, V)                                                                       \
    case T * NSCHED + V:                                                                                    \
        process_group<N0, N1, NX, group_g_v<N0, N1>(V), T, (V & SCHED_COL_ALT) ? 1 : 0>(items, plans, zall, \
                                                                                        nzmax, ll_out, bufcplx); \
        break;
#define PMF_GROUP_2D(T, N)           \
    PMF_GROUP_V(T, N, N, 2, 0)       \
    PMF_GROUP_V(T, N, N, 2, 1)       \
    PMF_GROUP_V(T, N, N, 2, 2)       \
    PMF_GROUP_V(T, N, N, 2, 3)
        switch (type) {
            PMF_GROUP_2D(GT_2D_128, 128)
            PMF_GROUP_2D(GT_2D_96, 96)
            PMF_GROUP_2D(GT_2D_64, 64)
            PMF_GROUP_2D(GT_2D_48, 48)
            PMF_GROUP_2D(GT_2D_32, 32)
            PMF_GROUP_V(GT_1D_256, 1, 256, 1, 0)
            PMF_GROUP_V(GT_1D_192, 1, 192, 1, 0)
            PMF_GROUP_V(GT_1D_128, 1, 128, 1, 0)
            PMF_GROUP_V(GT_1D_96, 1, 96, 1, 0)
            PMF_GROUP_V(GT_1D_64, 1, 64, 1, 0)
            PMF_GROUP_V(GT_1D_48, 1, 48, 1, 0)
            PMF_GROUP_V(GT_1D_32, 1, 32, 1, 0)
            // rectangular 2-D grids: the default schedule only
            PMF_GROUP_V(rect_type(128, 96), 128, 96, 2, 0)
            PMF_GROUP_V(rect_type(128, 64), 128, 64, 2, 0)
            PMF_GROUP_V(rect_type(128, 48), 128, 48, 2, 0)
            PMF_GROUP_V(rect_type(128, 32), 128, 32, 2, 0)
            PMF_GROUP_V(rect_type(96, 128), 96, 128, 2, 0)
            PMF_GROUP_V(rect_type(96, 64), 96, 64, 2, 0)
            PMF_GROUP_V(rect_type(96, 48), 96, 48, 2, 0)
            PMF_GROUP_V(rect_type(96, 32), 96, 32, 2, 0)
            PMF_GROUP_V(rect_type(64, 128), 64, 128, 2, 0)
            PMF_GROUP_V(rect_type(64, 96), 64, 96, 2, 0)
            PMF_GROUP_V(rect_type(64, 48), 64, 48, 2, 0)
            PMF_GROUP_V(rect_type(64, 32), 64, 32, 2, 0)
            PMF_GROUP_V(rect_type(48, 128), 48, 128, 2, 0)
            PMF_GROUP_V(rect_type(48, 96), 48, 96, 2, 0)
            PMF_GROUP_V(rect_type(48, 64), 48, 64, 2, 0)
            PMF_GROUP_V(rect_type(48, 32), 48, 32, 2, 0)
            PMF_GROUP_V(rect_type(32, 128), 32, 128, 2, 0)
            PMF_GROUP_V(rect_type(32, 96), 32, 96, 2, 0)
            PMF_GROUP_V(rect_type(32, 64), 32, 64, 2, 0)
            PMF_GROUP_V(rect_type(32, 48), 32, 48, 2, 0)
            default: break;
        }
#undef PMF_GROUP_2D
#undef PMF_GROUP_V
    }
}

// host copy of the group sizes / types
static int size_index(int n) {
    switch (n) {
        case 128: return 0;
        case 96: return 1;
        case 64: return 2;
        case 48: return 3;
        case 32: return 4;
    }
    return -1;
}

static int group_type(int nx, int n0, int n1) {
    if (nx == 2 && n0 != n1) {
        const int i0 = size_index(n0), i1 = size_index(n1);
        return (i0 < 0 || i1 < 0) ? -1 : GT_2R + 5 * i0 + i1;
    }
    if (nx == 2 && n0 == n1) {
        switch (n1) {
            case 128: return GT_2D_128;
            case 96: return GT_2D_96;
            case 64: return GT_2D_64;
            case 48: return GT_2D_48;
            case 32: return GT_2D_32;
        }
    }
    if (nx == 1) {
        switch (n1) {
            case 256: return GT_1D_256;
            case 192: return GT_1D_192;
            case 128: return GT_1D_128;
            case 96: return GT_1D_96;
            case 64: return GT_1D_64;
            case 48: return GT_1D_48;
            case 32: return GT_1D_32;
        }
    }
    return -1;
}

// the schedule variants offered for a group type (those that differ from the default)
static bool sched_offered(int type, int v) {
    if (v == 0) return true;
    int gmax = 1;
    bool alt = false;
    switch (type) {
        case GT_2D_128: gmax = group_g<128, 128>(); alt = plan_has_alt(128); break;
        case GT_2D_96: gmax = group_g<96, 96>(); alt = plan_has_alt(96); break;
        case GT_2D_64: gmax = group_g<64, 64>(); alt = plan_has_alt(64); break;
        case GT_2D_48: gmax = group_g<48, 48>(); alt = plan_has_alt(48); break;
        case GT_2D_32: gmax = group_g<32, 32>(); alt = plan_has_alt(32); break;
        default: return false;   // 1-D types: the default schedule only
    }
    if ((v & SCHED_HALF_G) && gmax < 2) return false;
    if ((v & SCHED_COL_ALT) && !alt) return false;
    return true;
}

static int group_capacity(int type, int v) {
    switch (type) {
        case GT_2D_128: return group_g_v<128, 128>(v);
        case GT_2D_96: return group_g_v<96, 96>(v);
        case GT_2D_64: return group_g_v<64, 64>(v);
        case GT_2D_48: return group_g_v<48, 48>(v);
        case GT_2D_32: return group_g_v<32, 32>(v);
        case GT_1D_256: return group_g<1, 256>();
        case GT_1D_192: return group_g<1, 192>();
        case GT_1D_128: return group_g<1, 128>();
        case GT_1D_96: return group_g<1, 96>();
        case GT_1D_64: return group_g<1, 64>();
        case GT_1D_48: return group_g<1, 48>();
        case GT_1D_32: return group_g<1, 32>();
        case rect_type(128, 96): return group_g<128, 96>();
        case rect_type(128, 64): return group_g<128, 64>();
        case rect_type(128, 48): return group_g<128, 48>();
        case rect_type(128, 32): return group_g<128, 32>();
        case rect_type(96, 128): return group_g<96, 128>();
        case rect_type(96, 64): return group_g<96, 64>();
        case rect_type(96, 48): return group_g<96, 48>();
        case rect_type(96, 32): return group_g<96, 32>();
        case rect_type(64, 128): return group_g<64, 128>();
        case rect_type(64, 96): return group_g<64, 96>();
        case rect_type(64, 48): return group_g<64, 48>();
        case rect_type(64, 32): return group_g<64, 32>();
        case rect_type(48, 128): return group_g<48, 128>();
        case rect_type(48, 96): return group_g<48, 96>();
        case rect_type(48, 64): return group_g<48, 64>();
        case rect_type(48, 32): return group_g<48, 32>();
        case rect_type(32, 128): return group_g<32, 128>();
        case rect_type(32, 96): return group_g<32, 96>();
        case rect_type(32, 64): return group_g<32, 64>();
        case rect_type(32, 48): return group_g<32, 48>();
    }
    return 0;
}

// density *= pending scale (one block), then the scale is cleared
__global__ void k_apply_pscale(float* P, int n, DevDesc* d) {
    const float s = (float)d->pscale;
    for (int i = threadIdx.x; i < n; i += blockDim.x) P[i] *= s;
    __syncthreads();
    if (threadIdx.x == 0) d->pscale = 1.0;
}

}  // namespace pmf

// ==================================================================== host side

struct BatchCache {
    std::vector<pmf_filter*> filters;
    double T = 0.0;
    hipStream_t stream = nullptr;
    int n = 0, nzmax = 1, ngroups = 0;
    pmf::BItem* d_items = nullptr;
    pmf::GItem* d_groups = nullptr;
    pmf::FPlan* d_plans = nullptr;
    pmf::FConst* d_consts = nullptr;
    double* d_z = nullptr;
    double* d_ll = nullptr;
    // z staging: step k writes slot k % ZSLOTS of mapped pinned memory, which its
    // planning kernel reads.  An event is recorded after every ZEVERY-th step only
    // (an event costs several microseconds of GPU time between steps); before
    // step k overwrites its slot it waits on the event of a step in
    // [k - ZSLOTS, k - ZEVERY - 1], which also covers step k - ZSLOTS.
    static constexpr int ZSLOTS = 8, ZEVERY = 4;
    double* h_z[ZSLOTS] = {};                 // pinned staging of z
    double* hz_dev[ZSLOTS] = {};              // the same memory as the device reads it
    hipEvent_t ev[2] = {nullptr, nullptr};    // alternate over groups of ZEVERY steps
    long long step = 0;
    size_t lds = 0;
    int grid = 0, bufcplx = 0;
    std::vector<int> order;                   // filter index of each item
    long long leaves_seen = -1;               // pmf_ctx::batch_leaves when all filters last entered
    // pmf_batch_run: K steps captured into one graph, replayed on a private stream
    int run_k = 0;
    hipStream_t run_st = nullptr;
    hipGraph_t run_graph = nullptr;
    hipGraphExec_t run_exec = nullptr;
    double* d_zrun = nullptr;                 // K rows of n * nzmax, item order
    double* d_llrun = nullptr;                // K rows of n, item order
    double* h_zrun = nullptr;                 // pinned staging of both
    double* h_llrun = nullptr;
    hipEvent_t run_ev = nullptr;
};

namespace pmf {

// the captured K-step graph and its buffers (the private stream stays)
static void run_free(pmf_ctx* ctx, BatchCache* c) {
    if (c->run_exec) (void)hipGraphExecDestroy(c->run_exec);
    if (c->run_graph) (void)hipGraphDestroy(c->run_graph);
    ctx_free(ctx, c->d_zrun, nullptr);
    ctx_free(ctx, c->d_llrun, nullptr);
    if (c->h_zrun) (void)hipHostFree(c->h_zrun);
    if (c->h_llrun) (void)hipHostFree(c->h_llrun);
    c->run_exec = nullptr;
    c->run_graph = nullptr;
    c->d_zrun = c->d_llrun = c->h_zrun = c->h_llrun = nullptr;
    c->run_k = 0;
}

static void cache_free(pmf_ctx* ctx, BatchCache* c) {
    if (!c) return;
    (void)hipDeviceSynchronize();
    ctx_free(ctx, c->d_items, nullptr);
    ctx_free(ctx, c->d_groups, nullptr);
    ctx_free(ctx, c->d_plans, nullptr);
    ctx_free(ctx, c->d_consts, nullptr);
    ctx_free(ctx, c->d_z, nullptr);
    ctx_free(ctx, c->d_ll, nullptr);
    for (int i = 0; i < BatchCache::ZSLOTS; ++i)
        if (c->h_z[i]) (void)hipHostFree(c->h_z[i]);
    for (int i = 0; i < 2; ++i)
        if (c->ev[i]) (void)hipEventDestroy(c->ev[i]);
    run_free(ctx, c);
    if (c->run_st) (void)hipStreamDestroy(c->run_st);
    if (c->run_ev) (void)hipEventDestroy(c->run_ev);
    delete c;
}

void batch_cache_release(pmf_ctx* ctx) {
    cache_free(ctx, ctx->batch);
    ctx->batch = nullptr;
}

void batch_forget_filter(pmf_ctx* ctx, pmf_filter* f) {
    if (!ctx->batch) return;
    for (pmf_filter* g : ctx->batch->filters)
        if (g == f) {
            batch_cache_release(ctx);
            return;
        }
}

// A filter's density lives in buffer desc->par, scaled lazily by desc->pscale,
// while it takes batched steps; bring it back before the generic kernels run.
hipError_t batch_leave(pmf_filter* f) {
    if (!f->in_batch) return hipSuccess;
    hipError_t e = hipDeviceSynchronize();
    int par = 0;
    if (e == hipSuccess) e = hipMemcpy(&par, &f->desc->par, sizeof(int), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_apply_pscale, dim3(1), dim3(1024), 0, nullptr, static_cast<float*>(f->buf[par]), f->ntot,
                       f->desc);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) return e;
    f->cur = par;
    f->in_batch = false;
    ++f->ctx->batch_leaves;
    return hipSuccess;
}

static hipError_t batch_enter(pmf_filter* f) {
    if (f->in_batch) return hipSuccess;
    hipError_t e = hipDeviceSynchronize();
    int par = 0;
    if (e == hipSuccess) e = hipMemcpy(&par, &f->desc->par, sizeof(int), hipMemcpyDeviceToHost);
    if (e == hipSuccess && f->cur != par)
        e = hipMemcpy(f->buf[par], f->buf[f->cur], (size_t)f->ntot * f->es, hipMemcpyDeviceToDevice);
    if (e != hipSuccess) return e;
    f->cur = par;
    f->in_batch = true;
    return hipSuccess;
}

bool batch_fusable(const pmf_filter* f, std::string* why) { return model_fusable(f->model, why); }

bool model_fusable(const pmf_model& m, std::string* why) {
    if (m.grid != PMF_GRID_FOURIER) return *why = "Chebyshev grid", false;
    if (m.precision != PMF_FP32) return *why = "FP64 density", false;
    if (m.integrator == PMF_INT_FDM || m.integrator == PMF_INT_SINE)
        return *why = "finite-difference or sine-series time update", false;
    if (m.meas_kind == PMF_H_TERRAIN) return *why = "terrain measurement", false;
    if (m.nx > 2) return *why = "nx > 2", false;
    if (m.nx == 2 && (m.N[0] > 128 || m.N[1] > 128)) return *why = "2-D N above 128", false;
    if (m.nx == 1 && m.N[0] > 256) return *why = "1-D N above 256", false;
    if (m.nx == 2 && m.interp == PMF_INTERP_AUTO && m.A[1] == 0.0 && m.A[2] == 0.0)
        return *why = "diagonal A: separable 2-D regrid", false;
    if (m.nx == 1 && m.interp == PMF_INTERP_LAGRANGE) return *why = "1-D Lagrange regrid", false;
    if (m.integrator != PMF_INT_EXACT && m.substeps > FUSED_LMAX) return *why = "more than 64 substeps", false;
    const int n0 = m.nx == 2 ? m.N[0] : 1, n1 = m.nx == 2 ? m.N[1] : m.N[0];
    if (group_type(m.nx, n0, n1) < 0)
        return *why = "grid size without a fused form (2-D: N0 x N1, N0 and N1 in {32,48,64,96,128}; "
                      "1-D: N in {32,48,64,96,128,192,256})", false;
    return true;
}

static int pow2_at_least(int v) {
    int p = 1;
    while (p < v) p <<= 1;
    return p;
}

// Same-size filters in groups of at most the group type's capacity, largest
// grids first (the dispatcher hands the longest work out first).  Array
// form without allocation: order (n ints) is working space, sorted receives the
// items in group order, groups at most n records (*ngroups of them).  Ties keep
// the input order.  sched (null: defaults) holds the schedule variant per group
// type.  Returns the largest complex LDS need of a group.
static int group_items_arr(const BItem* items, int n, int* order, BItem* sorted, GItem* groups, int* ngroups,
                           const int* sched) {
    for (int i = 0; i < n; ++i) order[i] = i;
    std::sort(order, order + n, [&](int a, int b) {
        const long pa = (long)items[a].n0 * items[a].n1, pb = (long)items[b].n0 * items[b].n1;
        if (pa != pb) return pa > pb;
        if (items[a].n1 != items[b].n1) return items[a].n1 > items[b].n1;
        if (items[a].nx != items[b].nx) return items[a].nx > items[b].nx;
        return a < b;
    });
    int ng = 0, maxcplx = 0;
    for (int q = 0; q < n;) {
        const BItem& b = items[order[q]];
        const int type = group_type(b.nx, b.n0, b.n1);
        const int v = sched && sched_offered(type, sched[type]) ? sched[type] : 0;
        const int G = group_capacity(type, v);
        GItem gi;
        gi.first = q;
        gi.n0 = b.n0;
        gi.n1 = b.n1;
        gi.nx = b.nx;
        gi.seg = std::max(32, pow2_at_least(b.n1));
        gi.type = type * NSCHED + v;
        gi.pad = 0;
        int cnt = 0;
        while (q < n && cnt < G && items[order[q]].n0 == b.n0 && items[order[q]].n1 == b.n1 &&
               items[order[q]].nx == b.nx) {
            sorted[q] = items[order[q]];
            ++q;
            ++cnt;
        }
        gi.G = cnt;
        groups[ng++] = gi;
        maxcplx = std::max(maxcplx, group_cplx(gi.n0, gi.n1, G, group_guard(gi.n0, gi.n1, G)));
    }
    *ngroups = ng;
    return maxcplx;
}

static int group_items(const std::vector<BItem>& items, std::vector<BItem>& sorted, std::vector<GItem>& groups,
                       const int* sched) {
    const int n = (int)items.size();
    std::vector<int> order(n);
    sorted.assign(n, BItem{});
    groups.assign(n, GItem{});
    int ng = 0;
    const int maxcplx = group_items_arr(items.data(), n, order.data(), sorted.data(), groups.data(), &ng, sched);
    groups.resize(ng);
    return maxcplx;
}

// dynamic LDS of the fused kernel for a given complex buffer size, and the
// largest it can be (two buffers of CPLX_BUDGET entries)
static size_t fused_lds(int maxcplx) {
    return 2 * (size_t)maxcplx * sizeof(float2) + (128 + 128 + 130) * sizeof(float2);
}

// Orders work on stream st after everything queued so far on the null stream (the
// host-to-device copies below go there; a launch on a non-blocking stream is not
// otherwise ordered after them).
static hipError_t stream_after_null(hipStream_t st) {
    if (st == nullptr) return hipSuccess;
    hipEvent_t ev = nullptr;
    hipError_t e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventRecord(ev, nullptr);
    if (e == hipSuccess) e = hipStreamWaitEvent(st, ev, 0);
    if (ev) (void)hipEventDestroy(ev);
    return e;
}

// The buffer budget takes the whole 160 KiB of a gfx950 compute unit together with
// the kernel's static LDS: checked here, so that a change to the static LDS fails
// with this message rather than as a launch error.
static pmf_status fused_lds_attribute() {
    hipFuncAttributes fa;
    hipError_t e = hipFuncGetAttributes(&fa, reinterpret_cast<const void*>(k_fused));
    if (e != hipSuccess) return hip_fail(e, "fused kernel attributes");
    if (fa.sharedSizeBytes + fused_lds(CPLX_BUDGET) > (size_t)160 * 1024)
        return fail(PMF_E_DEVICE, "fused kernel: static LDS plus the buffer budget exceed 160 KiB");
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_fused), hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)fused_lds(CPLX_BUDGET));
    if (e != hipSuccess) return hip_fail(e, "fused kernel LDS attribute");
    return PMF_OK;
}

static pmf_status build_cache(pmf_ctx* ctx, pmf_filter* const* filters, int n, double T, hipStream_t st) {
    batch_cache_release(ctx);
    BatchCache* c = new BatchCache();
    ctx->batch = c;
    c->filters.assign(filters, filters + n);
    c->T = T;
    c->stream = st;
    c->n = n;
    int nzmax = 1;
    for (int i = 0; i < n; ++i) nzmax = std::max(nzmax, filters[i]->model.nz);
    c->nzmax = nzmax;
    std::vector<FConst> consts(n);
    std::vector<BItem> items(n);
    for (int i = 0; i < n; ++i) {
        pmf_filter* f = filters[i];
        consts[i].m = f->km;
        consts[i].pa = predict_args(f, T);
        BItem& b = items[i];
        b.P[0] = static_cast<float*>(f->buf[0]);
        b.P[1] = static_cast<float*>(f->buf[1]);
        b.d = f->desc;
        b.coef = f->coef;
        b.idx = i;
        b.nx = f->model.nx;
        b.n0 = f->model.nx == 2 ? f->model.N[0] : 1;
        b.n1 = f->model.nx == 2 ? f->model.N[1] : f->model.N[0];
    }
    std::vector<BItem> sorted;
    std::vector<GItem> groups;
    const int maxcplx = group_items(items, sorted, groups, ctx->sched);
    c->ngroups = (int)groups.size();
    c->order.resize(n);
    for (int q = 0; q < n; ++q) c->order[q] = sorted[q].idx;
    bool ok = true;
    auto A = [&](size_t bytes) {
        void* p = ctx_alloc(ctx, bytes, st);
        if (!p) ok = false;
        return p;
    };
    c->d_consts = static_cast<FConst*>(A(sizeof(FConst) * n));
    c->d_items = static_cast<BItem*>(A(sizeof(BItem) * n));
    c->d_groups = static_cast<GItem*>(A(sizeof(GItem) * groups.size()));
    c->d_plans = static_cast<FPlan*>(A(sizeof(FPlan) * n));
    c->d_z = static_cast<double*>(A(sizeof(double) * n * nzmax));
    c->d_ll = static_cast<double*>(A(sizeof(double) * n));
    if (!ok) return fail(PMF_E_NOMEM, "batch allocation failed");
    for (int q = 0; q < n; ++q) sorted[q].k = c->d_consts + sorted[q].idx;
    hipError_t e = hipMemcpy(c->d_consts, consts.data(), sizeof(FConst) * n, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(c->d_items, sorted.data(), sizeof(BItem) * n, hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(c->d_groups, groups.data(), sizeof(GItem) * groups.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = stream_after_null(st);
    for (int i = 0; i < BatchCache::ZSLOTS && e == hipSuccess; ++i) {
        e = hipHostMalloc(reinterpret_cast<void**>(&c->h_z[i]), sizeof(double) * n * nzmax, hipHostMallocMapped);
        if (e == hipSuccess) e = hipHostGetDevicePointer(reinterpret_cast<void**>(&c->hz_dev[i]), c->h_z[i], 0);
    }
    for (int i = 0; i < 2 && e == hipSuccess; ++i) e = hipEventCreateWithFlags(&c->ev[i], hipEventDisableTiming);
    if (e != hipSuccess) return hip_fail(e, "batch setup");
    c->bufcplx = maxcplx;
    c->lds = fused_lds(maxcplx);
    pmf_status ls = fused_lds_attribute();
    if (ls != PMF_OK) return ls;
    int per_cu = 0;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_fused, FUSED_THREADS, c->lds);
    if (e != hipSuccess) return hip_fail(e, "occupancy");
    if (per_cu < 1) return fail(PMF_E_INVALID, "fused kernel does not fit on a compute unit");
    c->grid = c->ngroups;   // one workgroup per group
    return PMF_OK;
}

// ---------------------------------------------------------------- served batches

}  // namespace pmf

struct DynBatch {
    int cap = 0;                     // filters the buffers hold
    pmf::FPlan* d_plans = nullptr;   // device
    // mapped pinned host memory, read (items, groups, z) and written (log-likelihoods)
    // by the kernels in place: a served batch is two launches, no copies
    pmf::BItem* h_items = nullptr;
    pmf::GItem* h_groups = nullptr;
    double* h_z = nullptr;
    double* h_ll = nullptr;
    pmf::BItem* m_items = nullptr;   // the same memory as the device addresses it
    pmf::GItem* m_groups = nullptr;
    double* m_z = nullptr;
    double* m_ll = nullptr;
    bool attr = false;
    std::map<size_t, int> per_cu;    // resident fused workgroups per CU, by LDS size
};

namespace pmf {

static void dyn_free_buffers(pmf_ctx* ctx, DynBatch* db) {
    ctx_free(ctx, db->d_plans, nullptr);
    if (db->h_items) (void)hipHostFree(db->h_items);
    if (db->h_groups) (void)hipHostFree(db->h_groups);
    if (db->h_z) (void)hipHostFree(db->h_z);
    if (db->h_ll) (void)hipHostFree(db->h_ll);
    db->d_plans = nullptr;
    db->h_items = db->m_items = nullptr;
    db->h_groups = db->m_groups = nullptr;
    db->h_z = db->h_ll = db->m_z = db->m_ll = nullptr;
    db->cap = 0;
}

DynBatch* dyn_create(pmf_ctx*) { return new DynBatch(); }

size_t fused_const_bytes() { return sizeof(FConst); }

// the filter's fused-step constants for interval T in its device record
// f->dconst (uploaded only when T changed)
static pmf_status upload_consts(pmf_filter* f, double T, hipStream_t st) {
    if (f->dconst_T == T) return PMF_OK;
    FConst k;
    k.m = f->km;
    k.pa = predict_args(f, T);
    hipError_t e = hipMemcpy(f->dconst, &k, sizeof(FConst), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = stream_after_null(st);
    if (e != hipSuccess) return hip_fail(e, "fused constants upload");
    f->dconst_T = T;
    return PMF_OK;
}

void dyn_destroy(pmf_ctx* ctx, DynBatch* db) {
    if (!db) return;
    (void)hipDeviceSynchronize();
    dyn_free_buffers(ctx, db);
    delete db;
}

const double* dyn_loglik(const DynBatch* db) { return db->h_ll; }

static pmf_status dyn_reserve(pmf_ctx* ctx, DynBatch* db, int n) {
    if (n <= db->cap) return PMF_OK;
    int cap = std::max(64, db->cap);
    while (cap < n) cap *= 2;
    (void)hipDeviceSynchronize();   // the old buffers may still be read by a launch
    dyn_free_buffers(ctx, db);
    bool ok = true;
    auto A = [&](size_t bytes) {
        void* p = ctx_alloc(ctx, bytes, nullptr);
        if (!p) ok = false;
        return p;
    };
    db->d_plans = static_cast<FPlan*>(A(sizeof(FPlan) * cap));
    hipError_t e = hipSuccess;
    auto H = [&](void** h, void** m, size_t bytes) {
        if (e != hipSuccess) return;
        e = hipHostMalloc(h, bytes, hipHostMallocMapped);
        if (e == hipSuccess) e = hipHostGetDevicePointer(m, *h, 0);
    };
    H(reinterpret_cast<void**>(&db->h_items), reinterpret_cast<void**>(&db->m_items), sizeof(BItem) * cap);
    H(reinterpret_cast<void**>(&db->h_groups), reinterpret_cast<void**>(&db->m_groups), sizeof(GItem) * cap);
    H(reinterpret_cast<void**>(&db->h_z), reinterpret_cast<void**>(&db->m_z), sizeof(double) * 3 * cap);
    H(reinterpret_cast<void**>(&db->h_ll), reinterpret_cast<void**>(&db->m_ll), sizeof(double) * cap);
    if (!ok || e != hipSuccess) {
        dyn_free_buffers(ctx, db);
        return fail(PMF_E_NOMEM, "served batch allocation failed");
    }
    db->cap = cap;
    return PMF_OK;
}

pmf_status dyn_run(pmf_ctx* ctx, DynBatch* db, pmf_filter* const* filters, int n, double T, const double* z,
                   hipStream_t st) {
    if (n < 1) return PMF_OK;
    if (!std::isfinite(T) || !(T > 0.0)) return fail(PMF_E_INVALID, "T must be finite and > 0");
    pmf_status s = dyn_reserve(ctx, db, n);
    if (s != PMF_OK) return s;
    hipError_t e = hipSuccess;
    if (!db->attr) {
        const pmf_status ls = fused_lds_attribute();
        if (ls != PMF_OK) return ls;
        db->attr = true;
    }
    std::vector<BItem> items(n);
    for (int i = 0; i < n; ++i) {
        pmf_filter* f = filters[i];
        std::string why;
        if (!batch_fusable(f, &why)) return fail(PMF_E_INVALID, "filter not fusable: " + why);
        e = batch_enter(f);
        if (e != hipSuccess) return hip_fail(e, "batch enter");
        if (!f->dconst) {
            f->dconst = ctx_alloc(ctx, sizeof(FConst), nullptr);
            if (!f->dconst) return fail(PMF_E_NOMEM, "fused constants");
            f->bytes += sizeof(FConst);
            f->dconst_T = -1.0;
        }
        s = upload_consts(f, T, st);
        if (s != PMF_OK) return s;
        BItem& b = items[i];
        b.P[0] = static_cast<float*>(f->buf[0]);
        b.P[1] = static_cast<float*>(f->buf[1]);
        b.d = f->desc;
        b.k = static_cast<const FConst*>(f->dconst);
        b.coef = f->coef;
        b.idx = i;
        b.nx = f->model.nx;
        b.n0 = f->model.nx == 2 ? f->model.N[0] : 1;
        b.n1 = f->model.nx == 2 ? f->model.N[1] : f->model.N[0];
    }
    std::vector<BItem> sorted;
    std::vector<GItem> groups;
    const int maxcplx = group_items(items, sorted, groups, ctx->sched);
    const int ng = (int)groups.size();
    const size_t lds = fused_lds(maxcplx);
    auto it = db->per_cu.find(lds);
    if (it == db->per_cu.end()) {
        int pc = 0;
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&pc, k_fused, FUSED_THREADS, lds);
        if (e != hipSuccess) return hip_fail(e, "occupancy");
        if (pc < 1) return fail(PMF_E_INVALID, "fused kernel does not fit on a compute unit");
        db->per_cu.emplace(lds, pc);
    }
    // the staging set is written in place (the caller reuses a set only after the
    // launch that read it has completed); the kernels read it, and write the
    // log-likelihoods, through its mapped device addresses
    std::memcpy(db->h_items, sorted.data(), sizeof(BItem) * n);
    std::memcpy(db->h_groups, groups.data(), sizeof(GItem) * ng);
    for (int q = 0; q < n; ++q)   // rows in item order
        std::memcpy(db->h_z + (size_t)q * 3, z + (size_t)sorted[q].idx * 3, sizeof(double) * 3);
    hipLaunchKernelGGL(k_batch_plan, dim3((n + PLAN_THREADS - 1) / PLAN_THREADS), dim3(PLAN_THREADS), 0, st,
                       db->m_items, db->d_plans, n, db->m_z, nullptr, 3);
    hipLaunchKernelGGL(k_fused, dim3(ng), dim3(FUSED_THREADS), lds, st, db->m_groups, db->m_items, db->d_plans,
                       db->m_z, 3, db->m_ll, maxcplx);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "served batch launch");
    return PMF_OK;
}

}  // namespace pmf

namespace pmf {

// The cached launch set-up for (filters, T, stream), validated and built when the
// set is new or one of its filters took other calls since; zrows rows of z (each
// n * nz_max) are checked for finite values then.
static pmf_status batch_prepare(pmf_ctx* ctx, pmf_filter* const* filters, int n, double T, const double* z, int zrows,
                                hipStream_t st, BatchCache** out) {
    hipError_t e = hipSuccess;
    BatchCache* c = ctx->batch;
    const bool same = c && c->n == n && c->T == T && c->stream == st &&
                      std::equal(filters, filters + n, c->filters.begin());
    if (!same || c->leaves_seen != ctx->batch_leaves) {
        // a new filter set, or a filter of it took other calls since the last step:
        // validate, (re-)enter the batched layout, build the launch set-up.  An
        // unchanged set skips all of this (its filters were checked when it was built)
        int nzmax = 1;
        for (int i = 0; i < n; ++i) {
            if (!filters[i] || filters[i]->ctx != ctx) return fail(PMF_E_INVALID, "filter of another context");
            std::string why;
            if (!batch_fusable(filters[i], &why)) return fail(PMF_E_INVALID, "filter not fusable: " + why);
            nzmax = std::max(nzmax, filters[i]->model.nz);
        }
        for (size_t i = 0; i < (size_t)zrows * n * nzmax; ++i)
            if (!std::isfinite(z[i])) return fail(PMF_E_INVALID, "non-finite measurement");
        if (!same) {
            // a filter listed twice would be stepped twice in one launch, racing with itself
            std::vector<pmf_filter*> sorted(filters, filters + n);
            std::sort(sorted.begin(), sorted.end());
            if (std::adjacent_find(sorted.begin(), sorted.end()) != sorted.end())
                return fail(PMF_E_INVALID, "filter listed twice");
        }
        for (int i = 0; i < n; ++i) {
            e = batch_enter(filters[i]);
            if (e != hipSuccess) return hip_fail(e, "batch enter");
        }
        if (!same) {
            pmf_status s = build_cache(ctx, filters, n, T, st);
            if (s != PMF_OK) {
                batch_cache_release(ctx);
                return s;
            }
            c = ctx->batch;
        }
        c->leaves_seen = ctx->batch_leaves;
    }
    *out = c;
    return PMF_OK;
}

}  // namespace pmf

extern "C" pmf_status pmf_batch_step(pmf_ctx* ctx, pmf_filter* const* filters, int n, double T, const double* z,
                                     double* loglik, void* stream) {
    using namespace pmf;
    if (!ctx || n < 1 || !filters || !z) return fail(PMF_E_INVALID, "NULL argument or n < 1");
    if (!std::isfinite(T) || !(T > 0.0)) return fail(PMF_E_INVALID, "T must be finite and > 0");
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    const hipStream_t st = static_cast<hipStream_t>(stream);
    BatchCache* c = nullptr;
    {
        const pmf_status s = batch_prepare(ctx, filters, n, T, z, 1, st, &c);
        if (s != PMF_OK) return s;
    }
    const int nzmax = c->nzmax;
    // stage z in mapped pinned memory, rows in item order, checking it on the way;
    // the planning kernel reads it there, no separate copy.  First the event of
    // the group of steps before the previous one (never recorded before step
    // 2 ZEVERY: the first slots are fresh).
    const long long k = c->step;
    const int slot = (int)(k % BatchCache::ZSLOTS);
    const int evi = (int)((k / BatchCache::ZEVERY) & 1);
    e = hipEventSynchronize(c->ev[evi]);
    if (e != hipSuccess) return hip_fail(e, "staging wait");
    bool finite = true;
    double* dst = c->h_z[slot];
    for (int q = 0; q < n; ++q) {
        const double* src = z + (size_t)c->order[q] * nzmax;
        for (int j = 0; j < nzmax; ++j) {
            const double v = src[j];
            finite = finite && std::isfinite(v);
            dst[(size_t)q * nzmax + j] = v;
        }
    }
    if (!finite) return fail(PMF_E_INVALID, "non-finite measurement");
    c->step = k + 1;
    if (ctx->profile) {
        // the same launches with events around the fused kernel
        if ((int)ctx->ev_pool.size() < 2 * (ctx->ev_used + 1)) {
            for (int q = 0; q < 2 && e == hipSuccess; ++q) {
                hipEvent_t ev;
                e = hipEventCreate(&ev);
                if (e == hipSuccess) ctx->ev_pool.push_back(ev);
            }
        }
        if (e == hipSuccess) {
            hipEvent_t t0 = ctx->ev_pool[2 * ctx->ev_used];
            hipEvent_t t1 = ctx->ev_pool[2 * ctx->ev_used + 1];
            ctx->ev_used++;
            ctx->ev_stream = st;
            hipLaunchKernelGGL(k_batch_plan, dim3((n + PLAN_THREADS - 1) / PLAN_THREADS), dim3(PLAN_THREADS), 0, st,
                               c->d_items, c->d_plans, n, c->hz_dev[slot], c->d_z, c->nzmax);
            e = hipEventRecord(t0, st);
            if (e == hipSuccess) {
                hipLaunchKernelGGL(k_fused, dim3(c->grid), dim3(FUSED_THREADS), c->lds, st, c->d_groups, c->d_items,
                                   c->d_plans, c->d_z, c->nzmax, c->d_ll, c->bufcplx);
                e = hipGetLastError();
            }
            if (e == hipSuccess) e = hipEventRecord(t1, st);
        }
    } else {
        // plan every filter (reading its z from the slot), then the fused kernel
        hipLaunchKernelGGL(k_batch_plan, dim3((n + PLAN_THREADS - 1) / PLAN_THREADS), dim3(PLAN_THREADS), 0, st,
                           c->d_items, c->d_plans, n, c->hz_dev[slot], c->d_z, c->nzmax);
        hipLaunchKernelGGL(k_fused, dim3(c->grid), dim3(FUSED_THREADS), c->lds, st, c->d_groups, c->d_items,
                           c->d_plans, c->d_z, c->nzmax, c->d_ll, c->bufcplx);
        e = hipGetLastError();
    }
    if (e == hipSuccess && k % BatchCache::ZEVERY == BatchCache::ZEVERY - 1) e = hipEventRecord(c->ev[evi], st);
    if (e == hipSuccess && loglik) e = hipMemcpyAsync(loglik, c->d_ll, sizeof(double) * n, hipMemcpyDeviceToHost, st);
    if (e != hipSuccess) return hip_fail(e, "batch launch");
    return PMF_OK;
}

extern "C" pmf_status pmf_batch_run(pmf_ctx* ctx, pmf_filter* const* filters, int n, double T, int K,
                                    const double* z, double* loglik, void* stream) {
    using namespace pmf;
    if (!ctx || n < 1 || !filters || !z) return fail(PMF_E_INVALID, "NULL argument or n < 1");
    if (K < 1 || K > 256) return fail(PMF_E_INVALID, "K must be in 1..256");
    if (!std::isfinite(T) || !(T > 0.0)) return fail(PMF_E_INVALID, "T must be finite and > 0");
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    const hipStream_t st = static_cast<hipStream_t>(stream);
    BatchCache* c = nullptr;
    {
        const pmf_status s = batch_prepare(ctx, filters, n, T, z, K, st, &c);
        if (s != PMF_OK) return s;
    }
    const int nzmax = c->nzmax;
    const size_t zn = (size_t)K * n * nzmax;
    for (size_t i = 0; i < zn; ++i)
        if (!std::isfinite(z[i])) return fail(PMF_E_INVALID, "non-finite measurement");
    // the caller's earlier work on these filters first: the run goes on a private stream
    e = hipStreamSynchronize(st);
    if (e == hipSuccess && !c->run_st) e = hipStreamCreateWithFlags(&c->run_st, hipStreamNonBlocking);
    if (e != hipSuccess) return hip_fail(e, "batch run set-up");
    if (c->run_k != K) {
        run_free(ctx, c);
        c->d_zrun = static_cast<double*>(ctx_alloc(ctx, sizeof(double) * zn, nullptr));
        c->d_llrun = static_cast<double*>(ctx_alloc(ctx, sizeof(double) * K * n, nullptr));
        if (!c->d_zrun || !c->d_llrun) {
            run_free(ctx, c);
            return fail(PMF_E_NOMEM, "batch run buffers");
        }
        e = hipHostMalloc(reinterpret_cast<void**>(&c->h_zrun), sizeof(double) * zn, hipHostMallocDefault);
        if (e == hipSuccess)
            e = hipHostMalloc(reinterpret_cast<void**>(&c->h_llrun), sizeof(double) * K * n, hipHostMallocDefault);
        // the K steps as one graph: per step the planning kernel (z from row k of
        // the device copy) and the fused kernel (log-likelihoods into row k)
        if (e == hipSuccess) e = hipStreamBeginCapture(c->run_st, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            for (int k = 0; k < K; ++k) {
                const double* zk = c->d_zrun + (size_t)k * n * nzmax;
                hipLaunchKernelGGL(k_batch_plan, dim3((n + PLAN_THREADS - 1) / PLAN_THREADS), dim3(PLAN_THREADS), 0,
                                   c->run_st, c->d_items, c->d_plans, n, zk, nullptr, nzmax);
                hipLaunchKernelGGL(k_fused, dim3(c->grid), dim3(FUSED_THREADS), c->lds, c->run_st, c->d_groups,
                                   c->d_items, c->d_plans, zk, nzmax, c->d_llrun + (size_t)k * n, c->bufcplx);
            }
            const hipError_t el = hipGetLastError();
            e = hipStreamEndCapture(c->run_st, &c->run_graph);
            if (e == hipSuccess) e = el;
        }
        if (e == hipSuccess) e = hipGraphInstantiate(&c->run_exec, c->run_graph, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            run_free(ctx, c);
            return hip_fail(e, "batch run capture");
        }
        c->run_k = K;
    }
    // measurements in item order, one copy for all K steps
    for (int k = 0; k < K; ++k)
        for (int q = 0; q < n; ++q)
            std::memcpy(c->h_zrun + ((size_t)k * n + q) * nzmax, z + ((size_t)k * n + c->order[q]) * nzmax,
                        sizeof(double) * nzmax);
    e = hipMemcpyAsync(c->d_zrun, c->h_zrun, sizeof(double) * zn, hipMemcpyHostToDevice, c->run_st);
    if (e == hipSuccess) e = hipGraphLaunch(c->run_exec, c->run_st);
    if (e == hipSuccess && loglik)
        e = hipMemcpyAsync(c->h_llrun, c->d_llrun, sizeof(double) * K * n, hipMemcpyDeviceToHost, c->run_st);
    if (e == hipSuccess) e = hipStreamSynchronize(c->run_st);
    if (e != hipSuccess) return hip_fail(e, "batch run");
    if (loglik) std::memcpy(loglik, c->h_llrun, sizeof(double) * K * n);   // filter order
    return PMF_OK;
}

extern "C" pmf_status pmf_batch_profile(pmf_ctx* ctx, int enable) {
    using namespace pmf;
    if (!ctx) return fail(PMF_E_INVALID, "ctx is NULL");
    ctx->profile = enable != 0;
    ctx->ev_used = 0;
    return PMF_OK;
}

extern "C" pmf_status pmf_batch_kernel_time(pmf_ctx* ctx, double* total_ms, int* launches) {
    using namespace pmf;
    if (!ctx || !total_ms || !launches) return fail(PMF_E_INVALID, "NULL argument");
    hipError_t e = hipSetDevice(ctx->device);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->ev_stream);
    double tot = 0.0;
    for (int i = 0; i < ctx->ev_used && e == hipSuccess; ++i) {
        float ms = 0.f;
        e = hipEventElapsedTime(&ms, ctx->ev_pool[2 * i], ctx->ev_pool[2 * i + 1]);
        tot += ms;
    }
    if (e != hipSuccess) return hip_fail(e, "batch kernel time");
    *total_ms = tot;
    *launches = ctx->ev_used;
    ctx->ev_used = 0;
    return PMF_OK;
}

// ==================================================================== schedule autotuning
// Each 2-D group type has up to four compile-time schedules (filters per
// workgroup full or half, column radix order default or reversed).  The tuner
// times them with the real kernels on a synthetic batch with the caller's mix of
// sizes (one launch balances all sizes together, so a size's best
// schedule depends on the mix) and keeps the choice per type in the context; it
// is cached as a small JSON file keyed by device, HIP runtime, library build and
// mix.

namespace pmf {

static const int TUNE_N[5] = {32, 48, 64, 96, 128};
static const char* const BUILD_STAMP = __DATE__ " " __TIME__;

static std::string tune_key(int device) {
    hipDeviceProp_t p;
    if (hipGetDeviceProperties(&p, device) != hipSuccess) return std::string();
    int rt = 0;
    if (hipRuntimeGetVersion(&rt) != hipSuccess) return std::string();
    char buf[512];
    std::snprintf(buf, sizeof buf, "pmf-sched-1 arch=%s cus=%d hip=%d build=%s", p.gcnArchName,
                  p.multiProcessorCount, rt, BUILD_STAMP);
    return buf;
}

// the schedules of a cache file whose key matches, else false
static bool tune_read(const char* path, const std::string& key, int* out) {
    FILE* fp = std::fopen(path, "rb");
    if (!fp) return false;
    std::string s;
    char b[4096];
    size_t r;
    while ((r = std::fread(b, 1, sizeof b, fp)) > 0) s.append(b, r);
    std::fclose(fp);
    if (s.find("\"key\": \"" + key + "\"") == std::string::npos) return false;
    const size_t sp = s.find("\"schedules\"");
    if (sp == std::string::npos) return false;
    for (int i = 0; i < 5; ++i) {
        char name[32];
        std::snprintf(name, sizeof name, "\"%dx%d\": ", TUNE_N[i], TUNE_N[i]);
        const size_t q = s.find(name, sp);
        int v = -1;
        if (q == std::string::npos || std::sscanf(s.c_str() + q + std::strlen(name), "%d", &v) != 1) return false;
        if (v < 0 || v >= NSCHED || !sched_offered(group_type(2, TUNE_N[i], TUNE_N[i]), v)) return false;
        out[i] = v;
    }
    return true;
}

static bool tune_write(const char* path, const std::string& key, const int* sched, const double (*ms)[NSCHED],
                       const int* mix, int steps) {
    const std::string tmp = std::string(path) + ".tmp";
    FILE* fp = std::fopen(tmp.c_str(), "wb");
    if (!fp) return false;
    std::fprintf(fp, "{\n  \"key\": \"%s\",\n  \"mix\": [%d, %d, %d, %d, %d],\n  \"steps\": %d,\n  \"schedules\": {",
                 key.c_str(), mix[0], mix[1], mix[2], mix[3], mix[4], steps);
    for (int i = 0; i < 5; ++i) std::fprintf(fp, "%s\"%dx%d\": %d", i ? ", " : "", TUNE_N[i], TUNE_N[i], sched[i]);
    std::fprintf(fp, "},\n  \"kernel_ms\": {");
    for (int i = 0; i < 5; ++i) {
        std::fprintf(fp, "%s\"%dx%d\": [", i ? ", " : "", TUNE_N[i], TUNE_N[i]);
        for (int v = 0; v < NSCHED; ++v) {
            if (ms[i][v] > 0.0) std::fprintf(fp, "%s%.6f", v ? ", " : "", ms[i][v]);
            else std::fprintf(fp, "%snull", v ? ", " : "");
        }
        std::fprintf(fp, "]");
    }
    std::fprintf(fp, "}\n}\n");
    const bool ok = std::fclose(fp) == 0;
    return ok && std::rename(tmp.c_str(), path) == 0;
}

// one fusable synthetic 2-D filter of N x N points: sheared stable drift, linear
// measurement of both components, exact integrator, FP32 density
static void tune_model(int N, pmf_model* m, pmf_prior* p) {
    std::memset(m, 0, sizeof *m);
    std::memset(p, 0, sizeof *p);
    m->nx = 2;
    const double A[4] = {-0.5, 0.3, -0.2, -0.4};
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) m->A[i * 2 + j] = A[i * 2 + j];
    m->Q[0] = 0.5;
    m->Q[3] = 0.8;
    m->grid = PMF_GRID_FOURIER;
    m->N[0] = m->N[1] = N;
    m->span_sigmas = 8.0;
    m->t_nominal = 0.05;
    m->integrator = PMF_INT_EXACT;
    m->substeps = 1;
    m->precision = PMF_FP32;
    m->interp = PMF_INTERP_AUTO;
    m->meas_kind = PMF_H_LINEAR;
    m->nz = 2;
    m->H[0] = m->H[3] = 1.0;
    m->noise_ncomp = 1;
    m->noise_w[0] = 1.0;
    m->noise_cov[0] = m->noise_cov[3] = 0.09;   // row-major nz x nz
    p->ncomp = 1;
    p->w[0] = 1.0;
    p->cov[0] = p->cov[3] = 0.09;               // row-major nx x nx
}

}  // namespace pmf

extern "C" pmf_status pmf_autotune(pmf_ctx* ctx, const int* counts, int steps, const char* cache_path, char* report,
                                   size_t report_len) {
    using namespace pmf;
    if (!ctx) return fail(PMF_E_INVALID, "ctx is NULL");
    int mix[5];
    long total = 0;
    for (int i = 0; i < 5; ++i) {
        mix[i] = counts ? counts[i] : 1024;
        if (mix[i] < 0 || mix[i] > 65536) return fail(PMF_E_INVALID, "filters per size must be in 0..65536");
        total += mix[i];
    }
    if (total < 1) return fail(PMF_E_INVALID, "the mix has no filters");
    if (steps < 1 || steps > 1000) return fail(PMF_E_INVALID, "steps must be in 1..1000");
    if (report && report_len) report[0] = '\0';
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    std::string key = tune_key(ctx->device);
    if (key.empty()) return fail(PMF_E_DEVICE, "device properties for the tuning key");
    {
        char mb[96];
        std::snprintf(mb, sizeof mb, " mix=%d,%d,%d,%d,%d", mix[0], mix[1], mix[2], mix[3], mix[4]);
        key += mb;
    }
    int chosen[5] = {};
    double ms[5][NSCHED] = {};
    std::string rep;
    char line[256];
    if (cache_path && tune_read(cache_path, key, chosen)) {
        for (int i = 0; i < 5; ++i) ctx->sched[group_type(2, TUNE_N[i], TUNE_N[i])] = chosen[i];
        batch_cache_release(ctx);
        rep = std::string("schedules from ") + cache_path + ":";
        for (int i = 0; i < 5; ++i) {
            std::snprintf(line, sizeof line, " %dx%d:%d", TUNE_N[i], TUNE_N[i], chosen[i]);
            rep += line;
        }
        rep += "\n";
    } else {
        const bool prof = ctx->profile;
        int saved[16];
        std::memcpy(saved, ctx->sched, sizeof saved);
        pmf_status s = PMF_OK;
        // the synthetic mix, all sizes in one batch
        std::vector<pmf_filter*> fs;
        for (int i = 0; i < 5 && s == PMF_OK; ++i) {
            pmf_model m;
            pmf_prior p;
            tune_model(TUNE_N[i], &m, &p);
            for (int k = 0; k < mix[i] && s == PMF_OK; ++k) {
                pmf_filter* f = nullptr;
                s = pmf_create(ctx, &m, &p, &f);
                if (s == PMF_OK) fs.push_back(f);
            }
        }
        const int n = (int)fs.size();
        const double T = 0.05;
        std::vector<double> z(2 * (size_t)std::max(n, 1), 0.0);
        // mean fused-kernel time of the whole mix under the context's schedules
        auto time_mix = [&](double* out) {
            batch_cache_release(ctx);
            ctx->profile = false;
            for (int k = 0; k < 2 && s == PMF_OK; ++k) s = pmf_batch_step(ctx, fs.data(), n, T, z.data(), nullptr, nullptr);
            ctx->profile = true;
            ctx->ev_used = 0;
            for (int k = 0; k < steps && s == PMF_OK; ++k)
                s = pmf_batch_step(ctx, fs.data(), n, T, z.data(), nullptr, nullptr);
            double tot = 0.0;
            int nl = 0;
            if (s == PMF_OK) s = pmf_batch_kernel_time(ctx, &tot, &nl);
            if (s == PMF_OK && nl > 0) *out = std::min(*out, tot / nl);
        };
        for (int i = 0; i < 5; ++i) ctx->sched[group_type(2, TUNE_N[i], TUNE_N[i])] = 0;
        // one pass of coordinate descent over the sizes present, largest first:
        // each size's variants timed on the whole mix (three rounds, fastest mean
        // kept); a variant replaces the current one only when at least 1 % faster
        for (int i = 4; i >= 0 && s == PMF_OK; --i) {
            const int N = TUNE_N[i];
            const int type = group_type(2, N, N);
            std::vector<int> offered;
            for (int v = 0; v < NSCHED; ++v)
                if (sched_offered(type, v)) offered.push_back(v);
            if (mix[i] == 0 || offered.size() < 2) {
                std::snprintf(line, sizeof line, "%dx%d: %s -> 0\n", N, N,
                              mix[i] == 0 ? "not in the mix" : "one schedule");
                rep = line + rep;
                continue;
            }
            for (int v : offered) ms[i][v] = 1e300;
            for (int r = 0; r < 3 && s == PMF_OK; ++r)
                for (int v : offered) {
                    if (s != PMF_OK) break;
                    ctx->sched[type] = v;
                    time_mix(&ms[i][v]);
                }
            if (s != PMF_OK) break;
            int best = 0;
            for (int v : offered)
                if (ms[i][v] < ms[i][best]) best = v;
            if (!(ms[i][best] < 0.99 * ms[i][0])) best = 0;
            ctx->sched[type] = chosen[i] = best;
            std::string l;
            std::snprintf(line, sizeof line, "%dx%d (%d of %d filters), mix kernel:", N, N, mix[i], n);
            l += line;
            for (int v : offered) {
                std::snprintf(line, sizeof line, " v%d %.4f ms", v, ms[i][v]);
                l += line;
            }
            std::snprintf(line, sizeof line, " -> %d\n", best);
            rep = l + line + rep;
        }
        batch_cache_release(ctx);
        for (pmf_filter* f : fs) pmf_destroy(f);
        ctx->profile = prof;
        ctx->ev_used = 0;
        if (s != PMF_OK) {
            std::memcpy(ctx->sched, saved, sizeof saved);
            return s;
        }
        for (int i = 0; i < 5; ++i)
            for (int v = 0; v < NSCHED; ++v)
                if (ms[i][v] >= 1e300) ms[i][v] = 0.0;
        if (cache_path && !tune_write(cache_path, key, chosen, ms, mix, steps))
            return fail(PMF_E_INVALID, std::string("cannot write the schedule cache ") + cache_path);
    }
    if (report && report_len) {
        const size_t k = std::min(report_len - 1, rep.size());
        std::memcpy(report, rep.data(), k);
        report[k] = '\0';
    }
    return PMF_OK;
}

extern "C" pmf_status pmf_get_schedule(pmf_ctx* ctx, int nx, int N, int* variant) {
    using namespace pmf;
    if (!ctx || !variant) return fail(PMF_E_INVALID, "NULL argument");
    const int type = group_type(nx, nx == 2 ? N : 1, N);
    if (type < 0) return fail(PMF_E_INVALID, "no fused form for this grid size");
    *variant = sched_offered(type, ctx->sched[type]) ? ctx->sched[type] : 0;
    return PMF_OK;
}

extern "C" pmf_status pmf_set_schedule(pmf_ctx* ctx, int nx, int N, int variant) {
    using namespace pmf;
    if (!ctx) return fail(PMF_E_INVALID, "ctx is NULL");
    const int type = group_type(nx, nx == 2 ? N : 1, N);
    if (type < 0) return fail(PMF_E_INVALID, "no fused form for this grid size");
    if (variant < 0 || variant >= NSCHED || !sched_offered(type, variant))
        return fail(PMF_E_INVALID, "schedule variant not offered for this grid size");
    if (ctx->sched[type] != variant) {
        ctx->sched[type] = variant;
        batch_cache_release(ctx);
    }
    return PMF_OK;
}

// ==================================================================== step without allocation
// pmf_batch_step_noalloc: the same planning and fused kernels, with their
// per-step records (items, groups, plans, z, log-likelihoods) in a file-scope
// device array instead of library allocations.

namespace pmf {

constexpr int NOALLOC_MAX = 4096;   // filters per call
constexpr size_t al256(size_t b) { return (b + 255) / 256 * 256; }
// byte offsets of the parts inside the array (each 256-byte aligned)
constexpr size_t NA_ITEMS = 0;
constexpr size_t NA_GROUPS = NA_ITEMS + al256(sizeof(BItem) * NOALLOC_MAX);
constexpr size_t NA_PLANS = NA_GROUPS + al256(sizeof(GItem) * NOALLOC_MAX);
constexpr size_t NA_Z = NA_PLANS + al256(sizeof(FPlan) * NOALLOC_MAX);
constexpr size_t NA_LL = NA_Z + al256(sizeof(double) * 3 * NOALLOC_MAX);
constexpr size_t NA_BYTES = NA_LL + al256(sizeof(double) * NOALLOC_MAX);
static_assert(NA_BYTES <= (size_t)2 << 20, "the no-allocation scratch stays under 2 MiB");

}  // namespace pmf

// Every GPU the library runs on holds its own copy until the process ends.  In
// host code this name is only a stand-in for the symbol: the device address comes
// from hipGetSymbolAddress, once per device (na_device below).
static __device__ __align__(256) unsigned char scratch[pmf::NA_BYTES];

namespace pmf {

constexpr int NA_MAXDEV = 64;
static std::mutex na_mu;                      // one call at a time (host staging, scratch)
static unsigned char* na_ptr[NA_MAXDEV] = {};   // device address of scratch, per device
// host staging, reused by every call (calls are serialised by na_mu)
static BItem na_items[NOALLOC_MAX], na_sorted[NOALLOC_MAX];
static GItem na_groups[NOALLOC_MAX];
static int na_order[NOALLOC_MAX];
static pmf_filter* na_seen[NOALLOC_MAX];
static double na_z[3 * NOALLOC_MAX], na_ll[NOALLOC_MAX];

// the scratch address and LDS attribute of device dev (the device is current);
// set up on its first call
static pmf_status na_device(int dev, unsigned char** ptr) {
    if (dev < 0 || dev >= NA_MAXDEV) return fail(PMF_E_INVALID, "device index beyond 64");
    if (!na_ptr[dev]) {
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "scratch symbol address");
        const pmf_status ls = fused_lds_attribute();
        if (ls != PMF_OK) return ls;
        na_ptr[dev] = static_cast<unsigned char*>(p);
    }
    *ptr = na_ptr[dev];
    return PMF_OK;
}

}  // namespace pmf

extern "C" pmf_status pmf_batch_step_noalloc(pmf_ctx* ctx, pmf_filter* const* filters, int n, double T,
                                             const double* z, double* loglik, void* stream) {
    using namespace pmf;
    if (!ctx || n < 1 || !filters || !z) return fail(PMF_E_INVALID, "NULL argument or n < 1");
    if (n > NOALLOC_MAX) return fail(PMF_E_INVALID, "more than 4096 filters (the scratch array's limit)");
    if (!std::isfinite(T) || !(T > 0.0)) return fail(PMF_E_INVALID, "T must be finite and > 0");
    std::lock_guard<std::mutex> lk(na_mu);
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    unsigned char* base = nullptr;
    pmf_status s = na_device(ctx->device, &base);
    if (s != PMF_OK) return s;
    const hipStream_t st = static_cast<hipStream_t>(stream);

    // checks first: nothing runs unless every filter and every z is acceptable
    int nzmax = 1;
    for (int i = 0; i < n; ++i) {
        pmf_filter* f = filters[i];
        if (!f || f->ctx != ctx) return fail(PMF_E_INVALID, "filter of another context");
        std::string why;
        if (!batch_fusable(f, &why)) return fail(PMF_E_INVALID, "filter not fusable: " + why);
        if (!f->dconst) return fail(PMF_E_INVALID, "filter has no fused-step constants");
        nzmax = std::max(nzmax, f->model.nz);
        na_seen[i] = f;
    }
    for (int i = 0; i < n * nzmax; ++i)
        if (!std::isfinite(z[i])) return fail(PMF_E_INVALID, "non-finite measurement");
    std::sort(na_seen, na_seen + n);
    if (std::adjacent_find(na_seen, na_seen + n) != na_seen + n) return fail(PMF_E_INVALID, "filter listed twice");

    bool uploaded = false;
    for (int i = 0; i < n; ++i) {
        pmf_filter* f = filters[i];
        e = batch_enter(f);
        if (e != hipSuccess) return hip_fail(e, "batch enter");
        uploaded = uploaded || f->dconst_T != T;
        s = upload_consts(f, T, nullptr);   // ordered below without an event (nothing allocated)
        if (s != PMF_OK) return s;
        BItem& b = na_items[i];
        b.P[0] = static_cast<float*>(f->buf[0]);
        b.P[1] = static_cast<float*>(f->buf[1]);
        b.d = f->desc;
        b.k = static_cast<const FConst*>(f->dconst);
        b.coef = f->coef;
        b.idx = i;
        b.nx = f->model.nx;
        b.n0 = f->model.nx == 2 ? f->model.N[0] : 1;
        b.n1 = f->model.nx == 2 ? f->model.N[1] : f->model.N[0];
    }
    int ng = 0;
    const int maxcplx = group_items_arr(na_items, n, na_order, na_sorted, na_groups, &ng, ctx->sched);
    // z rows in item order, stride 3 (the kernels' layout)
    for (int q = 0; q < n; ++q)
        for (int j = 0; j < 3; ++j)
            na_z[(size_t)q * 3 + j] = j < nzmax ? z[(size_t)na_sorted[q].idx * nzmax + j] : 0.0;
    const size_t lds = fused_lds(maxcplx);
    int per_cu = 0;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_fused, FUSED_THREADS, lds);
    if (e != hipSuccess) return hip_fail(e, "occupancy");
    if (per_cu < 1) return fail(PMF_E_INVALID, "fused kernel does not fit on a compute unit");

    BItem* d_items = reinterpret_cast<BItem*>(base + NA_ITEMS);
    GItem* d_groups = reinterpret_cast<GItem*>(base + NA_GROUPS);
    FPlan* d_plans = reinterpret_cast<FPlan*>(base + NA_PLANS);
    double* d_z = reinterpret_cast<double*>(base + NA_Z);
    double* d_ll = reinterpret_cast<double*>(base + NA_LL);
    // constants uploaded above (on the null stream) are in place before the launches
    if (uploaded && st != nullptr) {
        e = hipStreamSynchronize(nullptr);
        if (e != hipSuccess) return hip_fail(e, "fused constants upload");
    }
    e = hipMemcpyAsync(d_items, na_sorted, sizeof(BItem) * n, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(d_groups, na_groups, sizeof(GItem) * ng, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(d_z, na_z, sizeof(double) * 3 * n, hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return hip_fail(e, "no-allocation step upload");
    hipLaunchKernelGGL(k_batch_plan, dim3((n + PLAN_THREADS - 1) / PLAN_THREADS), dim3(PLAN_THREADS), 0, st,
                       d_items, d_plans, n, d_z, nullptr, 3);
    hipLaunchKernelGGL(k_fused, dim3(ng), dim3(FUSED_THREADS), lds, st, d_groups, d_items, d_plans, d_z, 3, d_ll,
                       maxcplx);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(na_ll, d_ll, sizeof(double) * n, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "no-allocation step");
    if (loglik)
        for (int i = 0; i < n; ++i) loglik[i] = na_ll[i];
    return PMF_OK;
}
