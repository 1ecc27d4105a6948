// Batched predict + update: one persistent fused launch per step.
//
// A workgroup takes the next filter of a work list (largest grid first) and runs
// its whole cycle with the density resident in LDS:
//   load -> row r2c FFT (N/2-point complex FFT + split) -> column FFT ->
//   per-mode gain -> inverse column FFT -> row c2r (merge + N/2-point inverse) ->
//   likelihood (FP64 log-likelihood, FP32 exp) with FP64 moment sums ->
//   normaliser, log-likelihood, grid design -> interpolation onto the new grid
//   (cubic Lagrange for 2-D, trigonometric for 1-D) -> FP64 renormalisation ->
//   store.
// HBM traffic per filter: the density read once and written once.
#include <algorithm>
#include <cstring>
#include <vector>

#include "api_internal.h"

namespace pmf {

constexpr int FUSED_THREADS = 1024;
constexpr int FUSED_WAVES = FUSED_THREADS / 64;
constexpr int FUSED_LMAX = 64;

struct FConst {
    KModel m;
    PredictArgs pa;
};

struct BItem {
    float* P[2];
    DevDesc* d;
    const FConst* k;
    int idx;       // row of z / loglik
    int n0, n1;    // rows (1 for nx = 1) and row length
    int nx;
};

struct FShared {
    Grid g;        // grid after the move
    Grid gn;       // proposed grid
    double coef[(2 * FUSED_LMAX + 1) * 6];
    double h, etr;
    int l, ok, sep, item, bad;
    int fast;                  // linear-Gaussian log-likelihood as a quadratic in u
    double q0, qb[2], qQ[3];   // log l = q0 + qb.u - 1/2 u^T Q u  (Q packed 00, 11, 01)
    double s, inv_mass, loglik, mass;
    double amap[4], bmap[2];   // new index coords -> old index coords
    double inv_mass2;
    double red[FUSED_WAVES][8];
    double bits;
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

// One Stockham pass over nlines lines; element i of line L at L*ls + i*es.
// tw[m] = e^{-2 pi i m / n}.
template <int R>
__device__ void fpass(const float2* __restrict__ in, float2* __restrict__ out, int n, int Ns, int nlines, int ls,
                      int es, int sign, const float2* __restrict__ tw, bool line_fast) {
    const int nb = n / R;
    const int tot = nlines * nb;
    const int tws = n / (Ns * R);
    for (int w = threadIdx.x; w < tot; w += blockDim.x) {
        int line, j;
        if (line_fast) {
            line = w % nlines;
            j = w / nlines;
        } else {
            j = w % nb;
            line = w / nb;
        }
        const float2* src = in + line * ls;
        float2* dst = out + line * ls;
        float2 v[R];
#pragma unroll
        for (int r = 0; r < R; ++r) v[r] = src[(j + r * nb) * es];
        const int k = j % Ns;
        if (k) {
#pragma unroll
            for (int r = 1; r < R; ++r) {
                float2 t = tw[k * r * tws];
                if (sign > 0) t.y = -t.y;
                v[r] = f2mul(v[r], t);
            }
        }
        if (R == 2) fdft2(v);
        if (R == 3) fdft3(v, sign);
        if (R == 4) fdft4(v, sign);
        if (R == 8) fdft8(v, sign);
        const int base = (j / Ns) * Ns * R + k;
#pragma unroll
        for (int r = 0; r < R; ++r) dst[(base + r * Ns) * es] = v[r];
    }
}

// FFT of length n on nlines lines, ping-ponging between a and b; returns the
// buffer holding the result (natural order).
__device__ float2* ffft(float2* a, float2* b, int n, int nlines, int ls, int es, int sign, const float2* tw,
                        bool line_fast) {
    const FftPlan p = make_plan(n);
    int Ns = 1;
    float2* in = a;
    float2* out = b;
    for (int q = 0; q < p.np; ++q) {
        const int R = p.r[q];
        if (R == 8) fpass<8>(in, out, n, Ns, nlines, ls, es, sign, tw, line_fast);
        else if (R == 4) fpass<4>(in, out, n, Ns, nlines, ls, es, sign, tw, line_fast);
        else if (R == 3) fpass<3>(in, out, n, Ns, nlines, ls, es, sign, tw, line_fast);
        else fpass<2>(in, out, n, Ns, nlines, ls, es, sign, tw, line_fast);
        __syncthreads();
        float2* t = in;
        in = out;
        out = t;
        Ns *= R;
    }
    return in;
}

__device__ inline double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}
__device__ inline double wave_max(double v) {
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    return v;
}

// fixed-order workgroup sums of NV doubles; the result is valid in thread 0
template <int NV>
__device__ void fblock_sum(double* v, FShared& S) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
    for (int q = 0; q < NV; ++q) v[q] = wave_sum(v[q]);
    if (lane == 0)
        for (int q = 0; q < NV; ++q) S.red[wave][q] = v[q];
    __syncthreads();
    if (threadIdx.x == 0) {
        const int nw = blockDim.x >> 6;
        for (int q = 0; q < NV; ++q) {
            double acc = 0.0;
            for (int w = 0; w < nw; ++w) acc += S.red[w][q];
            v[q] = acc;
        }
    }
    __syncthreads();
}

__device__ double fblock_max(double v, FShared& S) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    v = wave_max(v);
    if (lane == 0) S.red[wave][0] = v;
    __syncthreads();
    double r = S.red[0][0];
    const int nw = blockDim.x >> 6;
    for (int w = 1; w < nw; ++w) r = fmax(r, S.red[w][0]);
    __syncthreads();
    return r;
}

// log p(z | x) at index coordinates u (general measurement models, FP64)
__device__ double floglik(const KModel& m, const FShared& S, const double* u, const double* z) {
    if (S.fast) {
        const double q = S.qQ[0] * u[0] * u[0] + S.qQ[1] * u[1] * u[1] + 2.0 * S.qQ[2] * u[0] * u[1];
        return S.q0 + S.qb[0] * u[0] + S.qb[1] * u[1] - 0.5 * q;
    }
    double x[3];
    for (int i = 0; i < m.nx; ++i) {
        double s = S.g.c[i];
        for (int k = 0; k < m.nx; ++k) s += S.g.M[i * 3 + k] * u[k];
        x[i] = s;
    }
    double hx[3] = {0, 0, 0};
    if (m.meas == PMF_H_LINEAR) {
        for (int i = 0; i < m.nz; ++i) {
            double s = 0.0;
            for (int k = 0; k < m.nx; ++k) s += m.H[i * 3 + k] * x[k];
            hx[i] = s;
        }
    } else if (m.meas == PMF_H_CUBIC1) {
        hx[0] = m.hp[0] * x[0] + m.hp[1] * x[0] * x[0] * x[0];
    } else {
        double s = 0.0;
        for (int k = 0; k < m.nx; ++k) s += x[k] * x[k];
        hx[0] = sqrt(s);
    }
    double best = -INFINITY, terms[MAXMIX];
    for (int g = 0; g < m.ncomp; ++g) {
        double r[3];
        for (int i = 0; i < m.nz; ++i) r[i] = z[i] - hx[i] - m.nmean[g][i];
        double q = 0.0;
        for (int i = 0; i < m.nz; ++i)
            for (int k = 0; k < m.nz; ++k) q += r[i] * m.nRi[g][i * 3 + k] * r[k];
        terms[g] = m.lw[g] - 0.5 * q;
        best = terms[g] > best ? terms[g] : best;
    }
    if (m.ncomp == 1) return terms[0];
    double acc = 0.0;
    for (int g = 0; g < m.ncomp; ++g) acc += exp(terms[g] - best);
    return best + log(acc);
}

// Thread 0: substeps, stage coefficients, trace factor, grid move (into S.g).
__device__ void fplan(const PredictArgs& a, const DevDesc* d, FShared& S) {
    const int n = a.nx;
    S.g = d->g;
    double Mi[9];
    mat_copy(Mi, S.g.Mi);
    int l = a.lmin;
    S.bad = 0;
    if (a.integ == PMF_INT_RK4 && a.T > 0.0) {
        double lam = 0.0;
        const double* Es[3] = {nullptr, a.emh, a.emT};
        for (int q = 0; q < 3; ++q) {
            double E[9], t1[9], Dy[9];
            if (q == 0) {
                mat_copy(E, a.D);
            } else {
                mat_mul(t1, Es[q], a.D, n);
                mat_mul_bt(E, t1, Es[q], n);
            }
            sandwich_inv(Dy, Mi, E, n);
            double lb = 0.0;
            for (int i = 0; i < n; ++i)
                for (int j = 0; j < n; ++j) lb += fabs(Dy[i * 3 + j]) * a.rho[i] * a.rho[j];
            lb *= 0.5;
            lam = lb > lam ? lb : lam;
        }
        const double need = ceil(a.T * lam / RK4_STABLE_STEP);
        if (need > (double)l) l = need > (double)FUSED_LMAX ? FUSED_LMAX + 1 : (int)need;
    }
    if (l > FUSED_LMAX) {
        l = FUSED_LMAX;
        S.bad = 1;
    }
    const double h = a.T / l;
    if (a.integ == PMF_INT_EXACT) {
        double Wy[9];
        sandwich_inv(Wy, Mi, a.W, n);
        pack_sym(S.coef, Wy);
    } else {
        const int cnt = (a.integ == PMF_INT_RK4) ? 2 * l + 1 : l;
        const double dt = (a.integ == PMF_INT_RK4) ? 0.5 * h : h;
        double Estep[9], Ek[9], t1[9], E[9], Dy[9], nxt[9];
        expm3(Estep, a.A, -dt, n);
        mat_eye(Ek, n);
        for (int k = 0; k < cnt; ++k) {
            mat_mul(t1, Ek, a.D, n);
            mat_mul_bt(E, t1, Ek, n);
            sandwich_inv(Dy, Mi, E, n);
            pack_sym(S.coef + 6 * k, Dy);
            mat_mul(nxt, Ek, Estep, n);
            mat_copy(Ek, nxt);
        }
    }
    S.l = l;
    S.h = h;
    S.etr = a.etr;
    double c2[3], M2[9];
    mat_vec(c2, a.Phi, S.g.c, n);
    mat_mul(M2, a.Phi, S.g.M, n);
    for (int i = 0; i < n; ++i) S.g.c[i] = c2[i];
    mat_copy(S.g.M, M2);
    grid_finish(S.g, n);
}

// linear-Gaussian fast path: log l(u) as a quadratic in index coordinates
__device__ void flik_setup(const KModel& m, const double* z, FShared& S) {
    S.fast = (m.meas == PMF_H_LINEAR && m.ncomp == 1 && m.nx <= 2) ? 1 : 0;
    if (!S.fast) return;
    const int nx = m.nx, nz = m.nz;
    double r0[3], G[9];
    for (int i = 0; i < nz; ++i) {
        double hc = 0.0;
        for (int k = 0; k < nx; ++k) hc += m.H[i * 3 + k] * S.g.c[k];
        r0[i] = z[i] - m.nmean[0][i] - hc;
        for (int b = 0; b < nx; ++b) {
            double s = 0.0;
            for (int k = 0; k < nx; ++k) s += m.H[i * 3 + k] * S.g.M[k * 3 + b];
            G[i * 3 + b] = s;
        }
    }
    // log l = lw - 1/2 (r0 - G u)^T Ri (r0 - G u)
    double Rir0[3];
    for (int i = 0; i < nz; ++i) {
        double s = 0.0;
        for (int k = 0; k < nz; ++k) s += m.nRi[0][i * 3 + k] * r0[k];
        Rir0[i] = s;
    }
    double rr = 0.0;
    for (int i = 0; i < nz; ++i) rr += r0[i] * Rir0[i];
    S.q0 = m.lw[0] - 0.5 * rr;
    double Qf[4] = {0, 0, 0, 0};
    S.qb[0] = S.qb[1] = 0.0;
    for (int a = 0; a < nx; ++a) {
        double s = 0.0;
        for (int i = 0; i < nz; ++i) s += G[i * 3 + a] * Rir0[i];
        S.qb[a] = s;
        for (int b = 0; b < nx; ++b) {
            double t = 0.0;
            for (int i = 0; i < nz; ++i)
                for (int k = 0; k < nz; ++k) t += G[i * 3 + a] * m.nRi[0][i * 3 + k] * G[k * 3 + b];
            Qf[a * 2 + b] = t;
        }
    }
    S.qQ[0] = Qf[0];
    S.qQ[1] = Qf[3];
    S.qQ[2] = Qf[1];
}

__device__ inline void cubic_weights(double t, float* w) {
    w[0] = (float)(-t * (t - 1.0) * (t - 2.0) / 6.0);
    w[1] = (float)((t + 1.0) * (t - 1.0) * (t - 2.0) / 2.0);
    w[2] = (float)(-(t + 1.0) * t * (t - 2.0) / 2.0);
    w[3] = (float)((t + 1.0) * t * (t - 1.0) / 6.0);
}

// ---------------------------------------------------------------- the kernel

__global__ void k_batch_reset(int* ctr) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *ctr = 0;
}

struct FBufs {
    float2* A;
    float2* B;
    float2* twr;   // 128: row transform (n1/2 points)
    float2* twc;   // 256: column transform (n0 points)
    float2* twp;   // 130: r2c split twiddles e^{-2 pi i s / n1}
    double* trig;  // 2 x 256: cos, sin of pi j / n1
};

// Time update of one filter with the density resident in LDS.  Uses S.coef,
// S.l, S.h, S.etr from fplan.  Returns the buffer holding the predicted real
// density, element (r, j) at r * 2 * (n1/2 + 1) + j.
__device__ float2* fused_predict(const BItem& I, const KModel& m, const float* Pin, FShared& S, const FBufs& F) {
    const int tid = threadIdx.x, nt = blockDim.x;
    const int n0 = I.n0, n1 = I.n1, nx = I.nx;
    const int h1 = n1 / 2, pitch = h1 + 1;
    float2* bufA = F.A;
    float2* bufB = F.B;
    // load rows as complex pairs (x_{2k}, x_{2k+1})
    const float2* Pin2 = reinterpret_cast<const float2*>(Pin);
    for (int e = tid; e < n0 * h1; e += nt) {
        const int r = e / h1, k = e - r * h1;
        bufA[r * pitch + k] = Pin2[e];
    }
    __syncthreads();
    // ---- forward: rows (r2c), columns
    float2* cur = ffft(bufA, bufB, h1, n0, pitch, 1, -1, F.twr, false);
    float2* oth = (cur == bufA) ? bufB : bufA;
    for (int e = tid; e < n0 * (h1 + 1); e += nt) {
        const int r = e / (h1 + 1), s = e - r * (h1 + 1);
        const float2 Zs = cur[r * pitch + (s == h1 ? 0 : s)];
        const float2 Zc = f2conj(cur[r * pitch + (s == 0 ? 0 : h1 - s)]);
        const float2 E = f2scale(f2add(Zs, Zc), 0.5f);
        const float2 Dd = f2sub(Zs, Zc);
        // X_s = E - i/2 W^s (Z_s - conj Z_{h1-s})
        const float2 t = f2mul(F.twp[s], Dd);
        oth[r * pitch + s] = f2add(E, make_float2(0.5f * t.y, -0.5f * t.x));
    }
    __syncthreads();
    cur = oth;
    oth = (cur == bufA) ? bufB : bufA;
    if (nx == 2) {
        cur = ffft(cur, oth, n0, h1 + 1, 1, pitch, -1, F.twc, true);
        oth = (cur == bufA) ? bufB : bufA;
    }
    // ---- per-mode gain, with 1/(n0 n1) of the unnormalised transforms
    {
        const float scale = (float)(S.etr / ((double)n0 * n1));
        const int l = S.l, integ = m.integ;
        const float hh = (float)S.h;
        for (int e = tid; e < n0 * (h1 + 1); e += nt) {
            const int s0 = e / (h1 + 1), s1 = e - s0 * (h1 + 1);
            float a1[2], a2[2];
            {
                const int kk = (s1 < h1) ? s1 : s1 - n1;
                const float kap = 6.283185307179586f * kk / n1;
                const int ax = (nx == 2) ? 1 : 0;
                a2[ax] = kap * kap;
                a1[ax] = (s1 == h1) ? 0.f : kap;
            }
            if (nx == 2) {
                const int kk = (s0 < n0 / 2) ? s0 : s0 - n0;
                const float kap = 6.283185307179586f * kk / n0;
                a2[0] = kap * kap;
                a1[0] = (2 * s0 == n0) ? 0.f : kap;
            } else {
                a1[1] = 0.f;
                a2[1] = 0.f;
            }
            auto sigma = [&](const double* p) {
                return (float)p[0] * a2[0] + (float)p[1] * a2[1] + 2.f * (float)p[3] * a1[0] * a1[1];
            };
            float g;
            if (integ == PMF_INT_EXACT) {
                g = expf(-0.5f * sigma(S.coef));
            } else if (integ == PMF_INT_EULER) {
                g = 1.f;
                for (int q = 0; q < l; ++q) g = g / (1.f + 0.5f * hh * sigma(S.coef + 6 * q));
            } else {
                g = 1.f;
                for (int q = 0; q < l; ++q) {
                    const float la = -0.5f * sigma(S.coef + 12 * q);
                    const float lb = -0.5f * sigma(S.coef + 12 * q + 6);
                    const float lc = -0.5f * sigma(S.coef + 12 * q + 12);
                    const float y2 = 1.f + 0.5f * hh * la;
                    const float y3 = 1.f + 0.5f * hh * lb * y2;
                    const float y4 = 1.f + hh * lb * y3;
                    g *= 1.f + hh / 6.f * (la + 2.f * lb * y2 + 2.f * lb * y3 + lc * y4);
                }
            }
            const float2 v = cur[s0 * pitch + s1];
            cur[s0 * pitch + s1] = f2scale(v, g * scale);
        }
    }
    __syncthreads();
    // ---- inverse: columns, rows (c2r)
    if (nx == 2) {
        cur = ffft(cur, oth, n0, h1 + 1, 1, pitch, +1, F.twc, true);
        oth = (cur == bufA) ? bufB : bufA;
    }
    for (int e = tid; e < n0 * h1; e += nt) {
        const int r = e / h1, s = e - r * h1;
        const float2 Xs = cur[r * pitch + s];
        const float2 Xc = f2conj(cur[r * pitch + h1 - s]);
        const float2 Aa = f2add(Xs, Xc);
        const float2 Bb = f2mul(f2conj(F.twp[s]), f2sub(Xs, Xc));
        // Z_s = (X_s + conj X_{h1-s}) + i W^{-s} (X_s - conj X_{h1-s})
        oth[r * pitch + s] = make_float2(Aa.x - Bb.y, Aa.y + Bb.x);
    }
    __syncthreads();
    return ffft(oth, cur, h1, n0, pitch, 1, +1, F.twr, false);
}

// store the predicted density (pitched in LDS) with the moved grid, update rejected
__device__ void fused_store_predicted(const BItem& I, const float* Pr, float* Pout, DevDesc* d, FShared& S,
                                      double* ll_out, int par, int extra_bits) {
    const int n0 = I.n0, n1 = I.n1, rp = 2 * (n1 / 2 + 1);
    for (int e = threadIdx.x; e < n0 * n1; e += blockDim.x) {
        const int r = e / n1, j = e - r * n1;
        Pout[e] = Pr[r * rp + j];
    }
    if (threadIdx.x == 0) {
        d->g = S.g;
        d->gn = S.g;
        d->t += I.k->pa.T;
        d->l = S.l;
        d->h = S.h;
        d->etr = S.etr;
        d->loglik = NAN;
        d->status |= PMF_E_DEGENERATE | extra_bits;
        d->par = 1 - par;
        ll_out[I.idx] = NAN;
    }
    __syncthreads();
}

__global__ void __launch_bounds__(FUSED_THREADS)
k_fused(const BItem* __restrict__ items, int nitems, int* ctr, const double* __restrict__ zall, int nzmax,
        double* __restrict__ ll_out, int bufcplx) {
    extern __shared__ __align__(16) unsigned char fsm[];
    __shared__ FShared S;
    FBufs F;
    F.A = reinterpret_cast<float2*>(fsm);
    F.B = F.A + bufcplx;
    F.twr = F.B + bufcplx;
    F.twc = F.twr + 128;
    F.twp = F.twc + 256;
    F.trig = reinterpret_cast<double*>(F.twp + 130);
    const int tid = threadIdx.x, nt = blockDim.x;

    for (;;) {
        if (tid == 0) S.item = atomicAdd(ctr, 1);
        __syncthreads();
        const int it = S.item;
        __syncthreads();
        if (it >= nitems) break;
        const BItem I = items[it];
        const KModel& m = I.k->m;
        DevDesc* d = I.d;
        const int n0 = I.n0, n1 = I.n1, nx = I.nx;
        const int h1 = n1 / 2, pitch = h1 + 1;
        const int par = d->par;
        const float* Pin = I.P[par];
        float* Pout = I.P[1 - par];
        const double* z = zall + (size_t)I.idx * nzmax;

        if (tid == 0) {
            fplan(I.k->pa, d, S);
            flik_setup(m, z, S);
        }
        for (int i = tid; i < h1; i += nt) {
            float s, c;
            sincospif(-2.0f * i / h1, &s, &c);
            F.twr[i] = make_float2(c, s);
        }
        for (int i = tid; i < n0; i += nt) {
            float s, c;
            sincospif(-2.0f * i / n0, &s, &c);
            F.twc[i] = make_float2(c, s);
        }
        for (int i = tid; i <= h1; i += nt) {
            float s, c;
            sincospif(-2.0f * i / n1, &s, &c);
            F.twp[i] = make_float2(c, s);
        }
        __syncthreads();
        float2* cur = fused_predict(I, m, Pin, S, F);
        float2* oth = (cur == F.A) ? F.B : F.A;
        const float* Pr = reinterpret_cast<const float*>(cur);   // predicted, (r, j) at r*rp + j
        float* Po = reinterpret_cast<float*>(oth);               // posterior, same layout
        const int rp = 2 * pitch;

        // ---- likelihood: max pass, multiply pass with FP64 sums
        const int npt = n0 * n1;
        const double half0 = (double)(n0 / 2), half1 = (double)(n1 / 2);
        double mx = -INFINITY;
        for (int e = tid; e < npt; e += nt) {
            const int r = e / n1, j = e - r * n1;
            double u[2];
            if (nx == 2) {
                u[0] = r - half0;
                u[1] = j - half1;
            } else {
                u[0] = j - half1;
                u[1] = 0.0;
            }
            mx = fmax(mx, floglik(m, S, u, z));
        }
        const double sh = fblock_max(mx, S);
        double acc[7] = {0, 0, 0, 0, 0, 0, 0};
        for (int e = tid; e < npt; e += nt) {
            const int r = e / n1, j = e - r * n1;
            double u[2];
            bool edge;
            if (nx == 2) {
                u[0] = r - half0;
                u[1] = j - half1;
                edge = (r == 0 || r == n0 - 1 || j == 0 || j == n1 - 1);
            } else {
                u[0] = j - half1;
                u[1] = 0.0;
                edge = (j == 0 || j == n1 - 1);
            }
            const double L = floglik(m, S, u, z);
            const float v = Pr[r * rp + j] * expf((float)(L - sh));
            Po[r * rp + j] = v;
            const double w = (double)v;
            acc[0] += w;
            acc[1] += w * u[0];
            acc[2] += w * u[1];
            acc[3] += w * u[0] * u[0];
            acc[4] += w * u[1] * u[1];
            acc[5] += w * u[0] * u[1];
            if (edge) acc[6] += w;
        }
        fblock_sum<7>(acc, S);
        if (tid == 0) {
            const double mass = S.g.vol * acc[0];
            S.ok = !S.bad && isfinite(sh) && isfinite(mass) && mass > 0.0;
            S.bits = 0.0;
            if (S.ok) {
                S.s = sh;
                S.mass = mass;
                S.inv_mass = 1.0 / mass;
                S.loglik = sh + log(mass);
                // moments in index coordinates -> physical
                const double ub[2] = {acc[1] / acc[0], acc[2] / acc[0]};
                double Cu[9];
                mat_zero(Cu);
                Cu[0] = acc[3] / acc[0] - ub[0] * ub[0];
                Cu[4] = acc[4] / acc[0] - ub[1] * ub[1];
                Cu[1] = Cu[3] = acc[5] / acc[0] - ub[0] * ub[1];
                double mu[3], mean[3], t1[9], C[9], cov[9];
                mat_vec(mu, S.g.M, ub, nx);
                for (int a = 0; a < nx; ++a) mean[a] = S.g.c[a] + mu[a];
                mat_mul(t1, S.g.M, Cu, nx);
                mat_mul_bt(C, t1, S.g.M, nx);
                mat_zero(cov);
                for (int a = 0; a < nx; ++a)
                    for (int b = 0; b < nx; ++b) cov[a * 3 + b] = 0.5 * (C[a * 3 + b] + C[b * 3 + a]);
                if (acc[6] / acc[0] > BOUNDARY_TOL) S.bits = (double)PMF_W_BOUNDARY;
                // grid design
                mat_zero(S.gn.M);
                for (int a = 0; a < nx; ++a) {
                    const double v = cov[a * 3 + a] + m.Wnom[a * 3 + a];
                    if (!(v > 0.0) || !isfinite(v)) S.ok = 0;
                    const double hw = m.span * sqrt(v);
                    S.gn.M[a * 3 + a] = 2.0 * hw / (nx == 2 ? (a == 0 ? n0 : n1) : n1);
                    S.gn.c[a] = mean[a];
                }
                for (int a = nx; a < 3; ++a) S.gn.c[a] = 0.0;
                grid_finish(S.gn, nx);
                bool aligned = true;
                for (int a = 0; a < nx; ++a)
                    for (int b = 0; b < nx; ++b)
                        if (a != b && S.g.M[a * 3 + b] != 0.0) aligned = false;
                S.sep = (m.interp == PMF_INTERP_AUTO && aligned) ? 1 : 0;
                if (nx == 2 && S.sep) S.ok = 0;   // separable 2-D regrid is not fused
                // new index coordinates u' -> old index coordinates
                double t2[9], dc[3], bb[3];
                mat_mul(t2, S.g.Mi, S.gn.M, nx);
                for (int a = 0; a < nx; ++a) dc[a] = S.gn.c[a] - S.g.c[a];
                mat_vec(bb, S.g.Mi, dc, nx);
                if (nx == 2) {
                    S.amap[0] = t2[0];
                    S.amap[1] = t2[1];
                    S.amap[2] = t2[3];
                    S.amap[3] = t2[4];
                    S.bmap[0] = bb[0] + half0;
                    S.bmap[1] = bb[1] + half1;
                } else {
                    S.amap[0] = t2[0];
                    S.bmap[0] = bb[0] + half1;
                }
            }
        }
        __syncthreads();
        if (!S.ok) {
            fused_store_predicted(I, Pr, Pout, d, S, ll_out, par, S.bad ? PMF_E_INVALID : 0);
            continue;
        }
        // ---- interpolation of the posterior onto the new grid (dense, into cur)
        float* Qv = reinterpret_cast<float*>(cur);
        const float inv_mass = (float)S.inv_mass;
        if (nx == 1) {
            for (int j = tid; j < n1; j += nt) {
                double sv, cv;
                sincospi((double)j / n1, &sv, &cv);
                F.trig[j] = cv;
                F.trig[256 + j] = sv;
            }
        }
        __syncthreads();   // every thread is done reading the predicted density
        double macc[1] = {0.0};
        for (int e = tid; e < npt; e += nt) {
            const int r = e / n1, j = e - r * n1;
            float val = 0.f;
            if (nx == 2) {
                const double u0 = r - half0, u1 = j - half1;
                const double nu0 = S.amap[0] * u0 + S.amap[1] * u1 + S.bmap[0];
                const double nu1 = S.amap[2] * u0 + S.amap[3] * u1 + S.bmap[1];
                if (nu0 >= 0.0 && nu0 <= (double)(n0 - 1) && nu1 >= 0.0 && nu1 <= (double)(n1 - 1)) {
                    const int i0 = (int)floor(nu0), i1 = (int)floor(nu1);
                    float w0[4], w1[4];
                    cubic_weights(nu0 - i0, w0);
                    cubic_weights(nu1 - i1, w1);
#pragma unroll
                    for (int a = 0; a < 4; ++a) {
                        const int ra = i0 - 1 + a;
                        if (ra < 0 || ra >= n0) continue;
                        float rs = 0.f;
#pragma unroll
                        for (int b = 0; b < 4; ++b) {
                            const int cb = i1 - 1 + b;
                            if (cb < 0 || cb >= n1) continue;
                            rs += w1[b] * Po[ra * rp + cb];
                        }
                        val += w0[a] * rs;
                    }
                }
            } else {
                const double nu = S.amap[0] * (j - half1) + S.bmap[0];
                if (nu >= 0.0 && nu <= (double)(n1 - 1)) {
                    const double fl = floor(nu);
                    if (nu == fl) {
                        val = Po[(int)fl];
                    } else {
                        double sa, ca, spn, cpn;
                        sincospi(nu / n1, &sa, &ca);
                        sincospi(nu, &spn, &cpn);
                        double acc1 = 0.0;
                        for (int q = 0; q < n1; ++q) {
                            const double cb = F.trig[q], sb = F.trig[256 + q];
                            const double num = ca * cb + sa * sb;
                            const double den = sa * cb - ca * sb;
                            const double wgt = ((q & 1) ? -spn : spn) * num / (n1 * den);
                            acc1 += wgt * (double)Po[q];
                        }
                        val = (float)acc1;
                    }
                }
            }
            val *= inv_mass;
            Qv[e] = val;
            macc[0] += (double)val;
        }
        fblock_sum<1>(macc, S);
        if (tid == 0) {
            const double mass2 = S.gn.vol * macc[0];
            if (!(mass2 > 0.0) || !isfinite(mass2)) {
                S.ok = 0;
            } else {
                S.inv_mass2 = 1.0 / mass2;
            }
        }
        __syncthreads();
        if (!S.ok) {
            // the new grid lost the mass: redo the time update and keep it
            float2* again = fused_predict(I, m, Pin, S, F);
            fused_store_predicted(I, reinterpret_cast<const float*>(again), Pout, d, S, ll_out, par, 0);
            continue;
        }
        const float inv2 = (float)S.inv_mass2;
        for (int e = tid; e < npt; e += nt) Pout[e] = Qv[e] * inv2;
        if (tid == 0) {
            d->g = S.gn;
            d->gn = S.gn;
            d->t += I.k->pa.T;
            d->l = S.l;
            d->h = S.h;
            d->etr = S.etr;
            d->loglik = S.loglik;
            d->status |= (int)S.bits;
            d->par = 1 - par;
            ll_out[I.idx] = S.loglik;
        }
        __syncthreads();
    }
}

}  // namespace pmf

// ==================================================================== host side

struct BatchCache {
    std::vector<pmf_filter*> filters;
    double T = 0.0;
    hipStream_t stream = nullptr;
    int n = 0, nzmax = 1;
    pmf::BItem* d_items = nullptr;
    pmf::FConst* d_consts = nullptr;
    double* d_z = nullptr;
    double* d_ll = nullptr;
    int* d_ctr = nullptr;
    double* h_z[2] = {nullptr, nullptr};
    hipEvent_t ev[2] = {nullptr, nullptr};
    int slot = 0;
    size_t lds = 0;
    int grid = 0, bufcplx = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace pmf {

static void cache_free(pmf_ctx* ctx, BatchCache* c) {
    if (!c) return;
    (void)hipDeviceSynchronize();
    if (c->exec) (void)hipGraphExecDestroy(c->exec);
    if (c->graph) (void)hipGraphDestroy(c->graph);
    ctx_free(ctx, c->d_items, nullptr);
    ctx_free(ctx, c->d_consts, nullptr);
    ctx_free(ctx, c->d_z, nullptr);
    ctx_free(ctx, c->d_ll, nullptr);
    ctx_free(ctx, c->d_ctr, nullptr);
    for (int i = 0; i < 2; ++i) {
        if (c->h_z[i]) (void)hipHostFree(c->h_z[i]);
        if (c->ev[i]) (void)hipEventDestroy(c->ev[i]);
    }
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

// Filters whose density lives in the batch buffer pair must be brought back
// before the generic kernels touch them (and the other way round).
hipError_t batch_leave(pmf_filter* f) {
    if (!f->in_batch) return hipSuccess;
    hipError_t e = hipDeviceSynchronize();
    int par = 0;
    if (e == hipSuccess) e = hipMemcpy(&par, &f->desc->par, sizeof(int), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return e;
    f->cur = par;
    f->in_batch = false;
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

bool batch_fusable(const pmf_filter* f, std::string* why) {
    const pmf_model& m = f->model;
    if (m.grid != PMF_GRID_FOURIER) return *why = "Chebyshev grid", false;
    if (m.precision != PMF_FP32) return *why = "FP64 density", false;
    if (m.nx > 2) return *why = "nx > 2", false;
    if (m.nx == 2 && (m.N[0] > 128 || m.N[1] > 128)) return *why = "2-D N above 128", false;
    if (m.nx == 1 && m.N[0] > 256) return *why = "1-D N above 256", false;
    if (m.nx == 2 && m.interp == PMF_INTERP_AUTO && m.A[1] == 0.0 && m.A[2] == 0.0)
        return *why = "diagonal A: separable 2-D regrid", false;
    if (m.nx == 1 && m.interp == PMF_INTERP_LAGRANGE) return *why = "1-D Lagrange regrid", false;
    if (m.nx == 2 && (m.N[1] / 2) > 128) return *why = "row too long", false;
    return true;
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
    int maxcplx = 0;
    for (int i = 0; i < n; ++i) {
        pmf_filter* f = filters[i];
        consts[i].m = f->km;
        consts[i].pa = predict_args(f, T);
        BItem& b = items[i];
        b.P[0] = static_cast<float*>(f->buf[0]);
        b.P[1] = static_cast<float*>(f->buf[1]);
        b.d = f->desc;
        b.idx = i;
        b.nx = f->model.nx;
        b.n0 = f->model.nx == 2 ? f->model.N[0] : 1;
        b.n1 = f->model.nx == 2 ? f->model.N[1] : f->model.N[0];
        maxcplx = std::max(maxcplx, b.n0 * (b.n1 / 2 + 1));
    }
    // largest grid first
    std::vector<int> order(n);
    for (int i = 0; i < n; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        return items[a].n0 * items[a].n1 > items[b].n0 * items[b].n1;
    });
    bool ok = true;
    auto A = [&](size_t bytes) {
        void* p = ctx_alloc(ctx, bytes, st);
        if (!p) ok = false;
        return p;
    };
    c->d_consts = static_cast<FConst*>(A(sizeof(FConst) * n));
    c->d_items = static_cast<BItem*>(A(sizeof(BItem) * n));
    c->d_z = static_cast<double*>(A(sizeof(double) * n * nzmax));
    c->d_ll = static_cast<double*>(A(sizeof(double) * n));
    c->d_ctr = static_cast<int*>(A(sizeof(int)));
    if (!ok) return fail(PMF_E_NOMEM, "batch allocation failed");
    std::vector<BItem> sorted(n);
    for (int i = 0; i < n; ++i) {
        sorted[i] = items[order[i]];
        sorted[i].k = c->d_consts + order[i];
    }
    hipError_t e = hipMemcpy(c->d_consts, consts.data(), sizeof(FConst) * n, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(c->d_items, sorted.data(), sizeof(BItem) * n, hipMemcpyHostToDevice);
    for (int i = 0; i < 2 && e == hipSuccess; ++i) {
        e = hipHostMalloc(reinterpret_cast<void**>(&c->h_z[i]), sizeof(double) * n * nzmax, hipHostMallocDefault);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&c->ev[i], hipEventDisableTiming);
    }
    if (e != hipSuccess) return hip_fail(e, "batch setup");
    c->bufcplx = maxcplx;
    c->lds = 2 * (size_t)maxcplx * sizeof(float2) + (128 + 256 + 130) * sizeof(float2) + 512 * sizeof(double);
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_fused), hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)c->lds);
    if (e != hipSuccess) return hip_fail(e, "fused kernel LDS attribute");
    int per_cu = 0;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_fused, FUSED_THREADS, c->lds);
    if (e != hipSuccess) return hip_fail(e, "occupancy");
    if (per_cu < 1) return fail(PMF_E_INVALID, "fused kernel does not fit on a compute unit");
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, ctx->device);
    if (e != hipSuccess) return hip_fail(e, "device properties");
    c->grid = std::min(n, per_cu * prop.multiProcessorCount);
    // record the step: reset the work counter, run the fused kernel
    hipStream_t cap;
    e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_batch_reset, dim3(1), dim3(64), 0, cap, c->d_ctr);
        hipLaunchKernelGGL(k_fused, dim3(c->grid), dim3(FUSED_THREADS), c->lds, cap, c->d_items, n, c->d_ctr,
                           c->d_z, nzmax, c->d_ll, c->bufcplx);
        e = hipStreamEndCapture(cap, &c->graph);
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&c->exec, c->graph, nullptr, nullptr, 0);
    (void)hipStreamDestroy(cap);
    if (e != hipSuccess) return hip_fail(e, "graph capture");
    return PMF_OK;
}

}  // namespace pmf

extern "C" pmf_status pmf_batch_step(pmf_ctx* ctx, pmf_filter* const* filters, int n, double T, const double* z,
                                     double* loglik, void* stream) {
    using namespace pmf;
    if (!ctx || n < 1 || !filters || !z) return fail(PMF_E_INVALID, "NULL argument or n < 1");
    if (!std::isfinite(T) || !(T > 0.0)) return fail(PMF_E_INVALID, "T must be finite and > 0");
    int nzmax = 1;
    for (int i = 0; i < n; ++i) {
        if (!filters[i] || filters[i]->ctx != ctx) return fail(PMF_E_INVALID, "filter of another context");
        std::string why;
        if (!batch_fusable(filters[i], &why)) return fail(PMF_E_INVALID, "filter not fusable: " + why);
        nzmax = std::max(nzmax, filters[i]->model.nz);
        for (int j = i + 1; j < n && j < i + 2; ++j)
            if (filters[j] == filters[i]) return fail(PMF_E_INVALID, "filter listed twice");
    }
    for (int i = 0; i < n * nzmax; ++i)
        if (!std::isfinite(z[i])) return fail(PMF_E_INVALID, "non-finite measurement");
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    const hipStream_t st = static_cast<hipStream_t>(stream);
    BatchCache* c = ctx->batch;
    bool same = c && c->n == n && c->T == T && c->stream == st;
    if (same)
        for (int i = 0; i < n; ++i)
            if (c->filters[i] != filters[i]) {
                same = false;
                break;
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
    // stage z in pinned memory (two slots, each reused only after its copy finished)
    const int slot = c->slot;
    c->slot ^= 1;
    e = hipEventSynchronize(c->ev[slot]);
    if (e != hipSuccess) return hip_fail(e, "staging wait");
    std::memcpy(c->h_z[slot], z, sizeof(double) * n * nzmax);
    e = hipMemcpyAsync(c->d_z, c->h_z[slot], sizeof(double) * n * nzmax, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipEventRecord(c->ev[slot], st);
    if (e == hipSuccess) e = hipGraphLaunch(c->exec, st);
    if (e == hipSuccess && loglik) e = hipMemcpyAsync(loglik, c->d_ll, sizeof(double) * n, hipMemcpyDeviceToHost, st);
    if (e != hipSuccess) return hip_fail(e, "batch launch");
    return PMF_OK;
}
