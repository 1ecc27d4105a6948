// Generic kernels of libpmf: any grid kind, nx <= 3, FP32 or FP64 density.
// Every filter can take this path; the fused batched kernel (fused.hip) and the
// MFMA Chebyshev products (cheb_mfma.hip) are faster forms of parts of it.
#include "kernels.h"

namespace pmf {

// ------------------------------------------------------------------ helpers

template <typename T> struct V2;
template <> struct V2<float> { using t = float2; };
template <> struct V2<double> { using t = double2; };

template <typename C> __device__ inline C cadd(C a, C b) { C r; r.x = a.x + b.x; r.y = a.y + b.y; return r; }
template <typename C> __device__ inline C csub(C a, C b) { C r; r.x = a.x - b.x; r.y = a.y - b.y; return r; }
template <typename C> __device__ inline C cmul(C a, C b) {
    C r;
    r.x = a.x * b.x - a.y * b.y;
    r.y = a.x * b.y + a.y * b.x;
    return r;
}
// multiply by s*i, s = +-1
template <typename C> __device__ inline C cmul_si(C a, int s) {
    C r;
    r.x = -s * a.y;
    r.y = s * a.x;
    return r;
}
template <typename C, typename T> __device__ inline C cscale(C a, T f) { C r; r.x = a.x * f; r.y = a.y * f; return r; }

__device__ inline void sincospi_t(float x, float* s, float* c) { sincospif(x, s, c); }
__device__ inline void sincospi_t(double x, double* s, double* c) { sincospi(x, s, c); }
__device__ inline float exp_t(float x) { return expf(x); }
__device__ inline double exp_t(double x) { return exp(x); }

// R-point DFTs, X_k = sum_r a_r e^{s 2 pi i r k / R}
template <typename C, typename T> __device__ inline void dft2(C* a) {
    C t = a[0];
    a[0] = cadd(t, a[1]);
    a[1] = csub(t, a[1]);
}
template <typename C, typename T> __device__ inline void dft3(C* a, int s) {
    const T h = (T)0.86602540378443864676;
    C t = cadd(a[1], a[2]);
    C d = csub(a[1], a[2]);
    C m = csub(a[0], cscale(t, (T)0.5));
    a[0] = cadd(a[0], t);
    C rot = cscale(cmul_si(d, s), h);
    a[1] = cadd(m, rot);
    a[2] = csub(m, rot);
}
template <typename C, typename T> __device__ inline void dft4(C* a, int s) {
    C t0 = cadd(a[0], a[2]), t1 = csub(a[0], a[2]);
    C t2 = cadd(a[1], a[3]), t3 = cmul_si(csub(a[1], a[3]), s);
    a[0] = cadd(t0, t2);
    a[2] = csub(t0, t2);
    a[1] = cadd(t1, t3);
    a[3] = csub(t1, t3);
}
template <typename C, typename T> __device__ inline void dft8(C* a, int s) {
    C e[4] = {a[0], a[2], a[4], a[6]};
    C o[4] = {a[1], a[3], a[5], a[7]};
    dft4<C, T>(e, s);
    dft4<C, T>(o, s);
    const T r = (T)0.70710678118654752440;
    C w1;
    w1.x = r;
    w1.y = s * r;
    C w3;
    w3.x = -r;
    w3.y = s * r;
    C o1 = cmul(o[1], w1), o2 = cmul_si(o[2], s), o3 = cmul(o[3], w3);
    a[0] = cadd(e[0], o[0]);
    a[4] = csub(e[0], o[0]);
    a[1] = cadd(e[1], o1);
    a[5] = csub(e[1], o1);
    a[2] = cadd(e[2], o2);
    a[6] = csub(e[2], o2);
    a[3] = cadd(e[3], o3);
    a[7] = csub(e[3], o3);
}

// 5-point DFT from t = a_1 + a_4, a_2 + a_3 and d = a_1 - a_4, a_2 - a_3 with
// cos and sin of 2 pi / 5 and 4 pi / 5
template <typename C, typename T> __device__ inline void dft5(C* a, int s) {
    const T c1 = (T)0.30901699437494742410, c2 = (T)-0.80901699437494742410;
    const T s1 = (T)0.95105651629515357212, s2 = (T)0.58778525229247312917;
    const C t1 = cadd(a[1], a[4]), t2 = cadd(a[2], a[3]);
    const C d1 = csub(a[1], a[4]), d2 = csub(a[2], a[3]);
    const C m1 = cadd(a[0], cadd(cscale(t1, c1), cscale(t2, c2)));
    const C m2 = cadd(a[0], cadd(cscale(t1, c2), cscale(t2, c1)));
    const C r1 = cmul_si(cadd(cscale(d1, s1), cscale(d2, s2)), s);
    const C r2 = cmul_si(csub(cscale(d1, s2), cscale(d2, s1)), s);
    a[0] = cadd(a[0], cadd(t1, t2));
    a[1] = cadd(m1, r1);
    a[4] = csub(m1, r1);
    a[2] = cadd(m2, r2);
    a[3] = csub(m2, r2);
}

// R-point DFT for an odd prime R without a factored butterfly (7, 11, 13, 17), by
// pairing r with R - r: with t_r = a_r + a_{R-r}, d_r = a_r - a_{R-r} (r = 1..H,
// H = (R - 1) / 2), cos / sin of 2 pi m / R written c_m, s_m,
//   X_0 = a_0 + sum_r t_r,   X_k, X_{R-k} = A_k +- i s B_k  (k = 1..H),
//   A_k = a_0 + sum_r c_{rk} t_r,   B_k = sum_r s_{rk} d_r   (rk taken mod R),
// about a quarter of the real multiplications of the plain sum.  wr[m - 1] holds
// e^{-2 pi i m / R}, m = 1..H (from the LDS root table).
template <typename C, typename T, int R> __device__ inline void dft_odd(C* a, int s, const C* wr) {
    constexpr int H = (R - 1) / 2;
    T cm[H + 1], sm[H + 1];
#pragma unroll
    for (int m = 1; m <= H; ++m) {
        cm[m] = wr[m - 1].x;
        sm[m] = -wr[m - 1].y;
    }
    C t[H + 1], d[H + 1];
    C x0 = a[0];
#pragma unroll
    for (int r = 1; r <= H; ++r) {
        t[r] = cadd(a[r], a[R - r]);
        d[r] = csub(a[r], a[R - r]);
        x0 = cadd(x0, t[r]);
    }
#pragma unroll
    for (int k = 1; k <= H; ++k) {
        C A = a[0], Bv;
        Bv.x = (T)0;
        Bv.y = (T)0;
#pragma unroll
        for (int r = 1; r <= H; ++r) {
            const int m = (r * k) % R;
            const T c = m <= H ? cm[m] : cm[R - m];
            const T sn = m <= H ? sm[m] : -sm[R - m];
            A.x += c * t[r].x;
            A.y += c * t[r].y;
            Bv.x += sn * d[r].x;
            Bv.y += sn * d[r].y;
        }
        const C iB = cmul_si(Bv, s);
        a[k] = cadd(A, iB);
        a[R - k] = csub(A, iB);
    }
    a[0] = x0;
}

// One Stockham autosort pass over `nlines` lines held in LDS (pitch `pitch`).
// tw: the n-th roots of unity e^{-2 pi i m / n}, m < n, in LDS; the twiddle
// e^{sign 2 pi i k r / (Ns R)} is entry k r n / (Ns R) (conjugated for sign > 0).
template <typename T, int R>
__device__ void stockham_pass(const typename V2<T>::t* in, typename V2<T>::t* out, const typename V2<T>::t* tw,
                              int n, int Ns, int nlines, int pitch, int sign) {
    using C = typename V2<T>::t;
    constexpr bool ODD = R == 7 || R == 11 || R == 13 || R == 17;
    const int nb = n / R;
    // the R-th roots of unity e^{-2 pi i m / R}, m = 1..(R-1)/2, of the odd-prime
    // butterflies: entries m n / R of the table (dft_odd applies the sign)
    C wr[ODD ? (R - 1) / 2 : 1];
    if constexpr (ODD) {
#pragma unroll
        for (int m = 1; m <= (R - 1) / 2; ++m) wr[m - 1] = tw[m * nb];
    }
    for (int w = threadIdx.x; w < nlines * nb; w += blockDim.x) {
        const int line = w / nb, j = w - line * nb;
        const C* src = in + line * pitch;
        C* dst = out + line * pitch;
        C v[R];
#pragma unroll
        for (int r = 0; r < R; ++r) v[r] = src[j + r * nb];
        const int k = j % Ns;
        if (k) {
            const int step = k * (n / (Ns * R));
#pragma unroll
            for (int r = 1; r < R; ++r) {
                C w2 = tw[r * step];
                if (sign > 0) w2.y = -w2.y;
                v[r] = cmul(v[r], w2);
            }
        }
        if constexpr (R == 2) dft2<C, T>(v);
        if constexpr (R == 3) dft3<C, T>(v, sign);
        if constexpr (R == 4) dft4<C, T>(v, sign);
        if constexpr (R == 8) dft8<C, T>(v, sign);
        if constexpr (R == 5) dft5<C, T>(v, sign);
        if constexpr (ODD) dft_odd<C, T, R>(v, sign, wr);
        const int base = (j / Ns) * Ns * R + k;
#pragma unroll
        for (int r = 0; r < R; ++r) dst[base + r * Ns] = v[r];
    }
}

// The n-th roots of unity e^{-2 pi i m / n}, m < n, into tw (block-wide; the
// caller's barrier publishes them).
template <typename T>
__device__ inline void fft_roots(typename V2<T>::t* tw, int n) {
    for (int m = threadIdx.x; m < n; m += blockDim.x) {
        T sn, cs;
        sincospi_t((T)(-2 * m) / (T)n, &sn, &cs);
        tw[m].x = cs;
        tw[m].y = sn;
    }
}

// All passes of an n-point transform of ntl lines held in LDS (A, ping-ponging
// with B; tw from fft_roots); returns the buffer holding the result.  Every
// thread must call it.
// ODD: the plan may hold radix 7, 11, 13 or 17 (their butterflies are compiled in
// only then: they set the kernel's register count).
template <typename T, bool ODD>
__device__ typename V2<T>::t* fft_passes(typename V2<T>::t* A, typename V2<T>::t* B, const typename V2<T>::t* tw,
                                         int n, int ntl, int pitch, int sign, const FftPlan& plan) {
    using C = typename V2<T>::t;
    int Ns = 1;
    C* in = A;
    C* out = B;
    for (int p = 0; p < plan.np; ++p) {
        const int R = plan.r[p];
        if (R == 8) stockham_pass<T, 8>(in, out, tw, n, Ns, ntl, pitch, sign);
        else if (R == 4) stockham_pass<T, 4>(in, out, tw, n, Ns, ntl, pitch, sign);
        else if (R == 3) stockham_pass<T, 3>(in, out, tw, n, Ns, ntl, pitch, sign);
        else if (R == 5) stockham_pass<T, 5>(in, out, tw, n, Ns, ntl, pitch, sign);
        else if (ODD && R == 7) stockham_pass<T, ODD ? 7 : 2>(in, out, tw, n, Ns, ntl, pitch, sign);
        else if (ODD && R == 11) stockham_pass<T, ODD ? 11 : 2>(in, out, tw, n, Ns, ntl, pitch, sign);
        else if (ODD && R == 13) stockham_pass<T, ODD ? 13 : 2>(in, out, tw, n, Ns, ntl, pitch, sign);
        else if (ODD && R == 17) stockham_pass<T, ODD ? 17 : 2>(in, out, tw, n, Ns, ntl, pitch, sign);
        else stockham_pass<T, 2>(in, out, tw, n, Ns, ntl, pitch, sign);
        __syncthreads();
        C* tmp = in;
        in = out;
        out = tmp;
        Ns *= R;
    }
    return in;
}

// Visits the elements (t, k), t < ntl lines, k < n entries, of a block's lines with
// consecutive threads on consecutive addresses: consecutive lines t for a strided
// axis (s > 1), consecutive entries k for the contiguous one.  The counters advance
// by the block size without a division per element.
template <typename F>
__device__ inline void for_line_elems(int ntl, int n, bool strided, F&& f) {
    const int M = strided ? ntl : n, NMAJ = strided ? n : ntl;
    const int bd = blockDim.x;
    int mi = threadIdx.x % M, ma = threadIdx.x / M;
    const int dmi = bd % M, dma = bd / M;
    while (ma < NMAJ) {
        if (strided) f(mi, ma);
        else f(ma, mi);
        mi += dmi;
        ma += dma;
        if (mi >= M) {
            mi -= M;
            ++ma;
        }
    }
}

// Element offset of entry 0 of line L (element k at + k s): (L / s) n s + L mod s,
// for the block's lines, into lb[0..ntl) (one division pair per line)
__device__ inline void line_bases(int* lb, int L0, int ntl, int n, int s) {
    for (int t = threadIdx.x; t < ntl; t += blockDim.x) {
        const int L = L0 + t;
        lb[t] = (L / s) * n * s + (L % s);
    }
}

// ------------------------------------------------------------------ FFT along one axis
// Lines of the C-order array: line L = (o, i) with o < prod(N[<a]), i < s = prod(N[>a]);
// element k of the line at o*n*s + i + k*s.  A block transforms TL consecutive lines.
template <typename T, bool ODD>
__global__ void __launch_bounds__(256) k_fft_axis(const T* rsrc, typename V2<T>::t* X, T* rdst, int n, int s,
                           int nlines, int sign, FftPlan plan, int TL) {
    using C = typename V2<T>::t;
    extern __shared__ __align__(16) unsigned char smem_fft[];
    const int pitch = n + 1;
    C* A = reinterpret_cast<C*>(smem_fft);
    C* B = A + TL * pitch;
    C* tw = B + TL * pitch;
    int* lb = reinterpret_cast<int*>(tw + n);
    const int L0 = blockIdx.x * TL;
    const int ntl = min(TL, nlines - L0);
    fft_roots<T>(tw, n);
    line_bases(lb, L0, ntl, n, s);
    __syncthreads();
    for_line_elems(ntl, n, s > 1, [&](int t, int k) {
        const int addr = lb[t] + k * s;
        C v;
        if (rsrc) {
            v.x = rsrc[addr];
            v.y = (T)0;
        } else {
            v = X[addr];
        }
        A[t * pitch + k] = v;
    });
    __syncthreads();
    const C* in = fft_passes<T, ODD>(A, B, tw, n, ntl, pitch, sign, plan);
    for_line_elems(ntl, n, s > 1, [&](int t, int k) {
        const int addr = lb[t] + k * s;
        const C v = in[t * pitch + k];
        if (rdst) rdst[addr] = v.x;
        else X[addr] = v;
    });
}

// ------------------------------------------------------------------ DST-I along one axis
// The fast sine transform of eq. FST in O(N log N): X_k = sum_{j=1..N} x_j sin(pi j k /
// (N + 1)), k = 1..N, from the DFT of the odd extension of each line to length
// L = 2 (N + 1) (y_0 = y_{N+1} = 0, y_j = x_j, y_{L-j} = -x_j): DFT(y)_k = -2i X_k.
// Lines as in k_fft_axis (element j of line (o, i) at o*N*s + i + j*s); each
// block transforms TL lines in LDS with the same Stockham passes.
template <typename T, bool ODD>
__global__ void __launch_bounds__(256) k_dst1_axis(const T* src, T* dst, int n, int s, int nlines, FftPlan plan, int TL) {
    using C = typename V2<T>::t;
    extern __shared__ __align__(16) unsigned char smem_dst[];
    const int L = 2 * (n + 1), pitch = L + 1;
    C* A = reinterpret_cast<C*>(smem_dst);
    C* B = A + TL * pitch;
    C* tw = B + TL * pitch;
    int* lb = reinterpret_cast<int*>(tw + L);
    const int L0 = blockIdx.x * TL;
    const int ntl = min(TL, nlines - L0);
    fft_roots<T>(tw, L);
    line_bases(lb, L0, ntl, n, s);
    __syncthreads();
    for_line_elems(ntl, L, s > 1, [&](int t, int k) {
        // position k of the extension: x_k for 1 <= k <= n, -x_{L-k} for n+2 <= k < L, else 0
        const int j = (k >= 1 && k <= n) ? k : (k >= n + 2 ? L - k : 0);
        T v = (T)0;
        if (j) {
            const T x = src[lb[t] + (j - 1) * s];
            v = (k <= n) ? x : -x;
        }
        C c;
        c.x = v;
        c.y = (T)0;
        A[t * pitch + k] = c;
    });
    __syncthreads();
    const C* Y = fft_passes<T, ODD>(A, B, tw, L, ntl, pitch, -1, plan);
    for_line_elems(ntl, n, s > 1, [&](int t, int k) {
        dst[lb[t] + k * s] = (T)(-0.5) * Y[t * pitch + k + 1].y;
    });
}

// ------------------------------------------------------------------ predict planning
// Substep count, per-stage diffusion in index coordinates, grid move.  Thread 0
// takes the substep decision and the powers E^(2^j) of the stage propagator
// E = e^{-A dt}; the stage sets k = 0..cnt-1 are then built in parallel from
// E^k = prod over the set bits of k (powers of one matrix commute).

__device__ double lambda_bound_dev(const double* Dy, const double* rho, int n) {
    double s = 0.0;
    for (int a = 0; a < n; ++a)
        for (int b = 0; b < n; ++b) s += fabs(Dy[a * MS + b]) * rho[a] * rho[b];
    return 0.5 * s;
}

constexpr int PLAN_THREADS = 256;
constexpr int PLAN_POW = 14;   // 2 LMAX + 1 < 2^14

template <int NX>
__global__ void __launch_bounds__(PLAN_THREADS) k_plan(PredictArgs a, DevDesc* d, double* coef) {
    constexpr int n = NX;
    __shared__ double pw[PLAN_POW][MSQ];
    __shared__ int s_l;
    double Mi[MSQ];
    mat_copy(Mi, d->g.Mi);
    if (threadIdx.x == 0) {
        int l = a.lmin;
        if (a.integ == PMF_INT_RK4 && a.T > 0.0) {
            double lam = 0.0;
            const double* Es[3] = {nullptr, a.emh, a.emT};
            for (int q = 0; q < 3; ++q) {
                double E[MSQ], t1[MSQ], Dy[MSQ];
                if (q == 0) {
                    mat_copy(E, a.D);
                } else {
                    mat_mul(t1, Es[q], a.D, n);
                    mat_mul_bt(E, t1, Es[q], n);
                }
                sandwich_inv(Dy, Mi, E, n);
                const double lb = lambda_bound_dev(Dy, a.rho, n);
                lam = lb > lam ? lb : lam;
            }
            const double need = ceil(a.T * lam / RK4_STABLE_STEP);
            if (need > (double)l) l = need > (double)a.lmax ? a.lmax + 1 : (int)need;
        }
        if (a.integ == PMF_INT_FDM && a.T > 0.0) {
            // explicit step: h sum_a D_y,aa(t) <= 1 at t = 0, T/2, T
            double lam = 0.0;
            const double* Es[3] = {nullptr, a.emh, a.emT};
            for (int q = 0; q < 3; ++q) {
                double E[MSQ], t1[MSQ], Dy[MSQ];
                if (q == 0) {
                    mat_copy(E, a.D);
                } else {
                    mat_mul(t1, Es[q], a.D, n);
                    mat_mul_bt(E, t1, Es[q], n);
                }
                sandwich_inv(Dy, Mi, E, n);
                double tr = 0.0;
                for (int i = 0; i < n; ++i) tr += Dy[i * MS + i];
                lam = tr > lam ? tr : lam;
            }
            const double need = ceil(a.T * lam / FDM_STABLE_STEP);
            if (need > (double)l) l = need > (double)a.lmax ? a.lmax + 1 : (int)need;
        }
        if (l > a.lmax) {
            l = a.lmax;
            d->status |= PMF_E_INVALID;   // substep limit reached: result is not trustworthy
        }
        s_l = l;
        const double h = a.T / l;
        if (a.integ == PMF_INT_EXACT || a.integ == PMF_INT_SINE) {
            double Wy[MSQ];
            sandwich_inv(Wy, Mi, a.W, n);
            pack_sym(coef, Wy);
        } else {
            const double dt = (a.integ == PMF_INT_RK4) ? 0.5 * h : h;
            double E[MSQ];
            expm3(E, a.A, -dt, n);
            for (int i = 0; i < MSQ; ++i) pw[0][i] = E[i];
            for (int j = 1; j < PLAN_POW; ++j) {
                double sq[MSQ];
                mat_mul(sq, pw[j - 1], pw[j - 1], n);
                for (int i = 0; i < MSQ; ++i) pw[j][i] = sq[i];
            }
        }
        d->l = l;
        d->h = h;
        d->etr = a.etr;
    }
    __syncthreads();
    if (a.integ != PMF_INT_EXACT && a.integ != PMF_INT_SINE) {
        const int l = s_l;
        const int cnt = (a.integ == PMF_INT_RK4) ? 2 * l + 1 : l;
        for (int k = threadIdx.x; k < cnt; k += PLAN_THREADS) {
            double Ek[MSQ], nxt[MSQ], t1[MSQ], E[MSQ], Dy[MSQ];
            mat_eye(Ek, n);
            for (int j = 0; j < PLAN_POW; ++j)
                if ((k >> j) & 1) {
                    mat_mul(nxt, Ek, pw[j], n);
                    mat_copy(Ek, nxt);
                }
            mat_mul(t1, Ek, a.D, n);
            mat_mul_bt(E, t1, Ek, n);
            sandwich_inv(Dy, Mi, E, n);
            pack_sym(coef + PACK * k, Dy);
        }
    }
    if (threadIdx.x == 0) {
        // grid follows x' = A x over T
        double c2[MS], M2[MSQ];
        mat_zero(M2);
        mat_vec(c2, a.Phi, d->g.c, n);
        mat_mul(M2, a.Phi, d->g.M, n);
        for (int i = 0; i < n; ++i) d->g.c[i] = c2[i];
        mat_copy(d->g.M, M2);
        grid_finish(d->g, n);
        d->t += a.T;
    }
}

// ------------------------------------------------------------------ spectral gain

// kappa^T S kappa from the packed S (00, 11, 22, 33, 01, 02, 03, 12, 13, 23):
// squares with the second-derivative wavenumbers, cross terms with the first
template <typename T>
__device__ inline T sigma_of(const double* p, const T* k1, const T* k2) {
    const T sq = (T)p[0] * k2[0] + (T)p[1] * k2[1] + (T)p[2] * k2[2] + (T)p[3] * k2[3];
    const T cr = (T)p[4] * k1[0] * k1[1] + (T)p[5] * k1[0] * k1[2] + (T)p[6] * k1[0] * k1[3] +
                 (T)p[7] * k1[1] * k1[2] + (T)p[8] * k1[1] * k1[3] + (T)p[9] * k1[2] * k1[3];
    return sq + (T)2 * cr;
}

template <typename T>
__device__ T mode_gain(int integ, int l, T h, const double* coef, const T* k1, const T* k2) {
    if (integ == PMF_INT_EXACT) return exp_t((T)-0.5 * sigma_of<T>(coef, k1, k2));
    T g = (T)1;
    if (integ == PMF_INT_EULER) {
        for (int n = 0; n < l; ++n) g = g / ((T)1 + (T)0.5 * h * sigma_of<T>(coef + PACK * n, k1, k2));
        return g;
    }
    for (int n = 0; n < l; ++n) {
        const T la = (T)-0.5 * sigma_of<T>(coef + 2 * PACK * n, k1, k2);
        const T lb = (T)-0.5 * sigma_of<T>(coef + 2 * PACK * n + PACK, k1, k2);
        const T lc = (T)-0.5 * sigma_of<T>(coef + 2 * PACK * n + 2 * PACK, k1, k2);
        const T hh = (T)0.5 * h;
        const T y2 = (T)1 + hh * la;
        const T y3 = (T)1 + hh * lb * y2;
        const T y4 = (T)1 + h * lb * y3;
        g *= (T)1 + h / (T)6 * (la + (T)2 * lb * y2 + (T)2 * lb * y3 + lc * y4);
    }
    return g;
}

template <typename T>
__device__ inline void mode_kappa(int s, int n, T* k1, T* k2) {
    const int k = (s < n / 2) ? s : s - n;
    const T kap = (T)(2.0 * M_PI) * (T)k / (T)n;
    *k2 = kap * kap;
    *k1 = (2 * s == n) ? (T)0 : kap;
}

// Per-mode gain over the whole spectrum, one thread per mode (the RK4 and Euler gains
// cost a product over the substeps per mode: spread over as many threads as modes)
template <typename T>
__global__ void k_gain(KModel m, const DevDesc* d, const double* coef, typename V2<T>::t* X) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= m.ntot) return;
    T k1[MS] = {0, 0, 0, 0}, k2[MS] = {0, 0, 0, 0};
    int rem = e;
    for (int a = m.nx - 1; a >= 0; --a) {
        const int s = rem % m.N[a];
        rem /= m.N[a];
        mode_kappa<T>(s, m.N[a], &k1[a], &k2[a]);
    }
    const T g = mode_gain<T>(m.integ, d->l, (T)d->h, coef, k1, k2) * (T)(d->etr / (double)m.ntot);
    typename V2<T>::t v = X[e];
    v.x *= g;
    v.y *= g;
    X[e] = v;
}

// Axis 0 of a Fourier predict in one launch: forward transform of each axis-0 line,
// the per-mode gain, inverse transform.  Axis 0 is the last axis of the
// forward transform and the first of the inverse one, so the three steps need no
// other line in between: one pass over the spectrum instead of three.  With nx = 1
// it is the whole predict (real density in, real density out, in place).
// LDS: A, B (TL lines of n + 1), the n roots, per line the wavenumbers k1, k2 of
// axes 1..nx-1, the TL line offsets.
template <typename T, bool ODD>
__global__ void __launch_bounds__(256)
k_fft_gain_axis0(KModel m, const DevDesc* d, const double* coef, const T* rsrc, typename V2<T>::t* X, T* rdst,
                 FftPlan plan, int TL) {
    using C = typename V2<T>::t;
    extern __shared__ __align__(16) unsigned char smem_fg[];
    const int n = m.N[0], s = m.ntot / n, nlines = s;
    const int pitch = n + 1;
    C* A = reinterpret_cast<C*>(smem_fg);
    C* B = A + TL * pitch;
    C* tw = B + TL * pitch;
    T* lk = reinterpret_cast<T*>(tw + n);   // line t: k1 of axes 1..3 at 6 t, k2 at 6 t + 3
    int* lb = reinterpret_cast<int*>(lk + 6 * TL);
    const int L0 = blockIdx.x * TL;
    const int ntl = min(TL, nlines - L0);
    fft_roots<T>(tw, n);
    line_bases(lb, L0, ntl, n, s);
    for (int t = threadIdx.x; t < ntl; t += blockDim.x) {
        int rem = L0 + t;
        for (int a = m.nx - 1; a >= 1; --a) {
            const int sa = rem % m.N[a];
            rem /= m.N[a];
            mode_kappa<T>(sa, m.N[a], &lk[6 * t + a - 1], &lk[6 * t + 3 + a - 1]);
        }
    }
    __syncthreads();
    for_line_elems(ntl, n, s > 1, [&](int t, int k) {
        const int addr = lb[t] + k * s;
        C v;
        if (rsrc) {
            v.x = rsrc[addr];
            v.y = (T)0;
        } else {
            v = X[addr];
        }
        A[t * pitch + k] = v;
    });
    __syncthreads();
    C* F = fft_passes<T, ODD>(A, B, tw, n, ntl, pitch, -1, plan);
    C* G = (F == A) ? B : A;
    const T scale = (T)(d->etr / (double)m.ntot);
    const int l = d->l;
    const T h = (T)d->h;
    for_line_elems(ntl, n, false, [&](int t, int k) {
        T k1[MS] = {0, 0, 0, 0}, k2[MS] = {0, 0, 0, 0};
        mode_kappa<T>(k, n, &k1[0], &k2[0]);
        for (int a = 1; a < m.nx; ++a) {
            k1[a] = lk[6 * t + a - 1];
            k2[a] = lk[6 * t + 3 + a - 1];
        }
        const T g = mode_gain<T>(m.integ, l, h, coef, k1, k2) * scale;
        C v = F[t * pitch + k];
        v.x *= g;
        v.y *= g;
        F[t * pitch + k] = v;
    });
    __syncthreads();
    const C* R = fft_passes<T, ODD>(F, G, tw, n, ntl, pitch, +1, plan);
    for_line_elems(ntl, n, s > 1, [&](int t, int k) {
        const int addr = lb[t] + k * s;
        const C v = R[t * pitch + k];
        if (rdst) rdst[addr] = v.x;
        else X[addr] = v;
    });
}

// ------------------------------------------------------------------ grid coordinates

// axis tables: per axis a at tab + a*TAB_STRIDE: u[N] (computational coordinate),
// qw[N] (quadrature weight in u), v[N+2] (full CGL nodes), beta[N+2] (barycentric)
__device__ inline void node_coords(const KModel& m, const double* tab, int j, double* u, int* idx) {
    int rem = j;
    for (int a = m.nx - 1; a >= 0; --a) {
        const int s = rem % m.N[a];
        rem /= m.N[a];
        idx[a] = s;
        u[a] = tab[a * TAB_STRIDE + s];
    }
}

// the same for a compile-time dimension (the axis loop unrolled)
template <int NX>
__device__ inline void node_coords_n(const KModel& m, const double* tab, int j, double* u, int* idx) {
    int rem = j;
#pragma unroll
    for (int a = NX - 1; a >= 0; --a) {
        const int s = rem % m.N[a];
        rem /= m.N[a];
        idx[a] = s;
        u[a] = tab[a * TAB_STRIDE + s];
    }
}

__device__ inline double node_qw(const KModel& m, const double* tab, const int* idx) {
    if (m.grid == PMF_GRID_FOURIER) return 1.0;
    double q = 1.0;
    for (int a = 0; a < m.nx; ++a) q *= tab[a * TAB_STRIDE + TAB_QW + idx[a]];
    return q;
}

__device__ inline bool node_on_boundary(const KModel& m, const int* idx) {
    for (int a = 0; a < m.nx; ++a)
        if (idx[a] == 0 || idx[a] == m.N[a] - 1) return true;
    return false;
}

__device__ inline void to_phys(const Grid& g, int nx, const double* u, double* x) {
    for (int i = 0; i < nx; ++i) {
        double s = g.c[i];
        for (int k = 0; k < nx; ++k) s += g.M[i * MS + k] * u[k];
        x[i] = s;
    }
}

// log p_v(z - h(x)) for a Gaussian-mixture v
__device__ double loglik_at(const KModel& m, const double* x, const double* z) {
    double hx[3] = {0, 0, 0};
    if (m.meas == PMF_H_LINEAR) {
        for (int i = 0; i < m.nz; ++i) {
            double s = 0.0;
            for (int k = 0; k < m.nx; ++k) s += m.H[i * MS + k] * x[k];
            hx[i] = s;
        }
    } else if (m.meas == PMF_H_CUBIC1) {
        hx[0] = m.hp[0] * x[0] + m.hp[1] * x[0] * x[0] * x[0];
    } else if (m.meas == PMF_H_TERRAIN) {
        double s = 0.0;
        for (int c = 0; c < m.nterr; ++c) {
            double ph = m.terr[c][1];
            for (int k = 0; k < m.nx; ++k) ph += m.terr[c][2 + k] * x[k];
            s += m.terr[c][0] * cos(ph);
        }
        hx[0] = s;
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
            for (int k = 0; k < m.nz; ++k) q += r[i] * m.nRi[g][i * MS + k] * r[k];
        terms[g] = m.lw[g] - 0.5 * q;
        best = terms[g] > best ? terms[g] : best;
    }
    if (m.ncomp == 1) return terms[0];
    double acc = 0.0;
    for (int g = 0; g < m.ncomp; ++g) acc += exp(terms[g] - best);
    return best + log(acc);
}

// per-thread FP64 sums of a weighted node: S0, S1[a] (u_a), S2[pk(a,b)] (u_a u_b),
// boundary mass
constexpr int NACC = 16;
__device__ inline void acc_point(double* acc, double w, const double* u, bool boundary) {
    acc[0] += w;
    for (int a = 0; a < MS; ++a) acc[1 + a] += w * u[a];
    for (int a = 0; a < MS; ++a)
        for (int b = a; b < MS; ++b) acc[5 + pk(a, b)] += w * u[a] * u[b];
    if (boundary) acc[NACC - 1] += w;
}

// the same sums over the first NX coordinates only (the others stay zero)
template <int NX>
__device__ inline void acc_point_n(double* acc, double w, const double* u, bool boundary) {
    acc[0] += w;
#pragma unroll
    for (int a = 0; a < NX; ++a) {
        const double wu = w * u[a];
        acc[1 + a] += wu;
#pragma unroll
        for (int b = a; b < NX; ++b) acc[5 + pk(a, b)] += wu * u[b];
    }
    if (boundary) acc[NACC - 1] += w;
}

// Fixed-order block reduction of NV doubles per thread (RED_THREADS threads, all
// of which must call it): a butterfly over the 64 lanes of each wave (partner
// lanes add the same two values, so every lane of a wave ends with the same sum),
// then every thread adds the per-wave sums in wave order.  No barrier inside a
// wave's tree; two block barriers in all.  Every thread returns the block sums.
template <int NV>
__device__ void block_sum(double (&v)[NV], double* sh) {
    constexpr int NW = RED_THREADS / 64;
#pragma unroll
    for (int q = 0; q < NV; ++q)
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) v[q] += __shfl_xor(v[q], o, 64);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0)
        for (int q = 0; q < NV; ++q) sh[q * NW + w] = v[q];
    __syncthreads();
    for (int q = 0; q < NV; ++q) {
        double t = sh[q * NW];
        for (int k = 1; k < NW; ++k) t += sh[q * NW + k];
        v[q] = t;
    }
    __syncthreads();
}

__device__ double block_max(double v, double* sh) {
    constexpr int NW = RED_THREADS / 64;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    double t = sh[0];
    for (int k = 1; k < NW; ++k) t = fmax(t, sh[k]);
    __syncthreads();
    return t;
}

// ------------------------------------------------------------------ likelihood + sums
constexpr int LIKE_CACHE = 1024;   // log-likelihoods kept per block between the two passes
// mode 0: sums of the density only; mode 1: P_out = P * exp(loglik - s_b) and its sums.
// Partial b: {s_b, S0, S1[4], S2[10] (packed as pk), Sboundary}, block-relative,
// stored by column: entry q at part[q nb + b].
template <typename T, int NX>
__global__ void __launch_bounds__(RED_THREADS)
k_like_pass(KModel m, const DevDesc* d, const double* tab, ZArg z, const T* P, T* Pout,
            double* part, int chunk, int mode) {
    __shared__ double sh[NACC * RED_THREADS];
    // the block's log-likelihoods from the max pass, reused by the multiply pass
    // (each thread reads back its own entries; blocks of more points recompute)
    __shared__ double Lsh[LIKE_CACHE];
    const int b = blockIdx.x;
    const int lo = b * chunk;
    const int hi = min(m.ntot, lo + chunk);
    const bool cached = chunk <= LIKE_CACHE;
    const Grid& g = d->g;
    double sb = 0.0;
    if (mode == 1) {
        double mx = -INFINITY;
        for (int j = lo + threadIdx.x; j < hi; j += RED_THREADS) {
            double u[MS] = {0, 0, 0, 0}, x[MS];
            int idx[MS];
            node_coords_n<NX>(m, tab, j, u, idx);
            to_phys(g, NX, u, x);
            const double L = loglik_at(m, x, z.v);
            if (cached) Lsh[j - lo] = L;
            mx = fmax(mx, L);
        }
        sb = block_max(mx, sh);
    }
    double acc[NACC];
    for (int q = 0; q < NACC; ++q) acc[q] = 0.0;
    for (int j = lo + threadIdx.x; j < hi; j += RED_THREADS) {
        double u[MS] = {0, 0, 0, 0};
        int idx[MS] = {0, 0, 0, 0};
        node_coords_n<NX>(m, tab, j, u, idx);
        T v = P[j];
        if (mode == 1) {
            double L;
            if (cached) {
                L = Lsh[j - lo];
            } else {
                double x[MS];
                to_phys(g, NX, u, x);
                L = loglik_at(m, x, z.v);
            }
            v = v * exp_t((T)(L - sb));
            Pout[j] = v;
        }
        const double w = node_qw(m, tab, idx) * (double)v;
        acc_point_n<NX>(acc, w, u, node_on_boundary(m, idx));
    }
    block_sum<NACC>(acc, sh);
    if (threadIdx.x == 0) {
        // partials stored by column: entry q of block b at q nb + b (nb = gridDim.x)
        part[b] = sb;
        for (int q = 0; q < NACC; ++q) part[(size_t)(1 + q) * gridDim.x + b] = acc[q];
    }
}

// Combine the per-block partials (all RED_THREADS threads of one block, fixed
// tree order): S0..Sb relative to the global shift, in every thread.  Partials
// are stored by column (entry q of block b at q nb + b), so consecutive threads
// read consecutive doubles.
__device__ void combine_partials(const double* part, int nb, double* s_out, double* S, double* sh) {
    double mx = -INFINITY;
    for (int b = threadIdx.x; b < nb; b += RED_THREADS) mx = fmax(mx, part[b]);
    const double s = block_max(mx, sh);
    double acc[NACC];
    for (int q = 0; q < NACC; ++q) acc[q] = 0.0;
    for (int b = threadIdx.x; b < nb; b += RED_THREADS) {
        const double f = (s == -INFINITY) ? 0.0 : exp(part[b] - s);
#pragma unroll
        for (int q = 0; q < NACC; ++q) acc[q] += f * part[(size_t)(1 + q) * nb + b];
    }
    block_sum<NACC>(acc, sh);
    for (int q = 0; q < NACC; ++q) S[q] = acc[q];
    *s_out = s;
}

// mean and covariance from sums in computational coordinates u (x = c + M u);
// NX at compile time, so the small matrices live in registers
template <int NX>
__device__ __forceinline__ void moments_from_sums(const Grid& g, const double* S, double* mean, double* cov) {
    const double S0 = S[0];
    double ub[NX], Cu[NX][NX];
#pragma unroll
    for (int a = 0; a < NX; ++a) ub[a] = S[1 + a] / S0;
#pragma unroll
    for (int a = 0; a < NX; ++a)
#pragma unroll
        for (int b = 0; b < NX; ++b) Cu[a][b] = S[5 + pk(a, b)] / S0 - ub[a] * ub[b];
#pragma unroll
    for (int a = 0; a < NX; ++a) {
        double mu = 0.0;
#pragma unroll
        for (int k = 0; k < NX; ++k) mu += g.M[a * MS + k] * ub[k];
        mean[a] = g.c[a] + mu;
    }
    // C = M Cu M^T
    double t1[NX][NX], C[NX][NX];
#pragma unroll
    for (int a = 0; a < NX; ++a)
#pragma unroll
        for (int b = 0; b < NX; ++b) {
            double t = 0.0;
#pragma unroll
            for (int k = 0; k < NX; ++k) t += g.M[a * MS + k] * Cu[k][b];
            t1[a][b] = t;
        }
#pragma unroll
    for (int a = 0; a < NX; ++a)
#pragma unroll
        for (int b = 0; b < NX; ++b) {
            double t = 0.0;
#pragma unroll
            for (int k = 0; k < NX; ++k) t += t1[a][k] * g.M[b * MS + k];
            C[a][b] = t;
        }
#pragma unroll
    for (int a = 0; a < NX; ++a)
#pragma unroll
        for (int b = 0; b < NX; ++b) cov[a * MS + b] = 0.5 * (C[a][b] + C[b][a]);
}

// Mi = M^-1 and vol = |det M| as grid_finish computes them (the same cofactor
// arithmetic), with the 4 x 4 minors' indices fixed at compile time
template <int NX>
__device__ __forceinline__ void grid_finish_c(Grid& g) {
    if constexpr (NX < 4) {
        grid_finish(g, NX);
    } else {
        const double* a = g.M;
        double* r = g.Mi;
        const double dt = mat_det(a, 4);
        mat_zero(r);
        if (dt != 0.0) {
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    int rr[3], cc[3], p = 0, q = 0;
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        if (k != i) rr[p++] = k;
                        if (k != j) cc[q++] = k;
                    }
                    const double mn = det3_at(a, rr[0], rr[1], rr[2], cc[0], cc[1], cc[2]);
                    r[j * MS + i] = (((i + j) & 1) ? -mn : mn) / dt;
                }
        }
        g.vol = fabs(dt);
    }
}

template <int NX>
__device__ __forceinline__ bool design_grid_dev(const KModel& m, const double* mean, const double* cov, Grid& gn) {
    mat_zero(gn.M);
#pragma unroll
    for (int a = 0; a < NX; ++a) {
        const double v = cov[a * MS + a] + m.Wnom[a * MS + a];
        if (!(v > 0.0) || !isfinite(v)) return false;
        const double h = m.span * sqrt(v);
        gn.M[a * MS + a] = (m.grid == PMF_GRID_FOURIER) ? 2.0 * h / m.N[a] : h;
        gn.c[a] = mean[a];
    }
    grid_finish_c<NX>(gn);
    return true;
}

// After k_like_pass(mode 1): normaliser, log-likelihood, moments, block factors,
// new grid.  On failure: ok = 0 and the DEGENERATE bit.  One block.
template <int NX>
__global__ void __launch_bounds__(RED_THREADS)
k_update_finalize(KModel m, DevDesc* d, const double* part, int nb, double* bfac) {
    __shared__ double sh[NACC * RED_THREADS];
    double s, S[NACC];
    combine_partials(part, nb, &s, S, sh);
    const double mass = d->g.vol * S[0];
    const bool good = isfinite(s) && isfinite(mass) && mass > 0.0;
    if (good)
        for (int b = threadIdx.x; b < nb; b += RED_THREADS) bfac[b] = exp(part[b] - s) / mass;
    if (threadIdx.x != 0) return;
    d->ok = 1;
    if (!good) {
        d->ok = 0;
    } else {
        d->s = s;
        d->mass = mass;
        d->loglik = s + log(mass);
        moments_from_sums<NX>(d->g, S, d->mean, d->cov);
        d->bfrac = S[NACC - 1] / S[0];
        if (d->bfrac > BOUNDARY_TOL) d->status |= ST_BOUNDARY;
        if (!design_grid_dev<NX>(m, d->mean, d->cov, d->gn)) d->ok = 0;
        // separable spectral interpolation when the old grid is axis aligned
        // (the new one always is); otherwise cubic Lagrange
        bool aligned = true;
#pragma unroll
        for (int a = 0; a < NX; ++a)
#pragma unroll
            for (int b = 0; b < NX; ++b)
                if (a != b && d->g.M[a * MS + b] != 0.0) aligned = false;
        d->sep = (m.interp == PMF_INTERP_AUTO && aligned) ? 1 : 0;
    }
    if (!d->ok) {
        d->status |= ST_DEGENERATE;
        d->loglik = NAN;
    }
}

// After k_like_pass(mode 0): mass, moments and 1/mass (in bfac[0..nb)).  One block.
template <int NX>
__global__ void __launch_bounds__(RED_THREADS)
k_sums_finalize(KModel m, DevDesc* d, const double* part, int nb, double* bfac) {
    __shared__ double sh[NACC * RED_THREADS];
    double s, S[NACC];
    combine_partials(part, nb, &s, S, sh);
    const double mass = d->g.vol * S[0];
    for (int b = threadIdx.x; b < nb; b += RED_THREADS) bfac[b] = 1.0 / mass;
    if (threadIdx.x != 0) return;
    d->mass = mass;
    moments_from_sums<NX>(d->g, S, d->mean, d->cov);
}

template <typename T>
__global__ void k_scale_blocks(T* P, int ntot, int chunk, const double* bfac) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= ntot) return;
    P[j] = (T)((double)P[j] * bfac[j / chunk]);
}

// ------------------------------------------------------------------ re-interpolation

// Separable spectral weights, one matrix per axis at W + a*wstride (row j' = new node):
// Fourier: periodic interpolation kernel sin(pi d) / (N tan(pi d / N)) of the
// trigonometric interpolant, zero when the new node is outside [0, N-1] in old
// index units; Chebyshev: barycentric form of the polynomial through the N+2
// Chebyshev-Gauss-Lobatto values (zero at +-1), zero outside [-1, 1].
__global__ void k_interp_weights(KModel m, const DevDesc* d, const double* tab, double* W) {
    const int a = blockIdx.y;
    const int n = m.N[a];
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (!d->sep || a >= m.nx || e >= n * n) return;
    const int jp = e / n, j = e - jp * n;
    const Grid& go = d->g;
    const Grid& gn = d->gn;
    const double xn = gn.c[a] + gn.M[a * MS + a] * tab[a * TAB_STRIDE + jp];
    double w = 0.0;
    if (m.grid == PMF_GRID_FOURIER) {
        const double nu = (xn - go.c[a]) * go.Mi[a * MS + a] + (double)(n / 2);
        if (nu >= 0.0 && nu <= (double)(n - 1)) {
            const double dd = nu - (double)j;
            if (dd == 0.0) {
                w = 1.0;
            } else {
                w = sinpi(dd) / ((double)n * tan(M_PI * dd / (double)n));
            }
        }
    } else {
        const double u = (xn - go.c[a]) * go.Mi[a * MS + a];
        if (u >= -1.0 && u <= 1.0) {
            const double* v = tab + a * TAB_STRIDE + TAB_V;
            const double* beta = tab + a * TAB_STRIDE + TAB_BETA;
            int hit = -1;
            double den = 0.0;
            for (int k = 0; k < n + 2; ++k) {
                const double dk = u - v[k];
                if (dk == 0.0) {
                    hit = k;
                    break;
                }
                den += beta[k] / dk;
            }
            if (hit >= 0) {
                w = (hit == j + 1) ? 1.0 : 0.0;
            } else {
                w = (beta[j + 1] / (u - v[j + 1])) / den;
            }
        }
    }
    W[(size_t)a * m.wstride + e] = w;
}

// out = (matrix W_a applied along axis a of in).  With want_sums the block also
// produces the FP64 sums of the result (new grid, block-ordered partials).
template <typename T>
__global__ void __launch_bounds__(RED_THREADS)
k_interp_axis(KModel m, const DevDesc* d, const double* tab, const double* Wall, int a,
              const T* in, T* out, double* part, int chunk, int want_sums) {
    __shared__ double sh[NACC * RED_THREADS];
    if (!d->sep) return;
    const int n = m.N[a];
    int s = 1;
    for (int b = a + 1; b < m.nx; ++b) s *= m.N[b];
    const double* W = Wall + (size_t)a * m.wstride;
    const int lo = blockIdx.x * chunk;
    const int hi = min(m.ntot, lo + chunk);
    double acc[NACC];
    for (int q = 0; q < NACC; ++q) acc[q] = 0.0;
    for (int j = lo + threadIdx.x; j < hi; j += RED_THREADS) {
        const int i = j % s;
        const int jp = (j / s) % n;
        const int o = j / (s * n);
        const T* src = in + (size_t)o * n * s + i;
        double v = 0.0;
        for (int k = 0; k < n; ++k) v += W[jp * n + k] * (double)src[(size_t)k * s];
        out[j] = (T)v;
        if (want_sums) {
            double u[MS] = {0, 0, 0, 0};
            int idx[MS] = {0, 0, 0, 0};
            node_coords(m, tab, j, u, idx);
            const double w = node_qw(m, tab, idx) * (double)(T)v;
            acc_point(acc, w, u, false);
        }
    }
    if (want_sums) {
        block_sum<NACC>(acc, sh);
        if (threadIdx.x == 0) {
            part[blockIdx.x] = 0.0;
            for (int q = 0; q < NACC; ++q) part[(size_t)(1 + q) * gridDim.x + blockIdx.x] = acc[q];
        }
    }
}

// cubic Lagrange weights through abscissae x0..x3 at t
__device__ inline void lagrange4(double t, const double* x, double* w) {
    for (int k = 0; k < 4; ++k) {
        double p = 1.0;
        for (int i = 0; i < 4; ++i)
            if (i != k) p *= (t - x[i]) / (x[k] - x[i]);
        w[k] = p;
    }
}

// Tensor cubic Lagrange interpolation in the old grid's computational coordinates,
// specialised per dimension NX (every axis loop unrolled, taps in registers).
template <typename T, int NX>
__global__ void __launch_bounds__(RED_THREADS)
k_interp_lagrange(KModel m, const DevDesc* d, const double* tab, const T* in, T* out,
                  double* part, int chunk) {
    __shared__ double sh[NACC * RED_THREADS];
    if (d->sep) return;
    const Grid& go = d->g;
    const Grid& gn = d->gn;
    const int lo = blockIdx.x * chunk;
    const int hi = min(m.ntot, lo + chunk);
    const bool fourier = m.grid == PMF_GRID_FOURIER;
    double acc[NACC];
    for (int q = 0; q < NACC; ++q) acc[q] = 0.0;
    for (int j = lo + threadIdx.x; j < hi; j += RED_THREADS) {
        double u[MS] = {0, 0, 0, 0}, x[MS], r[MS], nu[MS] = {0, 0, 0, 0};
        int idx[MS] = {0, 0, 0, 0};
        node_coords_n<NX>(m, tab, j, u, idx);
        to_phys(gn, NX, u, x);
#pragma unroll
        for (int a = 0; a < NX; ++a) r[a] = x[a] - go.c[a];
        mat_vec(nu, go.Mi, r, NX);
        bool inside = true;
        int first[NX];       // array index of tap 0 along each axis (taps first .. first + 3)
        double tw[NX][4];    // weights, zero for taps outside the array
#pragma unroll
        for (int a = 0; a < NX; ++a) {
            const int n = m.N[a];
            if (fourier) {
                const double q = nu[a] + (double)(n / 2);
                inside = inside && q >= 0.0 && q <= (double)(n - 1);
                const int i0 = (int)floor(fmin(fmax(q, 0.0), (double)(n - 1)));
                // the cubic through nodes i0 - 1 .. i0 + 2 (unit spacing) at t = q - i0
                const double t = q - (double)i0, tp = t + 1.0, tm = t - 1.0, tm2 = t - 2.0;
                tw[a][0] = -t * tm * tm2 / 6.0;
                tw[a][1] = tp * tm * tm2 / 2.0;
                tw[a][2] = -tp * t * tm2 / 2.0;
                tw[a][3] = tp * t * tm / 6.0;
                first[a] = i0 - 1;
            } else {
                const double q = nu[a];
                inside = inside && q >= -1.0 && q <= 1.0;
                const double qc = fmin(fmax(q, -1.0), 1.0);
                const int nn = n + 1;
                int k0 = (int)floor((double)nn * acos(-qc) / M_PI);
                k0 = k0 < 0 ? 0 : (k0 > nn - 1 ? nn - 1 : k0);
                int ks = k0 - 1;
                ks = ks < 0 ? 0 : (ks > nn - 3 ? nn - 3 : ks);
                const double* v = tab + a * TAB_STRIDE + TAB_V;
                lagrange4(qc, v + ks, tw[a]);
                // node kk of the n + 2 Gauss-Lobatto nodes is array entry kk - 1
                // (kk = 0 and n + 1 are the zero end nodes)
                first[a] = ks - 1;
            }
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int ii = first[a] + k;
                if (ii < 0 || ii > n - 1) tw[a][k] = 0.0;
            }
        }
        double val = 0.0;
        if (inside) {
            if constexpr (NX == 1) {
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const int ii = min(max(first[0] + k, 0), m.N[0] - 1);
                    val += tw[0][k] * (double)in[ii];
                }
            } else {
                // Along the last (contiguous) axis the four taps are read as four
                // consecutive entries from b = clamp(first, 0, n - 4), the weights
                // moved to match (taps outside the array have weight zero, and the
                // entries that replace them get weight zero); along the other axes
                // each tap is a 32-bit element offset (index times stride).
                constexpr int L = NX - 1;
                const int nl = m.N[L];
                const int b = min(max(first[L], 0), nl - 4), sh3 = first[L] - b;   // -1 .. 2
                double wl[4];
#pragma unroll
                for (int p = 0; p < 4; ++p) {
                    const int k = p - sh3;
                    wl[p] = (k == 0) ? tw[L][0] : (k == 1) ? tw[L][1] : (k == 2) ? tw[L][2] : (k == 3) ? tw[L][3] : 0.0;
                }
                int off[NX - 1][4];
                int stride = nl;
#pragma unroll
                for (int a = NX - 2; a >= 0; --a) {
#pragma unroll
                    for (int k = 0; k < 4; ++k) off[a][k] = min(max(first[a] + k, 0), m.N[a] - 1) * stride;
                    stride *= m.N[a];
                }
                const T* base = in + b;
                auto row4 = [&](int o) -> double {
                    const T* r = base + o;
                    return wl[0] * (double)r[0] + wl[1] * (double)r[1] + wl[2] * (double)r[2] + wl[3] * (double)r[3];
                };
                if constexpr (NX == 2) {
#pragma unroll
                    for (int k0 = 0; k0 < 4; ++k0) val += tw[0][k0] * row4(off[0][k0]);
                } else if constexpr (NX == 3) {
#pragma unroll
                    for (int k0 = 0; k0 < 4; ++k0) {
                        double ps = 0.0;
#pragma unroll
                        for (int k1 = 0; k1 < 4; ++k1) ps += tw[1][k1] * row4(off[0][k0] + off[1][k1]);
                        val += tw[0][k0] * ps;
                    }
                } else {
#pragma unroll
                    for (int k0 = 0; k0 < 4; ++k0) {
                        double s1 = 0.0;
#pragma unroll
                        for (int k1 = 0; k1 < 4; ++k1) {
                            const int o01 = off[0][k0] + off[1][k1];
                            double s2 = 0.0;
#pragma unroll
                            for (int k2 = 0; k2 < 4; ++k2) s2 += tw[2][k2] * row4(o01 + off[2][k2]);
                            s1 += tw[1][k1] * s2;
                        }
                        val += tw[0][k0] * s1;
                    }
                }
            }
        }
        const T vt = (T)val;
        out[j] = vt;
        const double w = node_qw(m, tab, idx) * (double)vt;
        acc_point_n<NX>(acc, w, u, false);
    }
    block_sum<NACC>(acc, sh);
    if (threadIdx.x == 0) {
        part[blockIdx.x] = 0.0;
        for (int q = 0; q < NACC; ++q) part[(size_t)(1 + q) * gridDim.x + blockIdx.x] = acc[q];
    }
}

// New grid's mass -> 1/mass, commit the grid.  A zero / non-finite mass rejects
// the update (state unchanged).  One block.
__global__ void __launch_bounds__(RED_THREADS)
k_interp_finalize(KModel m, DevDesc* d, const double* part, int nb) {
    __shared__ double sh[NACC * RED_THREADS];
    if (!d->ok) return;   // uniform over the block
    double s, S[NACC];
    combine_partials(part, nb, &s, S, sh);
    if (threadIdx.x != 0) return;
    const double mass2 = d->gn.vol * S[0];
    if (!isfinite(mass2) || !(mass2 > 0.0)) {
        d->ok = 0;
        d->status |= ST_DEGENERATE;
        d->loglik = NAN;
        return;
    }
    d->mass2 = mass2;
    d->g = d->gn;
}

// final density: out *= 1/mass2 when accepted, else out = old (state unchanged)
template <typename T>
__global__ void k_final_scale(T* out, const T* old, int ntot, const DevDesc* d) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= ntot) return;
    if (d->ok) out[j] = (T)((double)out[j] / d->mass2);
    else out[j] = old[j];
}

// ------------------------------------------------------------------ prior

__global__ void k_prior(KModel m, KPrior pr, const DevDesc* d, const double* tab, void* Pv, int prec) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= m.ntot) return;
    double u[MS] = {0, 0, 0, 0}, x[MS];
    int idx[MS];
    node_coords(m, tab, j, u, idx);
    to_phys(d->g, m.nx, u, x);
    double best = -INFINITY, terms[MAXMIX];
    for (int g = 0; g < pr.ncomp; ++g) {
        double r[MS];
        for (int i = 0; i < m.nx; ++i) r[i] = x[i] - pr.mean[g][i];
        double q = 0.0;
        for (int i = 0; i < m.nx; ++i)
            for (int k = 0; k < m.nx; ++k) q += r[i] * pr.Ci[g][i * MS + k] * r[k];
        terms[g] = pr.lw[g] - 0.5 * q;
        best = terms[g] > best ? terms[g] : best;
    }
    double acc = 0.0;
    for (int g = 0; g < pr.ncomp; ++g) acc += exp(terms[g] - best);
    const double p = exp(best) * acc;
    if (prec == PMF_FP64) static_cast<double*>(Pv)[j] = p;
    else static_cast<float*>(Pv)[j] = (float)p;
}

// ------------------------------------------------------------------ Chebyshev RK4 pieces

// out = beta*out + alpha*coef[cidx] * (Mat applied along axis a of in); Mat is n x n.
template <typename T>
__global__ void k_axis_mm(const T* Mat, const T* in, T* out, int n, int s, int ntot,
                          const double* coef, int cidx, double alpha, int accumulate) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= ntot) return;
    const int i = j % s;
    const int r = (j / s) % n;
    const int o = j / (s * n);
    const T* src = in + (size_t)o * n * s + i;
    T v = (T)0;
    for (int k = 0; k < n; ++k) v += Mat[r * n + k] * src[(size_t)k * s];
    const T f = (T)(alpha * (cidx >= 0 ? coef[cidx] : 1.0));
    out[j] = accumulate ? out[j] + f * v : f * v;
}

// RK4 stage bookkeeping.  stage 1..4 with kf = f(y):
//  1: acc = kf,     y = q + h/2 kf
//  2: acc += 2 kf,  y = q + h/2 kf
//  3: acc += 2 kf,  y = q + h kf
//  4: q += h/6 (acc + kf)
template <typename T>
__global__ void k_rk4_stage(T* q, T* y, const T* kf, T* acc, int ntot, const DevDesc* d, int stage) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= ntot) return;
    const T h = (T)d->h;
    const T k = kf[j];
    if (stage == 1) {
        acc[j] = k;
        y[j] = q[j] + (T)0.5 * h * k;
    } else if (stage == 2) {
        acc[j] += (T)2 * k;
        y[j] = q[j] + (T)0.5 * h * k;
    } else if (stage == 3) {
        acc[j] += (T)2 * k;
        y[j] = q[j] + h * k;
    } else {
        q[j] += h / (T)6 * (acc[j] + k);
    }
}

template <typename T>
__global__ void k_scale_by(T* q, int ntot, const DevDesc* d) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= ntot) return;
    q[j] = (T)((double)q[j] * d->etr);
}

template <typename T>
__global__ void k_copy(T* dst, const T* src, int ntot) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < ntot) dst[j] = src[j];
}

// ------------------------------------------------------------------ host launchers

static inline int cdiv(int a, int b) { return (a + b - 1) / b; }

// Lines per block of the LDS transforms along one axis: enough blocks for about
// two per compute unit (one transform of a small filter is otherwise a handful of
// blocks, each running all its lines' passes in turn), at most about 2048 points
// per block, and both line buffers plus the roots of unity within 64 KiB.
static inline int lines_per_block(int len, int nlines, size_t csize) {
    // A and B (TL lines of len + 1 entries each), the len roots and TL line offsets
    const int cap = (int)((65536 - (size_t)len * csize) / (2 * (size_t)(len + 1) * csize + sizeof(int)));
    int TL = std::min(2048 / len, std::max(1, nlines / 512));
    if (TL > cap) TL = cap;
    if (TL < 1) TL = 1;
    if (TL > nlines) TL = nlines;
    return TL;
}

// whether an FFT plan holds a radix-7, 11, 13 or 17 pass
static inline bool plan_has_odd(const FftPlan& p) {
    for (int i = 0; i < p.np; ++i)
        if (p.r[i] == 7 || p.r[i] == 11 || p.r[i] == 13 || p.r[i] == 17) return true;
    return false;
}

// threads per block for `points` points in LDS: about two points per thread, whole
// waves, 64..256
static inline int block_threads(int points) {
    const int t = (points / 2 + 63) / 64 * 64;
    return std::min(256, std::max(64, t));
}

template <typename T>
hipError_t launch_fft_axis(const KModel& m, int a, const T* rsrc, void* X, T* rdst, int sign,
                           hipStream_t st) {
    const int n = m.N[a];
    int s = 1;
    for (int b = a + 1; b < m.nx; ++b) s *= m.N[b];
    const int nlines = m.ntot / n;
    const int TL = lines_per_block(n, nlines, sizeof(typename V2<T>::t));
    const size_t lds = (2 * (size_t)TL * (n + 1) + n) * sizeof(typename V2<T>::t) + (size_t)TL * sizeof(int);
    const FftPlan plan = make_plan(n);
    if (plan_has_odd(plan))
        hipLaunchKernelGGL((k_fft_axis<T, true>), dim3(cdiv(nlines, TL)), dim3(block_threads(TL * n)), lds, st, rsrc,
                           static_cast<typename V2<T>::t*>(X), rdst, n, s, nlines, sign, plan, TL);
    else
        hipLaunchKernelGGL((k_fft_axis<T, false>), dim3(cdiv(nlines, TL)), dim3(block_threads(TL * n)), lds, st, rsrc,
                           static_cast<typename V2<T>::t*>(X), rdst, n, s, nlines, sign, plan, TL);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_predict_fourier(const KModel& m, DevDesc* d, const double* coef, void* cbuf, T* P,
                                  hipStream_t st) {
    hipError_t e;
    // The exact integrator's gain is one exponential per mode: axis 0's forward
    // transform, the gain and axis 0's inverse transform then run as one launch, and so
    // do they in 1-D, where the whole spectrum is one short line.  The RK4 and Euler
    // gains of a multi-dimensional grid take a product over the substeps per mode, which
    // wants one thread per mode: separate launches.
    if (m.integ != PMF_INT_EXACT && m.nx > 1) {
        for (int a = m.nx - 1; a >= 0; --a) {
            e = launch_fft_axis<T>(m, a, a == m.nx - 1 ? P : nullptr, cbuf, nullptr, -1, st);
            if (e != hipSuccess) return e;
        }
        hipLaunchKernelGGL(k_gain<T>, dim3(cdiv(m.ntot, 256)), dim3(256), 0, st, m, d, coef,
                           static_cast<typename V2<T>::t*>(cbuf));
        for (int a = 0; a < m.nx; ++a) {
            e = launch_fft_axis<T>(m, a, nullptr, cbuf, a == m.nx - 1 ? P : nullptr, +1, st);
            if (e != hipSuccess) return e;
        }
        return hipGetLastError();
    }
    // forward: last (contiguous) axis first, reading the real density; axis 0 below
    for (int a = m.nx - 1; a >= 1; --a) {
        e = launch_fft_axis<T>(m, a, a == m.nx - 1 ? P : nullptr, cbuf, nullptr, -1, st);
        if (e != hipSuccess) return e;
    }
    // axis 0: forward, gain, inverse in one launch
    {
        using C = typename V2<T>::t;
        const int n = m.N[0], nlines = m.ntot / n;
        int TL = lines_per_block(n, nlines, sizeof(C));
        auto lds_of = [&](int tl) {
            return (2 * (size_t)tl * (n + 1) + n) * sizeof(C) + (size_t)tl * (6 * sizeof(T) + sizeof(int));
        };
        while (TL > 1 && lds_of(TL) > 65536) --TL;
        const FftPlan plan = make_plan(n);
        const T* rs = m.nx == 1 ? P : nullptr;
        T* rd = m.nx == 1 ? P : nullptr;
        C* Xc = static_cast<C*>(cbuf);
        if (plan_has_odd(plan))
            hipLaunchKernelGGL((k_fft_gain_axis0<T, true>), dim3(cdiv(nlines, TL)), dim3(block_threads(TL * n)),
                               lds_of(TL), st, m, d, coef, rs, Xc, rd, plan, TL);
        else
            hipLaunchKernelGGL((k_fft_gain_axis0<T, false>), dim3(cdiv(nlines, TL)), dim3(block_threads(TL * n)),
                               lds_of(TL), st, m, d, coef, rs, Xc, rd, plan, TL);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    for (int a = 1; a < m.nx; ++a) {
        e = launch_fft_axis<T>(m, a, nullptr, cbuf, a == m.nx - 1 ? P : nullptr, +1, st);
        if (e != hipSuccess) return e;
    }
    return hipGetLastError();
}

hipError_t launch_plan(const PredictArgs& a, DevDesc* d, double* coef, hipStream_t st) {
    if (a.nx == 1)
        hipLaunchKernelGGL(k_plan<1>, dim3(1), dim3(PLAN_THREADS), 0, st, a, d, coef);
    else if (a.nx == 2)
        hipLaunchKernelGGL(k_plan<2>, dim3(1), dim3(PLAN_THREADS), 0, st, a, d, coef);
    else if (a.nx == 3)
        hipLaunchKernelGGL(k_plan<3>, dim3(1), dim3(PLAN_THREADS), 0, st, a, d, coef);
    else
        hipLaunchKernelGGL(k_plan<4>, dim3(1), dim3(PLAN_THREADS), 0, st, a, d, coef);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_like(const KModel& m, const DevDesc* d, const double* tab, const double* z,
                       const T* P, T* Pout, double* part, int nb, int chunk, int mode, hipStream_t st) {
    ZArg za;
    for (int i = 0; i < 3; ++i) za.v[i] = (z && i < m.nz) ? z[i] : 0.0;
    switch (m.nx) {
        case 1: hipLaunchKernelGGL((k_like_pass<T, 1>), dim3(nb), dim3(RED_THREADS), 0, st, m, d, tab, za, P, Pout, part, chunk, mode); break;
        case 2: hipLaunchKernelGGL((k_like_pass<T, 2>), dim3(nb), dim3(RED_THREADS), 0, st, m, d, tab, za, P, Pout, part, chunk, mode); break;
        case 3: hipLaunchKernelGGL((k_like_pass<T, 3>), dim3(nb), dim3(RED_THREADS), 0, st, m, d, tab, za, P, Pout, part, chunk, mode); break;
        default: hipLaunchKernelGGL((k_like_pass<T, 4>), dim3(nb), dim3(RED_THREADS), 0, st, m, d, tab, za, P, Pout, part, chunk, mode); break;
    }
    return hipGetLastError();
}

hipError_t launch_update_finalize(const KModel& m, DevDesc* d, const double* part, int nb, double* bfac,
                                  hipStream_t st) {
    switch (m.nx) {
        case 1: hipLaunchKernelGGL(k_update_finalize<1>, dim3(1), dim3(RED_THREADS), 0, st, m, d, part, nb, bfac); break;
        case 2: hipLaunchKernelGGL(k_update_finalize<2>, dim3(1), dim3(RED_THREADS), 0, st, m, d, part, nb, bfac); break;
        case 3: hipLaunchKernelGGL(k_update_finalize<3>, dim3(1), dim3(RED_THREADS), 0, st, m, d, part, nb, bfac); break;
        default: hipLaunchKernelGGL(k_update_finalize<4>, dim3(1), dim3(RED_THREADS), 0, st, m, d, part, nb, bfac); break;
    }
    return hipGetLastError();
}

hipError_t launch_sums_finalize(const KModel& m, DevDesc* d, const double* part, int nb, double* bfac,
                                hipStream_t st) {
    switch (m.nx) {
        case 1: hipLaunchKernelGGL(k_sums_finalize<1>, dim3(1), dim3(RED_THREADS), 0, st, m, d, part, nb, bfac); break;
        case 2: hipLaunchKernelGGL(k_sums_finalize<2>, dim3(1), dim3(RED_THREADS), 0, st, m, d, part, nb, bfac); break;
        case 3: hipLaunchKernelGGL(k_sums_finalize<3>, dim3(1), dim3(RED_THREADS), 0, st, m, d, part, nb, bfac); break;
        default: hipLaunchKernelGGL(k_sums_finalize<4>, dim3(1), dim3(RED_THREADS), 0, st, m, d, part, nb, bfac); break;
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_scale_blocks(T* P, int ntot, int chunk, const double* bfac, hipStream_t st) {
    hipLaunchKernelGGL(k_scale_blocks<T>, dim3(cdiv(ntot, 256)), dim3(256), 0, st, P, ntot, chunk, bfac);
    return hipGetLastError();
}

// Re-interpolate `post` (normalised posterior on the old grid) onto the proposed
// grid, unnormalised, into `res`.  The device chooses the separable spectral or
// the Lagrange path (the other kernels return at once); `tmp` is scratch and
// `post` may be overwritten.
template <typename T>
hipError_t launch_interp(const KModel& m, DevDesc* d, const double* tab, double* W, T* post, T* tmp, T* res,
                         double* part, int nb, int chunk, hipStream_t st) {
    int maxn = 0;
    for (int a = 0; a < m.nx; ++a) maxn = m.N[a] > maxn ? m.N[a] : maxn;
    hipLaunchKernelGGL(k_interp_weights, dim3(cdiv(maxn * maxn, 256), m.nx), dim3(256), 0, st, m, d, tab, W);
    // axis passes alternate between tmp and post and end in res
    T* seq[MS + 1] = {post, res, nullptr, nullptr, nullptr};
    for (int a = 1; a < m.nx; ++a) seq[a] = (a % 2) ? tmp : post;
    seq[m.nx] = res;
    for (int a = 0; a < m.nx; ++a)
        hipLaunchKernelGGL(k_interp_axis<T>, dim3(nb), dim3(RED_THREADS), 0, st, m, d, tab, W, a, seq[a],
                           seq[a + 1], part, chunk, a == m.nx - 1 ? 1 : 0);
    switch (m.nx) {
        case 1: hipLaunchKernelGGL((k_interp_lagrange<T, 1>), dim3(nb), dim3(RED_THREADS), 0, st, m, d, tab, post, res, part, chunk); break;
        case 2: hipLaunchKernelGGL((k_interp_lagrange<T, 2>), dim3(nb), dim3(RED_THREADS), 0, st, m, d, tab, post, res, part, chunk); break;
        case 3: hipLaunchKernelGGL((k_interp_lagrange<T, 3>), dim3(nb), dim3(RED_THREADS), 0, st, m, d, tab, post, res, part, chunk); break;
        default: hipLaunchKernelGGL((k_interp_lagrange<T, 4>), dim3(nb), dim3(RED_THREADS), 0, st, m, d, tab, post, res, part, chunk); break;
    }
    hipLaunchKernelGGL(k_interp_finalize, dim3(1), dim3(RED_THREADS), 0, st, m, d, part, nb);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_final_scale(T* out, const T* old, int ntot, const DevDesc* d, hipStream_t st) {
    hipLaunchKernelGGL(k_final_scale<T>, dim3(cdiv(ntot, 256)), dim3(256), 0, st, out, old, ntot, d);
    return hipGetLastError();
}

hipError_t launch_prior(const KModel& m, const KPrior& pr, const DevDesc* d, const double* tab, void* P,
                        int prec, hipStream_t st) {
    hipLaunchKernelGGL(k_prior, dim3(cdiv(m.ntot, 256)), dim3(256), 0, st, m, pr, d, tab, P, prec);
    return hipGetLastError();
}

// f(y) = 1/2 sum_a Dy_aa D2_a y + sum_{a<b} Dy_ab D1_a (D1_b y)  (stage coefficient set k)
template <typename T>
hipError_t launch_cheb_rhs(const KModel& m, const T* D1, const T* D2, const double* coef, int k, const T* y,
                           T* kf, T* t1, T* t2, hipStream_t st) {
    const int nx = m.nx;
    const int ntot = m.ntot;
    const int g = cdiv(ntot, 256);
    int strides[3];
    for (int a = 0; a < nx; ++a) {
        int s = 1;
        for (int b = a + 1; b < nx; ++b) s *= m.N[b];
        strides[a] = s;
    }
    for (int a = 0; a < nx; ++a) {
        hipLaunchKernelGGL(k_axis_mm<T>, dim3(g), dim3(256), 0, st, D2 + (size_t)a * 256 * 256, y, kf, m.N[a],
                           strides[a], ntot, coef, PACK * k + pk(a, a), 0.5, a > 0 ? 1 : 0);
    }
    T* tb[3] = {nullptr, t1, t2};
    for (int b = 1; b < nx; ++b) {
        hipLaunchKernelGGL(k_axis_mm<T>, dim3(g), dim3(256), 0, st, D1 + (size_t)b * 256 * 256, y, tb[b], m.N[b],
                           strides[b], ntot, coef, -1, 1.0, 0);
    }
    for (int a = 0; a < nx; ++a)
        for (int b = a + 1; b < nx; ++b)
            hipLaunchKernelGGL(k_axis_mm<T>, dim3(g), dim3(256), 0, st, D1 + (size_t)a * 256 * 256, tb[b], kf,
                               m.N[a], strides[a], ntot, coef, PACK * k + pk(a, b), 1.0, 1);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_rk4_stage(T* q, T* y, const T* kf, T* acc, int ntot, const DevDesc* d, int stage,
                            hipStream_t st) {
    hipLaunchKernelGGL(k_rk4_stage<T>, dim3(cdiv(ntot, 256)), dim3(256), 0, st, q, y, kf, acc, ntot, d, stage);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_scale_etr(T* q, int ntot, const DevDesc* d, hipStream_t st) {
    hipLaunchKernelGGL(k_scale_by<T>, dim3(cdiv(ntot, 256)), dim3(256), 0, st, q, ntot, d);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_copy(T* dst, const T* src, int ntot, hipStream_t st) {
    hipLaunchKernelGGL(k_copy<T>, dim3(cdiv(ntot, 256)), dim3(256), 0, st, dst, src, ntot);
    return hipGetLastError();
}

// ------------------------------------------------------------------ finite-difference baseline
// Sine-transform route of eq. FST: X <- S_a X along every axis (S_a[i][j] =
// sin((i+1)(j+1) pi / (N_a+1)), the DST-I), times the product over the l steps
// of the eigenvalues of the explicit step, times prod_a 2 / (N_a + 1) (R^-1 =
// 2/(N+1) R), then S_a again.

// sine: the sine-series variant of the spectral update instead: each sine mode
// decays by exp(-1/2 sum_a Wy_aa k_a^2) e^{-tr(A) T}, k_a = (i_a + 1) pi / (N_a + 1)
// (coef holds W_y packed 00, 11, 22, ... as for the exact integrator)
template <typename T>
__global__ void k_fdm_gain(T* X, KModel m, const DevDesc* d, const double* coef, double trA, int sine) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= m.ntot) return;
    double cm1[MS] = {0.0, 0.0, 0.0, 0.0};   // cos(theta_a) - 1
    double norm = 1.0;
    int rem = j;
    for (int a = m.nx - 1; a >= 0; --a) {
        const int ia = rem % m.N[a];
        rem /= m.N[a];
        cm1[a] = cospi((double)(ia + 1) / (double)(m.N[a] + 1)) - 1.0;
        norm *= 2.0 / (double)(m.N[a] + 1);
    }
    double g = norm;
    if (sine) {
        double q = 0.0;
        rem = j;
        for (int a = m.nx - 1; a >= 0; --a) {
            const int ia = rem % m.N[a];
            rem /= m.N[a];
            const double k = M_PI * (double)(ia + 1) / (double)(m.N[a] + 1);
            q += coef[a] * k * k;
        }
        g *= d->etr * exp(-0.5 * q);
    } else {
        const int l = d->l;
        const double h = d->h;
        for (int n = 0; n < l; ++n) {
            const double* c = coef + PACK * n;   // packed diagonal first
            double lam = 1.0 - h * trA;
            for (int a = 0; a < m.nx; ++a) lam += h * c[a] * cm1[a];
            g *= lam;
        }
    }
    X[j] = (T)((double)X[j] * g);
}

template <typename T>
hipError_t launch_dst1_axis(const KModel& m, int a, const T* src, T* dst, hipStream_t st) {
    const int n = m.N[a];
    const int L = 2 * (n + 1);
    int s = 1;
    for (int b = a + 1; b < m.nx; ++b) s *= m.N[b];
    const int nlines = m.ntot / n;
    const int TL = lines_per_block(L, nlines, sizeof(typename V2<T>::t));
    const size_t lds = (2 * (size_t)TL * (L + 1) + L) * sizeof(typename V2<T>::t) + (size_t)TL * sizeof(int);
    const FftPlan plan = make_plan(L);
    if (plan_has_odd(plan))
        hipLaunchKernelGGL((k_dst1_axis<T, true>), dim3(cdiv(nlines, TL)), dim3(block_threads(TL * L)), lds, st, src,
                           dst, n, s, nlines, plan, TL);
    else
        hipLaunchKernelGGL((k_dst1_axis<T, false>), dim3(cdiv(nlines, TL)), dim3(block_threads(TL * L)), lds, st, src,
                           dst, n, s, nlines, plan, TL);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_predict_fdm(const KModel& m, const DevDesc* d, const double* coef, T* X, T* t1, T* t2,
                              double trA, int sine, hipStream_t st) {
    const int g = cdiv(m.ntot, 256);
    hipError_t e = hipSuccess;
    // forward sine transform along every axis: X -> t1 -> t2 -> ...
    const T* cur = X;
    for (int a = 0; a < m.nx && e == hipSuccess; ++a) {
        T* dst = (cur == t1) ? t2 : t1;
        e = launch_dst1_axis<T>(m, a, cur, dst, st);
        cur = dst;
    }
    if (e != hipSuccess) return e;
    T* spec = const_cast<T*>(cur);
    hipLaunchKernelGGL(k_fdm_gain<T>, dim3(g), dim3(256), 0, st, spec, m, d, coef, trA, sine);
    // back along every axis (the DST-I is its own inverse up to the factors the gain carries), ending in X
    for (int a = 0; a < m.nx && e == hipSuccess; ++a) {
        T* dst = (a == m.nx - 1) ? X : ((cur == t1) ? t2 : t1);
        e = launch_dst1_axis<T>(m, a, cur, dst, st);
        cur = dst;
    }
    if (e != hipSuccess) return e;
    return hipGetLastError();
}

#define PMF_INSTANTIATE(T)                                                                                   \
    template hipError_t launch_predict_fourier<T>(const KModel&, DevDesc*, const double*, void*, T*,         \
                                                  hipStream_t);                                              \
    template hipError_t launch_like<T>(const KModel&, const DevDesc*, const double*, const double*, const T*, \
                                       T*, double*, int, int, int, hipStream_t);                             \
    template hipError_t launch_scale_blocks<T>(T*, int, int, const double*, hipStream_t);                    \
    template hipError_t launch_interp<T>(const KModel&, DevDesc*, const double*, double*, T*, T*, T*,        \
                                         double*, int, int, hipStream_t);                                    \
    template hipError_t launch_final_scale<T>(T*, const T*, int, const DevDesc*, hipStream_t);               \
    template hipError_t launch_cheb_rhs<T>(const KModel&, const T*, const T*, const double*, int, const T*,  \
                                           T*, T*, T*, hipStream_t);                                         \
    template hipError_t launch_rk4_stage<T>(T*, T*, const T*, T*, int, const DevDesc*, int, hipStream_t);   \
    template hipError_t launch_scale_etr<T>(T*, int, const DevDesc*, hipStream_t);                           \
    template hipError_t launch_predict_fdm<T>(const KModel&, const DevDesc*, const double*, T*, T*, T*,      \
                                              double, int, hipStream_t);                                       \
    template hipError_t launch_copy<T>(T*, const T*, int, hipStream_t);

PMF_INSTANTIATE(float)
PMF_INSTANTIATE(double)

}  // namespace pmf
