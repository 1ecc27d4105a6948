// Chebyshev time update (RK4 method of lines, Sec. 4) with the dense
// differentiation matrices applied on MFMA (v_mfma_f32_16x16x4f32), FP32.
//
// One RK stage evaluates f(y) = 1/2 sum_a Dy_aa D2_a y + sum_{a<b} Dy_ab D1_a (D1_b y)
// in one pass per axis, last axis first, with 7 line products in 3-D (5 in 2-D):
//   last axis b = nx-1 : kf  = 1/2 Dy_bb D2_b y;  t = D1_b y, stored as
//                        u = Dy_01 t in 2-D and as t_2 = t in 3-D
//   middle axis (nx=3) : kf += 1/2 Dy_11 D2_1 y + Dy_12 D1_1 t_2;
//                        u = Dy_01 D1_1 y + Dy_02 t_2
//   first axis 0       : f = kf + 1/2 Dy_00 D2_0 y + D1_0 u   (D1_0 is linear, so
//                        Dy_01 D1_0 D1_1 y + Dy_02 D1_0 D1_2 y = D1_0 u),
//                        followed by the RK4 stage bookkeeping on (q, y, acc)
// Along axis a the N x N matrices multiply N-element lines.  A workgroup owns 16
// lines, held in LDS as In[line][k]; wave w computes output rows 16 w .. 16 w + 15
// of them as one 16 x 16 MFMA accumulator summed over K = N in blocks of 16 (4
// MFMAs of K = 4 per block; the k of a block is spread as 4 lk + m so that each
// lane reads 4 consecutive k with one 16-byte load from the matrix row and from
// the tile).  Every global load of a pass (tile, matrix rows, epilogue operands)
// is issued before the first wait, so a pass costs one memory round trip.
#include "api_internal.h"
#include "kernels.h"

namespace pmf {

typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int CL = 16;   // lines per workgroup

struct ChebGeom {
    int nx, ntot, N[3], stride[3];
};

enum { PASS_LAST = 0, PASS_MID = 1, PASS_FIRST = 2 };

__device__ inline floatx4 mfma4(const float4& a, const float4& b, floatx4 c) {
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, b.x, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, b.y, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(a.z, b.z, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(a.w, b.w, c, 0, 0, 0);
    return c;
}

// This thread's share of the 16-line tile starting at line L0: one float4.
// ROWS (s == 1): lines are contiguous rows, the float4 is 4 consecutive k of
// one line.  Otherwise s is a multiple of 16, the 16 lines share their outer
// index, and the float4 is lines 4c .. 4c+3 at one k.
template <int NB, bool ROWS>
__device__ inline float4 tile_fetch(const float* src, int L0, int s) {
    constexpr int n = 16 * NB;
    const int e = threadIdx.x;
    if (ROWS) {
        const int line = e / (n / 4), k4 = e - line * (n / 4);
        return *reinterpret_cast<const float4*>(src + (size_t)(L0 + line) * n + 4 * k4);
    }
    const int k = e >> 2, c = e & 3;
    const int o = L0 / s, i0 = L0 - o * s;
    return *reinterpret_cast<const float4*>(src + (size_t)o * n * s + i0 + (size_t)k * s + 4 * c);
}

template <int NB, bool ROWS>
__device__ inline void tile_store(float* T, const float4& v) {
    constexpr int n = 16 * NB, TS = n + 4;
    const int e = threadIdx.x;
    if (ROWS) {
        const int line = e / (n / 4), k4 = e - line * (n / 4);
        *reinterpret_cast<float4*>(T + line * TS + 4 * k4) = v;
    } else {
        const int k = e >> 2, c = e & 3;
        T[(4 * c + 0) * TS + k] = v.x;
        T[(4 * c + 1) * TS + k] = v.y;
        T[(4 * c + 2) * TS + k] = v.z;
        T[(4 * c + 3) * TS + k] = v.w;
    }
}

// One pass (see the header).  Block = NB waves (64 NB threads), 16 lines.
// coef holds the packed sets of D_y at the stage times (diagonal first, see pk).
template <int NB, int KIND>
__global__ void __launch_bounds__(64 * NB)
k_cheb_pass(ChebGeom G, int axis, const float* __restrict__ D1, const float* __restrict__ D2,
            const double* __restrict__ coef, int cidx, const DevDesc* __restrict__ d, int stage,
            const float* y, const float* tin, float* kf, float* tout, float* q, float* ynext, float* acc) {
    constexpr int n = 16 * NB, TS = n + 4;
    constexpr bool ROWS = KIND == PASS_LAST;
    constexpr bool TWO = KIND != PASS_LAST;   // a second tile: t_2 (middle) or u (first)
    __shared__ float Ty[CL * TS];
    __shared__ float Tt[TWO ? CL * TS : 1];
    const int s = G.stride[axis];
    const int L0 = blockIdx.x * CL;
    const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int li = l & 15, lk = l >> 4;
    const int i0 = 16 * w + 4 * lk;   // this lane's 4 output rows i0 .. i0+3 of line L0 + li

    // ---- issue every global load
    const float4 vy = tile_fetch<NB, ROWS>(y, L0, s);
    float4 vt;
    if (TWO) vt = tile_fetch<NB, ROWS>(tin, L0, s);
    float4 a1[NB], a2[NB];
    {
        const size_t r = (size_t)axis * 256 * 256 + (size_t)(16 * w + li) * n + 4 * lk;
#pragma unroll
        for (int kb = 0; kb < NB; ++kb) {
            a2[kb] = *reinterpret_cast<const float4*>(D2 + r + 16 * kb);
            a1[kb] = *reinterpret_cast<const float4*>(D1 + r + 16 * kb);
        }
    }
    size_t addr[4];
    {
        const int line = L0 + li;
        const int o = line / s, il = line - o * s;
        const size_t base = (size_t)o * n * s + il;
#pragma unroll
        for (int r = 0; r < 4; ++r) addr[r] = base + (size_t)(i0 + r) * s;
    }
    float kv[4] = {0.f, 0.f, 0.f, 0.f}, qv[4] = {0.f, 0.f, 0.f, 0.f}, av[4] = {0.f, 0.f, 0.f, 0.f};
    if (KIND != PASS_LAST) {
#pragma unroll
        for (int r = 0; r < 4; ++r) kv[r] = kf[addr[r]];
    }
    if (KIND == PASS_FIRST) {
#pragma unroll
        for (int r = 0; r < 4; ++r) qv[r] = q[addr[r]];
        if (stage > 1) {
#pragma unroll
            for (int r = 0; r < 4; ++r) av[r] = acc[addr[r]];
        }
    }
    const double* c = coef + PACK * cidx;
    const float h = (float)d->h;
    float cP, cX = 1.f, cY = 0.f, cT = 0.f;
    if (KIND == PASS_LAST) {
        cP = 0.5f * (float)c[G.nx - 1];
        cX = G.nx == 2 ? (float)c[pk(0, 1)] : 1.f;
    } else if (KIND == PASS_MID) {
        cP = 0.5f * (float)c[1];
        cX = (float)c[pk(0, 1)];   // u = Dy_01 D1_1 y + Dy_02 t_2
        cT = (float)c[pk(0, 2)];
        cY = (float)c[pk(1, 2)];   // kf += Dy_12 D1_1 t_2
    } else {
        cP = 0.5f * (float)c[0];
    }

    // ---- tiles to LDS
    tile_store<NB, ROWS>(Ty, vy);
    if (TWO) tile_store<NB, ROWS>(Tt, vt);
    __syncthreads();

    // ---- products: P = D2 y; X = D1 y (last, middle) or D1 u (first); Y = D1 t_2 (middle)
    floatx4 P = {0.f, 0.f, 0.f, 0.f}, X = P, Y = P;
#pragma unroll
    for (int kb = 0; kb < NB; ++kb) {
        const int kk = 16 * kb + 4 * lk;
        const float4 by = *reinterpret_cast<const float4*>(Ty + li * TS + kk);
        P = mfma4(a2[kb], by, P);
        if (KIND == PASS_FIRST) {
            const float4 bu = *reinterpret_cast<const float4*>(Tt + li * TS + kk);
            X = mfma4(a1[kb], bu, X);
        } else {
            X = mfma4(a1[kb], by, X);
        }
        if (KIND == PASS_MID) {
            const float4 bt = *reinterpret_cast<const float4*>(Tt + li * TS + kk);
            Y = mfma4(a1[kb], bt, Y);
        }
    }

    // ---- epilogue
    if (KIND == PASS_LAST) {
        // s == 1: the 4 rows are consecutive addresses of one line
        const float4 k4 = {cP * P[0], cP * P[1], cP * P[2], cP * P[3]};
        const float4 t4 = {cX * X[0], cX * X[1], cX * X[2], cX * X[3]};
        *reinterpret_cast<float4*>(kf + addr[0]) = k4;
        *reinterpret_cast<float4*>(tout + addr[0]) = t4;
    } else if (KIND == PASS_MID) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const float t2 = Tt[li * TS + i0 + r];
            kf[addr[r]] = kv[r] + cP * P[r] + cY * Y[r];
            tout[addr[r]] = cX * X[r] + cT * t2;
        }
    } else {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const float v = kv[r] + cP * P[r] + X[r];
            if (stage == 1) {
                acc[addr[r]] = v;
                ynext[addr[r]] = qv[r] + 0.5f * h * v;
            } else if (stage == 2) {
                acc[addr[r]] = av[r] + 2.f * v;
                ynext[addr[r]] = qv[r] + 0.5f * h * v;
            } else if (stage == 3) {
                acc[addr[r]] = av[r] + 2.f * v;
                ynext[addr[r]] = qv[r] + h * v;
            } else {
                q[addr[r]] = qv[r] + h / 6.f * (av[r] + v);
            }
        }
    }
}

// 3-D with square planes (N_1 = N_2 = n): the last- and middle-axis passes fused.
// A workgroup owns plane i0 (all of it in LDS) and a chunk of 16 columns j2.
//   step 1 (last axis, lines j1):    t2 = D1_2 y,  kp = 1/2 Dy_22 D2_2 y   on the chunk
//   step 2 (middle axis, lines j2):  kf = kp + 1/2 Dy_11 D2_1 y + Dy_12 D1_1 t2,
//                                    u  = Dy_01 D1_1 y + Dy_02 t2
// so t2 never leaves LDS and one launch replaces two.  Wave w takes lines
// 16w .. 16w+15 in step 1 and output rows 16w .. 16w+15 in step 2.
template <int NB>
__global__ void __launch_bounds__(64 * NB)
k_cheb_plane(int n0, const float* __restrict__ D1, const float* __restrict__ D2, const double* __restrict__ coef,
             int cidx, const float* __restrict__ y, float* __restrict__ kf, float* __restrict__ u) {
    constexpr int n = 16 * NB, TS = n + 4, CS = CL + 1;
    __shared__ float Yp[n * TS];      // the plane, Yp[j1][j2]
    __shared__ float T2[n * CS];      // t2 on the chunk, T2[j1][j2 - 16c]
    __shared__ float KP[n * CS];      // 1/2 Dy_22 D2_2 y on the chunk
    const int c = blockIdx.x, i0 = blockIdx.y;
    const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int li = l & 15, lk = l >> 4;
    const float* yp = y + (size_t)i0 * n * n;
    // ---- issue the global loads: the plane, the rows of the four matrices
    float4 vp[NB];
#pragma unroll
    for (int q = 0; q < NB; ++q) {
        const int e = threadIdx.x + q * 64 * NB;   // float4 index in the plane
        vp[q] = *reinterpret_cast<const float4*>(yp + 4 * e);
    }
    const float* D1a2 = D1 + (size_t)2 * 256 * 256;   // axis 2
    const float* D2a2 = D2 + (size_t)2 * 256 * 256;
    const float* D1a1 = D1 + (size_t)1 * 256 * 256;   // axis 1
    const float* D2a1 = D2 + (size_t)1 * 256 * 256;
    float4 s1[NB], s2[NB], m1[NB], m2[NB];
    {
        const size_t rc = (size_t)(16 * c + li) * n + 4 * lk;   // chunk rows of the axis-2 matrices
        const size_t rw = (size_t)(16 * w + li) * n + 4 * lk;   // this wave's rows of the axis-1 matrices
#pragma unroll
        for (int kb = 0; kb < NB; ++kb) {
            s1[kb] = *reinterpret_cast<const float4*>(D1a2 + rc + 16 * kb);
            s2[kb] = *reinterpret_cast<const float4*>(D2a2 + rc + 16 * kb);
            m1[kb] = *reinterpret_cast<const float4*>(D1a1 + rw + 16 * kb);
            m2[kb] = *reinterpret_cast<const float4*>(D2a1 + rw + 16 * kb);
        }
    }
    const double* cc = coef + PACK * cidx;
    const float c22h = 0.5f * (float)cc[2], c11h = 0.5f * (float)cc[1];
    const float c12 = (float)cc[pk(1, 2)], c01 = (float)cc[pk(0, 1)], c02 = (float)cc[pk(0, 2)];
#pragma unroll
    for (int q = 0; q < NB; ++q) {
        const int e = threadIdx.x + q * 64 * NB;
        const int r = e / (n / 4), k4 = e - r * (n / 4);
        *reinterpret_cast<float4*>(Yp + r * TS + 4 * k4) = vp[q];
    }
    __syncthreads();

    // ---- step 1: lines j1 = 16w + li, output rows j2 = 16c + 4lk + r
    {
        floatx4 P = {0.f, 0.f, 0.f, 0.f}, X = P;
#pragma unroll
        for (int kb = 0; kb < NB; ++kb) {
            const float4 b = *reinterpret_cast<const float4*>(Yp + (16 * w + li) * TS + 16 * kb + 4 * lk);
            P = mfma4(s2[kb], b, P);
            X = mfma4(s1[kb], b, X);
        }
        const int j1 = 16 * w + li;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            T2[j1 * CS + 4 * lk + r] = X[r];
            KP[j1 * CS + 4 * lk + r] = c22h * P[r];
        }
    }
    __syncthreads();

    // ---- step 2: lines j2 = 16c + li, output rows j1 = 16w + 4lk + r
    floatx4 P = {0.f, 0.f, 0.f, 0.f}, X = P, Y = P;
#pragma unroll
    for (int kb = 0; kb < NB; ++kb) {
        const int k0 = 16 * kb + 4 * lk;
        float4 by, bt;
        by.x = Yp[(k0 + 0) * TS + 16 * c + li];
        by.y = Yp[(k0 + 1) * TS + 16 * c + li];
        by.z = Yp[(k0 + 2) * TS + 16 * c + li];
        by.w = Yp[(k0 + 3) * TS + 16 * c + li];
        bt.x = T2[(k0 + 0) * CS + li];
        bt.y = T2[(k0 + 1) * CS + li];
        bt.z = T2[(k0 + 2) * CS + li];
        bt.w = T2[(k0 + 3) * CS + li];
        P = mfma4(m2[kb], by, P);
        X = mfma4(m1[kb], by, X);
        Y = mfma4(m1[kb], bt, Y);
    }
    float* kfp = kf + (size_t)i0 * n * n;
    float* up = u + (size_t)i0 * n * n;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int j1 = 16 * w + 4 * lk + r;
        const size_t a = (size_t)j1 * n + 16 * c + li;
        kfp[a] = KP[j1 * CS + li] + c11h * P[r] + c12 * Y[r];
        up[a] = c01 * X[r] + c02 * T2[j1 * CS + li];
    }
    (void)n0;
}

bool cheb_mfma_available(pmf_filter* f) {
    if (f->model.grid != PMF_GRID_CHEBYSHEV || f->model.precision != PMF_FP32) return false;
    if (f->model.nx < 2) return false;
    for (int a = 0; a < f->model.nx; ++a)
        if (f->model.N[a] % 16 != 0 || f->model.N[a] > 128) return false;
    return true;
}

template <int NB, int KIND>
static hipError_t launch_pass(const ChebGeom& G, int axis, pmf_filter* f, int cidx, int stage, const float* y,
                              const float* tin, float* kf, float* tout, float* q, float* ynext, float* acc,
                              hipStream_t st) {
    const int lines = G.ntot / G.N[axis];
    hipLaunchKernelGGL((k_cheb_pass<NB, KIND>), dim3(lines / CL), dim3(64 * NB), 0, st, G, axis,
                       static_cast<const float*>(f->D1), static_cast<const float*>(f->D2), f->coef, cidx, f->desc,
                       stage, y, tin, kf, tout, q, ynext, acc);
    return hipGetLastError();
}

template <int KIND>
static hipError_t launch_pass_n(const ChebGeom& G, int axis, pmf_filter* f, int cidx, int stage, const float* y,
                                const float* tin, float* kf, float* tout, float* q, float* ynext, float* acc,
                                hipStream_t st) {
#define PMF_CHEB_CASE(nb) \
    case nb: return launch_pass<nb, KIND>(G, axis, f, cidx, stage, y, tin, kf, tout, q, ynext, acc, st);
    switch (G.N[axis] / 16) {
        PMF_CHEB_CASE(1)
        PMF_CHEB_CASE(2)
        PMF_CHEB_CASE(3)
        PMF_CHEB_CASE(4)
        PMF_CHEB_CASE(5)
        PMF_CHEB_CASE(6)
        PMF_CHEB_CASE(7)
        PMF_CHEB_CASE(8)
    }
#undef PMF_CHEB_CASE
    return hipErrorInvalidValue;
}

static hipError_t launch_plane(const ChebGeom& G, pmf_filter* f, int cidx, const float* y, float* kf, float* u,
                               hipStream_t st) {
    const float* D1 = static_cast<const float*>(f->D1);
    const float* D2 = static_cast<const float*>(f->D2);
    const dim3 grid(G.N[2] / CL, G.N[0]);
#define PMF_PLANE_CASE(nb)                                                                                  \
    case nb:                                                                                                \
        hipLaunchKernelGGL(k_cheb_plane<nb>, grid, dim3(64 * nb), 0, st, G.N[0], D1, D2, f->coef, cidx, y, kf, u); \
        return hipGetLastError();
    switch (G.N[2] / 16) {
        PMF_PLANE_CASE(1)
        PMF_PLANE_CASE(2)
        PMF_PLANE_CASE(3)
        PMF_PLANE_CASE(4)
        PMF_PLANE_CASE(5)
        PMF_PLANE_CASE(6)
        PMF_PLANE_CASE(7)
        PMF_PLANE_CASE(8)
    }
#undef PMF_PLANE_CASE
    return hipErrorInvalidValue;
}

pmf_status cheb_predict_mfma(pmf_filter* f, int l, hipStream_t st) {
    ChebGeom G;
    G.nx = f->model.nx;
    G.ntot = f->ntot;
    for (int a = 0; a < 3; ++a) G.N[a] = a < G.nx ? f->model.N[a] : 1;
    for (int a = 0; a < 3; ++a) {
        int s = 1;
        for (int b = a + 1; b < G.nx; ++b) s *= G.N[b];
        G.stride[a] = s;
    }
    if (!cheb_mfma_available(f)) return fail(PMF_E_INVALID, "MFMA Chebyshev path: unsupported shape");
    float* q = static_cast<float*>(f->buf[f->cur]);
    float* y = static_cast<float*>(f->rk[0]);
    float* kf = static_cast<float*>(f->rk[1]);
    float* acc = static_cast<float*>(f->rk[2]);
    float* t1 = static_cast<float*>(f->rk[3]);
    float* t2 = static_cast<float*>(f->rk[4]);
    hipError_t e = hipSuccess;
    const int nx = G.nx;
    float* u = t1;   // D1_0 operand of the first-axis pass
    // square planes: the last- and middle-axis passes run fused
    const bool plane = nx == 3 && G.N[1] == G.N[2];
    for (int n = 0; n < l && e == hipSuccess; ++n) {
        // coefficient sets at the substep start, midpoint (twice) and end
        const int ks[4] = {2 * n, 2 * n + 1, 2 * n + 1, 2 * n + 2};
        for (int stg = 1; stg <= 4 && e == hipSuccess; ++stg) {
            const float* in = (stg == 1) ? q : y;
            const int k = ks[stg - 1];
            if (plane) {
                e = launch_plane(G, f, k, in, kf, u, st);
            } else {
                e = launch_pass_n<PASS_LAST>(G, nx - 1, f, k, stg, in, nullptr, kf, nx == 3 ? t2 : u, q, y, acc, st);
                if (e == hipSuccess && nx == 3)
                    e = launch_pass_n<PASS_MID>(G, 1, f, k, stg, in, t2, kf, u, q, y, acc, st);
            }
            if (e == hipSuccess) e = launch_pass_n<PASS_FIRST>(G, 0, f, k, stg, in, u, kf, nullptr, q, y, acc, st);
        }
    }
    if (e == hipSuccess) e = launch_scale_etr<float>(q, f->ntot, f->desc, st);
    if (e != hipSuccess) return hip_fail(e, "chebyshev MFMA predict");
    return PMF_OK;
}

}  // namespace pmf
