// Internal definitions of libpmf: device descriptor, kernel-side model, and the
// small FP64 matrix routines (4x4 at most) used on both host and device.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "../../include/pmf.h"

#define PMF_HD __host__ __device__ inline

namespace pmf {

constexpr int MAXNX = 4;
constexpr int MS = 4;                 // row stride of every small matrix (double[MS * MS])
constexpr int MSQ = MS * MS;
constexpr int PACK = 10;              // packed symmetric entries: 4 diagonal + 6 off-diagonal
constexpr int MAXMIX = 4;
constexpr double FDM_STABLE_STEP = 1.0;   // h * sum_a D_y,aa kept at or below this (explicit FDM)
constexpr int LMAX = 4096;            // largest substep count a predict may use
constexpr int NPART = 20;             // doubles per reduction partial
constexpr int RED_THREADS = 256;      // threads of every reduction block
constexpr double RK4_STABLE_STEP = 2.5;
constexpr double BOUNDARY_TOL = 1e-4;

enum { ST_DEGENERATE = PMF_E_DEGENERATE, ST_BOUNDARY = PMF_W_BOUNDARY };

// ---------------------------------------------------------------- small matrices
// row-major n x n stored in double[MSQ] with row stride MS

PMF_HD void mat_zero(double* a) {
    for (int i = 0; i < MSQ; ++i) a[i] = 0.0;
}
PMF_HD void mat_eye(double* a, int n) {
    mat_zero(a);
    for (int i = 0; i < n; ++i) a[i * MS + i] = 1.0;
}
PMF_HD void mat_copy(double* d, const double* s) {
    for (int i = 0; i < MSQ; ++i) d[i] = s[i];
}
// C = A B (n x n), C may not alias
PMF_HD void mat_mul(double* C, const double* A, const double* B, int n) {
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            double s = 0.0;
            for (int k = 0; k < n; ++k) s += A[i * MS + k] * B[k * MS + j];
            C[i * MS + j] = s;
        }
}
// C = A B^T
PMF_HD void mat_mul_bt(double* C, const double* A, const double* B, int n) {
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            double s = 0.0;
            for (int k = 0; k < n; ++k) s += A[i * MS + k] * B[j * MS + k];
            C[i * MS + j] = s;
        }
}
PMF_HD void mat_vec(double* y, const double* A, const double* x, int n) {
    for (int i = 0; i < n; ++i) {
        double s = 0.0;
        for (int k = 0; k < n; ++k) s += A[i * MS + k] * x[k];
        y[i] = s;
    }
}
// determinant of the 3x3 block of rows r0..r2, columns c0..c2
PMF_HD double det3_at(const double* a, int r0, int r1, int r2, int c0, int c1, int c2) {
    return a[r0 * MS + c0] * (a[r1 * MS + c1] * a[r2 * MS + c2] - a[r1 * MS + c2] * a[r2 * MS + c1]) -
           a[r0 * MS + c1] * (a[r1 * MS + c0] * a[r2 * MS + c2] - a[r1 * MS + c2] * a[r2 * MS + c0]) +
           a[r0 * MS + c2] * (a[r1 * MS + c0] * a[r2 * MS + c1] - a[r1 * MS + c1] * a[r2 * MS + c0]);
}
PMF_HD double mat_det(const double* a, int n) {
    if (n == 1) return a[0];
    if (n == 2) return a[0] * a[MS + 1] - a[1] * a[MS];
    if (n == 3) return det3_at(a, 0, 1, 2, 0, 1, 2);
    // expansion along the first row
    return a[0] * det3_at(a, 1, 2, 3, 1, 2, 3) - a[1] * det3_at(a, 1, 2, 3, 0, 2, 3) +
           a[2] * det3_at(a, 1, 2, 3, 0, 1, 3) - a[3] * det3_at(a, 1, 2, 3, 0, 1, 2);
}
// inverse by cofactors; returns the determinant (0 -> inverse undefined)
PMF_HD double mat_inv(double* r, const double* a, int n) {
    double d = mat_det(a, n);
    mat_zero(r);
    if (d == 0.0) return 0.0;
    if (n == 1) {
        r[0] = 1.0 / a[0];
    } else if (n == 2) {
        r[0] = a[MS + 1] / d;
        r[1] = -a[1] / d;
        r[MS] = -a[MS] / d;
        r[MS + 1] = a[0] / d;
    } else if (n == 3) {
        const double* A = a;
#define PMF_A(i, j) A[(i) * MS + (j)]
        r[0 * MS + 0] = (PMF_A(1, 1) * PMF_A(2, 2) - PMF_A(1, 2) * PMF_A(2, 1)) / d;
        r[0 * MS + 1] = (PMF_A(0, 2) * PMF_A(2, 1) - PMF_A(0, 1) * PMF_A(2, 2)) / d;
        r[0 * MS + 2] = (PMF_A(0, 1) * PMF_A(1, 2) - PMF_A(0, 2) * PMF_A(1, 1)) / d;
        r[1 * MS + 0] = (PMF_A(1, 2) * PMF_A(2, 0) - PMF_A(1, 0) * PMF_A(2, 2)) / d;
        r[1 * MS + 1] = (PMF_A(0, 0) * PMF_A(2, 2) - PMF_A(0, 2) * PMF_A(2, 0)) / d;
        r[1 * MS + 2] = (PMF_A(0, 2) * PMF_A(1, 0) - PMF_A(0, 0) * PMF_A(1, 2)) / d;
        r[2 * MS + 0] = (PMF_A(1, 0) * PMF_A(2, 1) - PMF_A(1, 1) * PMF_A(2, 0)) / d;
        r[2 * MS + 1] = (PMF_A(0, 1) * PMF_A(2, 0) - PMF_A(0, 0) * PMF_A(2, 1)) / d;
        r[2 * MS + 2] = (PMF_A(0, 0) * PMF_A(1, 1) - PMF_A(0, 1) * PMF_A(1, 0)) / d;
#undef PMF_A
    } else {
        // adjugate: r_ji = (-1)^{i+j} det(minor_ij) / d
        for (int i = 0; i < 4; ++i)
            for (int j = 0; j < 4; ++j) {
                int rr[3], cc[3], p = 0, q = 0;
                for (int k = 0; k < 4; ++k) {
                    if (k != i) rr[p++] = k;
                    if (k != j) cc[q++] = k;
                }
                const double m = det3_at(a, rr[0], rr[1], rr[2], cc[0], cc[1], cc[2]);
                r[j * MS + i] = (((i + j) & 1) ? -m : m) / d;
            }
    }
    return d;
}

// Matrix exponential of an n x n matrix (n <= 8, row-major with leading
// dimension ld): scaling and squaring with a degree-18 Taylor polynomial.
PMF_HD void expm_ld(double* out, const double* a, int n, int ld) {
    double nrm = 0.0;
    for (int i = 0; i < n; ++i) {
        double r = 0.0;
        for (int j = 0; j < n; ++j) r += fabs(a[i * ld + j]);
        nrm = r > nrm ? r : nrm;
    }
    int sq = 0;
    double scale = 1.0;
    while (nrm * scale > 0.25 && sq < 60) {
        scale *= 0.5;
        ++sq;
    }
    double X[64], term[64], tmp[64];
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            X[i * 8 + j] = a[i * ld + j] * scale;
            term[i * 8 + j] = (i == j) ? 1.0 : 0.0;
            out[i * ld + j] = term[i * 8 + j];
        }
    for (int k = 1; k <= 18; ++k) {
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                double s = 0.0;
                for (int m = 0; m < n; ++m) s += term[i * 8 + m] * X[m * 8 + j];
                tmp[i * 8 + j] = s / k;
            }
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                term[i * 8 + j] = tmp[i * 8 + j];
                out[i * ld + j] += tmp[i * 8 + j];
            }
    }
    for (int s = 0; s < sq; ++s) {
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                double v = 0.0;
                for (int m = 0; m < n; ++m) v += out[i * ld + m] * out[m * ld + j];
                tmp[i * 8 + j] = v;
            }
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) out[i * ld + j] = tmp[i * 8 + j];
    }
}

// e^{A t} for an MS-stride n x n matrix
PMF_HD void expm3(double* out, const double* A, double t, int n) {
    double a[MSQ];
    mat_zero(a);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) a[i * MS + j] = A[i * MS + j] * t;
    mat_zero(out);
    expm_ld(out, a, n, MS);
}

// W(T) = int_0^T e^{-As} D e^{-A^T s} ds via the block exponential
// expm([[-A, D], [0, A^T]] T) = [[e^{-AT}, W(T) e^{A^T T}], [0, e^{A^T T}]].
PMF_HD void w_integral(double* W, const double* A, const double* D, double T, int n) {
    double blk[64], E[64];
    for (int i = 0; i < 64; ++i) blk[i] = 0.0;
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            blk[i * 8 + j] = -A[i * MS + j] * T;
            blk[i * 8 + n + j] = D[i * MS + j] * T;
            blk[(n + i) * 8 + n + j] = A[j * MS + i] * T;
        }
    expm_ld(E, blk, 2 * n, 8);
    double E12[MSQ], emAT[MSQ], Wt[MSQ];
    mat_zero(E12);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) E12[i * MS + j] = E[i * 8 + n + j];
    // e^{-A^T T} is the transpose of E11 = e^{-AT}
    mat_zero(emAT);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) emAT[i * MS + j] = E[j * 8 + i];
    mat_mul(Wt, E12, emAT, n);
    mat_zero(W);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) W[i * MS + j] = 0.5 * (Wt[i * MS + j] + Wt[j * MS + i]);
}

// packed symmetric coefficients: the diagonal 00, 11, 22, 33, then 01, 02, 03,
// 12, 13, 23
PMF_HD int pk(int a, int b) {
    if (a == b) return a;
    const int lo = a < b ? a : b, hi = a < b ? b : a;
    // offset of (lo, hi) among the pairs lo < hi in row order
    return 4 + (lo == 0 ? hi - 1 : (lo == 1 ? hi + 1 : 5));
}
PMF_HD void pack_sym(double* p, const double* S) {
    for (int a = 0; a < MS; ++a)
        for (int b = a; b < MS; ++b) p[pk(a, b)] = S[a * MS + b];
}

// M0^-1 E M0^-T
PMF_HD void sandwich_inv(double* out, const double* Mi, const double* E, int n) {
    double t[MSQ];
    mat_mul(t, Mi, E, n);
    mat_mul_bt(out, t, Mi, n);
}

// ---------------------------------------------------------------- descriptors

struct Grid {
    double c[MS];
    double M[MSQ];
    double Mi[MSQ];
    double vol;   // |det M|
};

PMF_HD void grid_finish(Grid& g, int n) {
    double d = mat_inv(g.Mi, g.M, n);
    g.vol = fabs(d);
}

// Per-filter state that lives in device memory (FP64).
struct DevDesc {
    Grid g;          // current grid
    Grid gn;         // grid proposed by the running update
    double t;
    int l;           // substeps of the last predict
    int status;      // sticky status bits since the last synchronising call
    int ok;          // 1 while the running update is accepted
    int sep;         // running update: separable spectral interpolation
    int par;         // batched steps: which of buffers 0/1 holds the density
    int pad_i;
    double s;        // likelihood shift
    double mass, loglik, bfrac;
    double mean[MS], cov[MSQ];
    double mass2;
    double h;        // substep length of the last predict
    double etr;      // e^{-tr(A) T} of the last predict
    double pscale;   // batched steps: the stored density times pscale is the density
    double pad1;
};

// Model constants passed to kernels by value.
struct KModel {
    int nx, grid, meas, nz, ncomp, interp, integ, prec;
    int N[MS];
    int ntot;
    int wstride;                 // doubles per axis in the separable weight buffer
    int nterr;                   // terrain measurement: number of cosine components
    int pad_k;
    double H[3 * MS];            // nz x nx, row stride MS
    double hp[4];
    double lw[MAXMIX];           // log w_g - 1/2 log det(2 pi R_g)
    double nmean[MAXMIX][3];
    double nRi[MAXMIX][MSQ];     // R_g^-1, row-major nz x nz (stride MS)
    double span;
    double Wnom[MSQ];
    double rho[MS];
    double terr[PMF_MAX_TERRAIN][2 + MS];   // amplitude, phase, frequency per state component
};

struct ZArg {
    double v[3];
};

// Host-side per-interval constants for a predict (depend on A, D, T only).
struct PredictArgs {
    double T;
    double etr;                  // e^{-tr(A) T}
    double A[MSQ], D[MSQ];
    double Phi[MSQ];             // e^{AT}
    double emh[MSQ];             // e^{-A T/2}
    double emT[MSQ];             // e^{-A T}
    double W[MSQ];               // W(T)
    int lmin, integ, nx, lmax;
    double rho[MS];
};

struct FftPlan {
    int np;
    int r[10];
};

PMF_HD FftPlan make_plan(int n) {
    FftPlan p;
    p.np = 0;
    while (n % 8 == 0 && n > 1) { p.r[p.np++] = 8; n /= 8; }
    while (n % 4 == 0) { p.r[p.np++] = 4; n /= 4; }
    while (n % 2 == 0) { p.r[p.np++] = 2; n /= 2; }
    while (n % 3 == 0) { p.r[p.np++] = 3; n /= 3; }
    while (n % 5 == 0 && p.np < 9) { p.r[p.np++] = 5; n /= 5; }
    while (n % 7 == 0 && p.np < 9) { p.r[p.np++] = 7; n /= 7; }
    while (n % 11 == 0 && p.np < 9) { p.r[p.np++] = 11; n /= 11; }
    while (n % 13 == 0 && p.np < 9) { p.r[p.np++] = 13; n /= 13; }
    while (n % 17 == 0 && p.np < 9) { p.r[p.np++] = 17; n /= 17; }
    if (n != 1) p.np = -1;
    return p;
}

}  // namespace pmf
