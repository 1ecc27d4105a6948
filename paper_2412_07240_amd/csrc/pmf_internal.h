// Internal definitions of libpmf: device descriptor, kernel-side model, and the
// small FP64 matrix routines (3x3 at most) used on both host and device.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "../../include/pmf.h"

#define PMF_HD __host__ __device__ inline

namespace pmf {

constexpr int MAXNX = 3;
constexpr int MAXMIX = 4;
constexpr double FDM_STABLE_STEP = 1.0;   // h * sum_a D_y,aa kept at or below this (explicit FDM)
constexpr int LMAX = 4096;            // largest substep count a predict may use
constexpr int NPART = 16;             // doubles per reduction partial
constexpr int RED_THREADS = 256;      // threads of every reduction block
constexpr double RK4_STABLE_STEP = 2.5;
constexpr double BOUNDARY_TOL = 1e-4;

enum { ST_DEGENERATE = PMF_E_DEGENERATE, ST_BOUNDARY = PMF_W_BOUNDARY };

// ---------------------------------------------------------------- small matrices
// row-major n x n stored in double[9]

PMF_HD void mat_zero(double* a) {
    for (int i = 0; i < 9; ++i) a[i] = 0.0;
}
PMF_HD void mat_eye(double* a, int n) {
    mat_zero(a);
    for (int i = 0; i < n; ++i) a[i * 3 + i] = 1.0;
}
PMF_HD void mat_copy(double* d, const double* s) {
    for (int i = 0; i < 9; ++i) d[i] = s[i];
}
// C = A B (n x n), C may not alias
PMF_HD void mat_mul(double* C, const double* A, const double* B, int n) {
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            double s = 0.0;
            for (int k = 0; k < n; ++k) s += A[i * 3 + k] * B[k * 3 + j];
            C[i * 3 + j] = s;
        }
}
// C = A B^T
PMF_HD void mat_mul_bt(double* C, const double* A, const double* B, int n) {
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            double s = 0.0;
            for (int k = 0; k < n; ++k) s += A[i * 3 + k] * B[j * 3 + k];
            C[i * 3 + j] = s;
        }
}
PMF_HD void mat_vec(double* y, const double* A, const double* x, int n) {
    for (int i = 0; i < n; ++i) {
        double s = 0.0;
        for (int k = 0; k < n; ++k) s += A[i * 3 + k] * x[k];
        y[i] = s;
    }
}
PMF_HD double mat_det(const double* a, int n) {
    if (n == 1) return a[0];
    if (n == 2) return a[0] * a[4] - a[1] * a[3];
    return a[0] * (a[4] * a[8] - a[5] * a[7]) - a[1] * (a[3] * a[8] - a[5] * a[6]) +
           a[2] * (a[3] * a[7] - a[4] * a[6]);
}
// inverse by cofactors; returns the determinant (0 -> inverse undefined)
PMF_HD double mat_inv(double* r, const double* a, int n) {
    double d = mat_det(a, n);
    mat_zero(r);
    if (d == 0.0) return 0.0;
    if (n == 1) {
        r[0] = 1.0 / a[0];
    } else if (n == 2) {
        r[0] = a[4] / d;
        r[1] = -a[1] / d;
        r[3] = -a[3] / d;
        r[4] = a[0] / d;
    } else {
        r[0] = (a[4] * a[8] - a[5] * a[7]) / d;
        r[1] = (a[2] * a[7] - a[1] * a[8]) / d;
        r[2] = (a[1] * a[5] - a[2] * a[4]) / d;
        r[3] = (a[5] * a[6] - a[3] * a[8]) / d;
        r[4] = (a[0] * a[8] - a[2] * a[6]) / d;
        r[5] = (a[2] * a[3] - a[0] * a[5]) / d;
        r[6] = (a[3] * a[7] - a[4] * a[6]) / d;
        r[7] = (a[1] * a[6] - a[0] * a[7]) / d;
        r[8] = (a[0] * a[4] - a[1] * a[3]) / d;
    }
    return d;
}

// Matrix exponential of an n x n matrix (n <= 6, row-major with leading
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
    double X[36], term[36], tmp[36];
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            X[i * 6 + j] = a[i * ld + j] * scale;
            term[i * 6 + j] = (i == j) ? 1.0 : 0.0;
            out[i * ld + j] = term[i * 6 + j];
        }
    for (int k = 1; k <= 18; ++k) {
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                double s = 0.0;
                for (int m = 0; m < n; ++m) s += term[i * 6 + m] * X[m * 6 + j];
                tmp[i * 6 + j] = s / k;
            }
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                term[i * 6 + j] = tmp[i * 6 + j];
                out[i * ld + j] += tmp[i * 6 + j];
            }
    }
    for (int s = 0; s < sq; ++s) {
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                double v = 0.0;
                for (int m = 0; m < n; ++m) v += out[i * ld + m] * out[m * ld + j];
                tmp[i * 6 + j] = v;
            }
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) out[i * ld + j] = tmp[i * 6 + j];
    }
}

// e^{A t} for a 3x3-stored n x n matrix
PMF_HD void expm3(double* out, const double* A, double t, int n) {
    double a[9];
    mat_zero(a);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) a[i * 3 + j] = A[i * 3 + j] * t;
    mat_zero(out);
    expm_ld(out, a, n, 3);
}

// W(T) = int_0^T e^{-As} D e^{-A^T s} ds via the block exponential
// expm([[-A, D], [0, A^T]] T) = [[e^{-AT}, W(T) e^{A^T T}], [0, e^{A^T T}]].
PMF_HD void w_integral(double* W, const double* A, const double* D, double T, int n) {
    double blk[36], E[36];
    for (int i = 0; i < 36; ++i) blk[i] = 0.0;
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            blk[i * 6 + j] = -A[i * 3 + j] * T;
            blk[i * 6 + n + j] = D[i * 3 + j] * T;
            blk[(n + i) * 6 + n + j] = A[j * 3 + i] * T;
        }
    expm_ld(E, blk, 2 * n, 6);
    double E12[9], emAT[9], Wt[9];
    mat_zero(E12);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) E12[i * 3 + j] = E[i * 6 + n + j];
    // e^{-A^T T} is the transpose of E11 = e^{-AT}
    mat_zero(emAT);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) emAT[i * 3 + j] = E[j * 6 + i];
    mat_mul(Wt, E12, emAT, n);
    mat_zero(W);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) W[i * 3 + j] = 0.5 * (Wt[i * 3 + j] + Wt[j * 3 + i]);
}

// packed symmetric coefficients: 00, 11, 22, 01, 02, 12
PMF_HD void pack_sym(double* p, const double* S) {
    p[0] = S[0];
    p[1] = S[4];
    p[2] = S[8];
    p[3] = S[1];
    p[4] = S[2];
    p[5] = S[5];
}

// M0^-1 E M0^-T
PMF_HD void sandwich_inv(double* out, const double* Mi, const double* E, int n) {
    double t[9];
    mat_mul(t, Mi, E, n);
    mat_mul_bt(out, t, Mi, n);
}

// ---------------------------------------------------------------- descriptors

struct Grid {
    double c[3];
    double M[9];
    double Mi[9];
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
    double mean[3], cov[9];
    double mass2;
    double h;        // substep length of the last predict
    double etr;      // e^{-tr(A) T} of the last predict
    double pscale;   // batched steps: the stored density times pscale is the density
    double pad1;
};

// Model constants passed to kernels by value.
struct KModel {
    int nx, grid, meas, nz, ncomp, interp, integ, prec;
    int N[3];
    int ntot;
    int wstride;                 // doubles per axis in the separable weight buffer
    int pad_k;
    double H[9];
    double hp[4];
    double lw[MAXMIX];           // log w_g - 1/2 log det(2 pi R_g)
    double nmean[MAXMIX][3];
    double nRi[MAXMIX][9];       // R_g^-1, row-major nz x nz
    double span;
    double Wnom[9];
    double rho[3];
};

struct ZArg {
    double v[3];
};

// Host-side per-interval constants for a predict (depend on A, D, T only).
struct PredictArgs {
    double T;
    double etr;                  // e^{-tr(A) T}
    double A[9], D[9];
    double Phi[9];               // e^{AT}
    double emh[9];               // e^{-A T/2}
    double emT[9];               // e^{-A T}
    double W[9];                 // W(T)
    int lmin, integ, nx, lmax;
    double rho[3];
};

struct FftPlan {
    int np;
    int r[8];
};

PMF_HD FftPlan make_plan(int n) {
    FftPlan p;
    p.np = 0;
    while (n % 8 == 0 && n > 1) { p.r[p.np++] = 8; n /= 8; }
    while (n % 4 == 0) { p.r[p.np++] = 4; n /= 4; }
    while (n % 2 == 0) { p.r[p.np++] = 2; n /= 2; }
    while (n % 3 == 0) { p.r[p.np++] = 3; n /= 3; }
    while (n % 5 == 0 && p.np < 8) { p.r[p.np++] = 5; n /= 5; }
    if (n != 1) p.np = -1;
    return p;
}

}  // namespace pmf
