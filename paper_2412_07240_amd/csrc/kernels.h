// Host-side launchers of the generic kernels (kernels.hip).
#pragma once

#include "pmf_internal.h"

namespace pmf {

// per-axis FP64 table layout (stride TAB_STRIDE doubles per axis)
constexpr int TAB_QW = 256;     // quadrature weight of each index (Fourier: 1)
constexpr int TAB_V = 512;      // Chebyshev: all N+2 CGL nodes, ascending
constexpr int TAB_BETA = 770;   // Chebyshev: barycentric weights of those nodes
constexpr int TAB_STRIDE = 1040;

struct KPrior {
    int ncomp, pad[3];
    double lw[MAXMIX];          // log w_g - 1/2 log det(2 pi C_g)
    double mean[MAXMIX][MS];
    double Ci[MAXMIX][MSQ];
};

template <typename T>
hipError_t launch_predict_fourier(const KModel& m, DevDesc* d, const double* coef, void* cbuf, T* P,
                                  hipStream_t st);
hipError_t launch_plan(const PredictArgs& a, DevDesc* d, double* coef, hipStream_t st);
template <typename T>
hipError_t launch_like(const KModel& m, const DevDesc* d, const double* tab, const double* z, const T* P,
                       T* Pout, double* part, int nb, int chunk, int mode, hipStream_t st);
hipError_t launch_update_finalize(const KModel& m, DevDesc* d, const double* part, int nb, double* bfac,
                                  hipStream_t st);
hipError_t launch_sums_finalize(const KModel& m, DevDesc* d, const double* part, int nb, double* bfac,
                                hipStream_t st);
template <typename T>
hipError_t launch_scale_blocks(T* P, int ntot, int chunk, const double* bfac, hipStream_t st);
template <typename T>
hipError_t launch_interp(const KModel& m, DevDesc* d, const double* tab, double* W, T* post, T* tmp, T* res,
                         double* part, int nb, int chunk, hipStream_t st);
template <typename T>
hipError_t launch_final_scale(T* out, const T* old, int ntot, const DevDesc* d, hipStream_t st);
hipError_t launch_prior(const KModel& m, const KPrior& pr, const DevDesc* d, const double* tab, void* P,
                        int prec, hipStream_t st);
template <typename T>
hipError_t launch_cheb_rhs(const KModel& m, const T* D1, const T* D2, const double* coef, int k, const T* y,
                           T* kf, T* t1, T* t2, hipStream_t st);
template <typename T>
hipError_t launch_rk4_stage(T* q, T* y, const T* kf, T* acc, int ntot, const DevDesc* d, int stage,
                            hipStream_t st);
template <typename T>
hipError_t launch_scale_etr(T* q, int ntot, const DevDesc* d, hipStream_t st);

// finite-difference baseline by the sine-transform route, or (sine != 0) the
// sine-series variant of the spectral update, with the fast sine transform (DST-I
// through an FFT of length 2 (N_a + 1) per axis); t1, t2: two scratch densities;
// result in X
template <typename T>
hipError_t launch_predict_fdm(const KModel& m, const DevDesc* d, const double* coef, T* X, T* t1, T* t2,
                              double trA, int sine, hipStream_t st);
template <typename T>
hipError_t launch_copy(T* dst, const T* src, int ntot, hipStream_t st);

}  // namespace pmf
