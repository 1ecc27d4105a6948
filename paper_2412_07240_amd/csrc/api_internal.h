// Host-side objects behind the opaque handles of include/pmf.h.
#pragma once

#include <map>
#include <string>
#include <vector>

#include "pmf_internal.h"

struct BatchCache;
struct DynBatch;

struct pmf_ctx {
    int device = 0;
    bool has_alloc = false;
    pmf_allocator alloc{};
    BatchCache* batch = nullptr;
    long long batch_leaves = 0;                 // filters that left batched steps so far
    bool profile = false;                       // record events around batched launches
    std::vector<hipEvent_t> ev_pool;             // start/stop pairs, reused
    int ev_used = 0;
    hipStream_t ev_stream = nullptr;
    int sched[40] = {};                          // fused-kernel schedule per group type (autotuner)
};

struct pmf_filter {
    pmf_ctx* ctx = nullptr;
    pmf_model model{};
    pmf::KModel km{};
    double Wnom[pmf::MSQ] = {0};
    int ntot = 0;
    size_t es = 0;                 // bytes per density value
    void* buf[4] = {nullptr, nullptr, nullptr, nullptr};
    int cur = 0;                   // buffer holding the current density
    void* cbuf = nullptr;          // complex work array (Fourier)
    double* part = nullptr;        // reduction partials
    double* bfac = nullptr;        // per-block scale factors
    double* coef = nullptr;        // per-stage diffusion coefficients
    double* W = nullptr;           // separable interpolation weights
    double* tab = nullptr;         // per-axis tables
    pmf::DevDesc* desc = nullptr;
    void* D1 = nullptr;            // Chebyshev differentiation matrices (density precision)
    void* D2 = nullptr;
    void* rk[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};   // Chebyshev RK4 scratch
    bool cheb_d32_ready = false;
    bool in_batch = false;         // density lives in buffer desc->par (batched steps)
    int nb = 0, chunk = 0;         // reduction partition
    bool have_pa = false;
    pmf::PredictArgs pa{};
    size_t bytes = 0;              // device bytes this filter holds
    void* dconst = nullptr;        // device copy of the fused-step constants (served batches)
    double dconst_T = -1.0;        // interval those constants were built for
};

namespace pmf {

constexpr int MAX_RED_BLOCKS = 2048;   // reduction blocks per filter (more points: longer chunks)

// The reduction partition of a filter's ntot points: about 1024 blocks, each of 256 to
// 1024 points (one to four per thread of a reduction block), at most MAX_RED_BLOCKS
// blocks (longer chunks beyond), so that the generic passes of small grids still spread
// over many compute units.
inline void red_partition(int ntot, int* chunk, int* nb) {
    int c = (ntot + 1023) / 1024;
    c = c < 256 ? 256 : (c > 1024 ? 1024 : c);
    *chunk = c;
    *nb = (ntot + c - 1) / c;
    if (*nb > MAX_RED_BLOCKS) {
        *nb = MAX_RED_BLOCKS;
        *chunk = (ntot + *nb - 1) / *nb;
    }
}

extern thread_local std::string g_last_error;
pmf_status fail(pmf_status s, const std::string& msg);
pmf_status hip_fail(hipError_t e, const char* where);
void* ctx_alloc(pmf_ctx* ctx, size_t bytes, hipStream_t st);
void ctx_free(pmf_ctx* ctx, void* p, hipStream_t st);

hipError_t normalise_current(pmf_filter* f, hipStream_t st);
pmf_status take_status(pmf_filter* f);
const PredictArgs& predict_args(pmf_filter* f, double T);
pmf_status cheb_predict(pmf_filter* f, hipStream_t st);
void cheb_matrices(int N, std::vector<double>& D1, std::vector<double>& D2);

// Chebyshev products on MFMA (cheb_mfma.hip)
bool cheb_mfma_available(pmf_filter* f);
pmf_status cheb_predict_mfma(pmf_filter* f, int l, hipStream_t st);

// fused batched step (batch.hip)
void batch_cache_release(pmf_ctx* ctx);
void batch_forget_filter(pmf_ctx* ctx, pmf_filter* f);
hipError_t batch_leave(pmf_filter* f);
bool batch_fusable(const pmf_filter* f, std::string* why);
bool model_fusable(const pmf_model& m, std::string* why);
// device bytes pmf_create allocates for a validated model (without the fused-step
// constants, which fusable filters add: fused_const_bytes)
size_t filter_device_bytes(const pmf_model& model);
// validation of a model as pmf_create does it (PMF_OK or the error it returns)
pmf_status check_model(const pmf_model* model);
// bytes of a filter's fused-step constants (its record f->dconst; allocated at
// create for every filter the fused kernel accepts)
size_t fused_const_bytes();

// fused steps over a changing set of filters (served batches, batch.hip): the
// items are rebuilt on every call (nothing cached).  Asynchronous on st; the host
// staging is reused by the next call, so the caller waits for st in between.
DynBatch* dyn_create(pmf_ctx* ctx);
void dyn_destroy(pmf_ctx* ctx, DynBatch* db);
// z: n x 3 doubles (row i for filters[i]); after st completes, dyn_loglik(db)[i]
// is filter i's log-likelihood (NaN when its update was rejected)
pmf_status dyn_run(pmf_ctx* ctx, DynBatch* db, pmf_filter* const* filters, int n, double T, const double* z,
                   hipStream_t st);
const double* dyn_loglik(const DynBatch* db);

}  // namespace pmf
