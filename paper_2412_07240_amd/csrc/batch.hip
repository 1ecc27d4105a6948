// Batched predict + update over many filters.
#include "api_internal.h"

namespace pmf {

void batch_cache_release(pmf_ctx*) {}
void batch_forget_filter(pmf_ctx*, pmf_filter*) {}

}  // namespace pmf

extern "C" pmf_status pmf_batch_step(pmf_ctx* ctx, pmf_filter* const* filters, int n, double T,
                                     const double* z, double* loglik, void* stream) {
    using namespace pmf;
    if (!ctx || (n > 0 && (!filters || !z))) return fail(PMF_E_INVALID, "NULL argument");
    int nzmax = 1;
    for (int i = 0; i < n; ++i) nzmax = filters[i]->model.nz > nzmax ? filters[i]->model.nz : nzmax;
    for (int i = 0; i < n; ++i) {
        pmf_status s = pmf_predict(filters[i], T, stream);
        if (s == PMF_OK) s = pmf_update(filters[i], z + (size_t)i * nzmax, loglik ? loglik + i : nullptr, stream);
        if (s != PMF_OK) return s;
    }
    return PMF_OK;
}
