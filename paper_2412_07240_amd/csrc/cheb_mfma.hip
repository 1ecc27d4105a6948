// Chebyshev differentiation-matrix products on MFMA.
#include "api_internal.h"

namespace pmf {

bool cheb_mfma_available(pmf_filter*) { return false; }

pmf_status cheb_predict_mfma(pmf_filter*, int, hipStream_t) {
    return fail(PMF_E_INVALID, "MFMA Chebyshev path not available");
}

}  // namespace pmf
