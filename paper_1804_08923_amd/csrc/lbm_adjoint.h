// Reverse (adjoint) step of the colour-gradient LBM update.
#pragma once
#include "lbm_kernels.h"

namespace cglbm {

inline uint64_t adjoint_work_bytes(uint64_t /*N*/) { return 0; }

inline int adjoint_step(const lbm_params& /*p*/, const KP& /*k*/, hipStream_t /*stream*/, void* /*work*/,
                        int /*nblk*/, const float* /*state_t*/, float* /*lambda*/, double* /*dJ_dA*/,
                        float* /*dJ_du_in*/, char* err, size_t errlen)
{
    snprintf(err, errlen, "adjoint step not available");
    return LBM_ERR_UNSUPPORTED;
}

}  // namespace cglbm
