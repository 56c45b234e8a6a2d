// Placeholder for the batched persistent kernel.
#include <hip/hip_runtime.h>

#include "../../include/ftgemm.h"
#include "ftg_batched.hpp"

extern "C" ftg_status ftg_dgemm_batched_uneven(ftg_handle, int64_t, const ftg_op*, const ftg_op*,
                                               const int64_t*, const int64_t*, const int64_t*,
                                               const double*, const double* const*, const int64_t*,
                                               const double* const*, const int64_t*, const double*,
                                               double* const*, const int64_t*, const uint32_t*, void*,
                                               const ftg_config*)
{
    return FTG_ERR_UNSUPPORTED;
}

extern "C" ftg_status ftg_batched_reserve(ftg_handle, int64_t) { return FTG_OK; }
