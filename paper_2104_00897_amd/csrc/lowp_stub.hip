// Placeholder for the low-precision kernels (tile table only).
#include <hip/hip_runtime.h>

#include "ftg_lowp.hpp"

namespace ftg {

void lowp_tile_shape(ftg_dtype, int, int* bm, int* bn, int* bk) { *bm = *bn = *bk = 0; }
int lowp_heuristic_tile(ftg_dtype, int64_t, int64_t, int64_t) { return 0; }

}  // namespace ftg

extern "C" ftg_status ftg_gemm_ex(ftg_handle, ftg_op, ftg_op, int64_t, int64_t, int64_t, ftg_dtype,
                                  ftg_dtype, const float*, const float*, float, const void*, int64_t,
                                  const void*, int64_t, float, void*, int64_t, void*,
                                  const ftg_config*)
{
    return FTG_ERR_UNSUPPORTED;
}
