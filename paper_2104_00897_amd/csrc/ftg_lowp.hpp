// Low-precision (BF16 / FP8-e4m3 operands, FP32 accumulation) protected GEMM:
// tile table and launch interface.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/ftgemm.h"
#include "ftg_common.hpp"

namespace ftg {

void lowp_tile_shape(ftg_dtype t, int id, int* bm, int* bn, int* bk);
int lowp_heuristic_tile(ftg_dtype t, int64_t m, int64_t n, int64_t k);

}  // namespace ftg
