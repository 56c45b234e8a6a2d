// Batched (many uneven problems, one persistent launch) protected FP64 GEMM.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ftg_common.hpp"

namespace ftg {

// One problem of a batched call (device-resident descriptor table).
struct BatchDesc {
    const double* A;
    const double* B;
    double* C;
    int lda, ldb, ldc;
    int m, n, k;
    int ta, tb;
    int tile;          // tile configuration id
    int tiles_m, tiles_n;
    int kc;
    double alpha, beta;
    InjectParams inj;
};

hipError_t launch_report_reset(DevReport* rep, hipStream_t s);

}  // namespace ftg
