// Repair-kernel interface shared by the single, batched and low-precision entry points.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ftg_common.hpp"

namespace ftg {

// What the repair kernel needs to know about one problem.
struct RepairProblem {
    const void* A;
    const void* B;
    void* C;
    int64_t lda, ldb, ldc, k;
    int ta, tb, correct_policy, ab_type, c_type, pad;
    double alpha, beta;
    const float* scale_a;  // device per-tensor scales of FP8 operands (NULL = 1)
    const float* scale_b;
};

constexpr int kRepairBlocks = 256;  // one queued request per workgroup, one workgroup per CU

hipError_t launch_report_reset(DevReport* rep, hipStream_t s);
hipError_t launch_repair(DevReport* rep, const RepairProblem& single, const RepairProblem* table,
                         hipStream_t s);

}  // namespace ftg
