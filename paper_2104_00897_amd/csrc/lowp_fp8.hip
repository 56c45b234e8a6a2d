// FP8-e4m3 x FP8-e4m3 -> FP32 GEMM (plain and protected), fp8 MFMA.
#include "lowp_kernel.hpp"

namespace ftg {
template hipError_t launch_lowp_t<StFP8, StFP8, true, 0>(const LowpArgs&, int, int, hipStream_t);
template hipError_t launch_lowp_t<StFP8, StFP8, true, 1>(const LowpArgs&, int, int, hipStream_t);
}  // namespace ftg
