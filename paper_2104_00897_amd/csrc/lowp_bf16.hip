// BF16 x BF16 -> FP32 GEMM (plain and protected), bf16 MFMA.
#include "lowp_kernel.hpp"

namespace ftg {
template hipError_t launch_lowp_t<StBF16, StBF16, false, 0>(const LowpArgs&, int, int, hipStream_t);
template hipError_t launch_lowp_t<StBF16, StBF16, false, 1>(const LowpArgs&, int, int, hipStream_t);
}  // namespace ftg
