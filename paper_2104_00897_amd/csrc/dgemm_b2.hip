// FP64 protected GEMM, batched persistent launch with tile configuration 2
// (128 x 128 output tile, 2 x 2 waves).
#include "dgemm_kernel.hpp"

namespace ftg {
template hipError_t launch_batched<128, 128, 2, 2, true, 2>(const BatchLaunch&, int, int, bool, bool, bool, bool, hipStream_t);
}  // namespace ftg
