// FP64 protected GEMM, batched persistent launch with tile configuration 3
// (64 x 64 output tile, 2 x 2 waves).
#include "dgemm_kernel.hpp"

namespace ftg {
template hipError_t launch_batched<64, 64, 2, 2, true, 2>(const BatchLaunch&, int, int, bool, bool, bool, bool, hipStream_t);
}  // namespace ftg
