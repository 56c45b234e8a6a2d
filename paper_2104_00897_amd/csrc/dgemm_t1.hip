// FP64 protected GEMM, tile configuration 1: 256 x 128 output tile, 2 x 2 waves.
#include "dgemm_kernel.hpp"

namespace ftg {
template hipError_t launch_tile<256, 128, 2, 2, false, 1>(const DGemmArgs&, bool, hipStream_t);
}  // namespace ftg
