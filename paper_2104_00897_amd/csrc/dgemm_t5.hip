// FP64 protected GEMM, tile configuration 5: 128 x 128 output tile on 4 x 2 waves.
#include "dgemm_kernel.hpp"

namespace ftg {
template hipError_t launch_tile<128, 128, 4, 2, true, 1>(const DGemmArgs&, bool, hipStream_t);
}  // namespace ftg
