// FP64 protected GEMM, tile configuration 5 at one workgroup per CU: the
// 128 x 128 output tile on 4 x 2 waves with the whole register file, for
// protected calls with beta != 0 whose epilogue outweighs the k loop (chosen
// by launch_dgemm).
#include "dgemm_kernel.hpp"

namespace ftg {
template hipError_t launch_tile<128, 128, 4, 2, true, 0>(const DGemmArgs&, bool, hipStream_t);
}  // namespace ftg
