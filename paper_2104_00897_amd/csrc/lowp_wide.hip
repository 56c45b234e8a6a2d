// Wide (256 x 256 workgroup tile) low-precision GEMM launches.
#include "lowp_wide.hpp"

namespace ftg {

bool lowp_wide_ok(const LowpArgs& a, ftg_dtype t, int mode)
{
    const int bk = t == FTG_F8_E4M3 ? WCfg<true>::BK : WCfg<false>::BK;
    (void)mode;
    const bool type_ok = t == FTG_BF16 || t == FTG_F8_E4M3;
    return type_ok && a.vec_a && a.vec_b && a.k >= bk && a.k % bk == 0;
}

hipError_t launch_lowp_wide(const LowpArgs& a, ftg_dtype t, int mode, hipStream_t s)
{
    if (a.tiles_m <= 0 || a.tiles_n <= 0) return hipSuccess;
    if (!lowp_wide_ok(a, t, mode)) return hipErrorInvalidValue;
    if (mode == 1) {
        // the piece rows are read at 32-bit offsets: XSB's from XSA (bf16) or
        // from XSB (fp8), each row's k elements within its ldxs
        const int64_t pieces = t == FTG_F8_E4M3 ? kFp8Pieces : 3, eb = t == FTG_F8_E4M3 ? 1 : 2;
        if (!a.XSA || !a.XSB || a.XSB <= a.XSA || a.ldxs < a.k) return hipErrorInvalidValue;
        const int64_t gap = (const char*)a.XSB - (const char*)a.XSA;
        const int64_t span_a = pieces * a.tiles_m * (int64_t)a.ldxs * eb;
        const int64_t span_b = pieces * a.tiles_n * (int64_t)a.ldxs * eb;
        if (span_a >= (int64_t(1) << 31) || gap + span_b >= (int64_t(1) << 31)) return hipErrorInvalidValue;
    }
    if (t == FTG_F8_E4M3) return mode ? launch_lowp_wide_t<true, 1>(a, s) : launch_lowp_wide_t<true, 0>(a, s);
    return mode ? launch_lowp_wide_t<false, 1>(a, s) : launch_lowp_wide_t<false, 0>(a, s);
}

}  // namespace ftg
