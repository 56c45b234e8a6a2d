// Low-precision (BF16 / FP8-e4m3 operands, FP32 accumulation) protected GEMM:
// launch interfaces used by the C ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/ftgemm.h"
#include "ftg_common.hpp"

namespace ftg {

// storage element types of the operands
struct StBF16 {
    using T = uint16_t;
    static constexpr int bytes = 2;
};
struct StFP8 {
    using T = uint8_t;
    static constexpr int bytes = 1;
};

// One low-precision GEMM launch: C (FP32, column-major) := alpha s_A s_B
// op(A) op(B) + beta C with 128 x 128 output tiles.  In protected mode the
// epilogue checks every tile against the checksum products ER, EC and the
// magnitude bounds RA, MB, CB, MA (see lowp_kernel.hpp).
struct LowpArgs {
    const void* A;
    const void* B;
    float* C;
    int lda, ldb, ldc;  // elements; < 2^20
    int m, n, k;
    int tiles_m, tiles_n;
    int vec_a, vec_b;   // 16-byte vector loads allowed (alignment of base and ld)
    float alpha, beta;
    const float* scale_a;  // device, NULL = 1
    const float* scale_b;
    // protected mode
    const float* ER;  // m x 3 tiles_n: A_I (B_J e) as three partial products per tile column
    const float* EC;  // 3 tiles_m x n: (e^T A_I) B_J likewise
    int lder, ldec;
    const float* RA;  // m: sum_p |a_ip|
    const float* MB;  // tiles_n: max_p sum_{j in J} |b_pj|
    const float* CB;  // n: sum_p |b_pj|
    const float* MA;  // tiles_m: max_p sum_{i in I} |a_ip|
    double lambda;
    int problem, pad;
    InjectParams inj;
    DevReport* rep;
    // plain mode: the k range split in `ksplit` slices (one workgroup per tile
    // and slice), slice s writing C + s cslice; protected mode: ER and EC hold
    // `slices` / `slices_c` such partial products, er_stride / ec_stride apart
    int ksplit, slices, slices_c;
    int vec_c;  // C base 16-byte aligned and ldc a multiple of 4
    // wide tile, protected: the encode pass's checksum pieces of A and B
    // (k-major rows of K elements: bf16 XS, or e4m3 XS8 for fp8 operands; XSB
    // after XSA, less than 2^31 bytes apart), multiplied inside the product
    // instead of by separate GEMMs
    const void* XSA;
    const void* XSB;
    int64_t cslice, er_stride, ec_stride;
    // verification intervals: this launch is the rank-k update of interval
    // `interval` of n_int (steps plo .. plo + k - 1 of the whole product; A, B
    // and XSA / XSB already point at step plo), whose injection slot is
    // tile * n_int + interval; ldxs = elements between rows of XSA / XSB
    int n_int, interval;
    int64_t plo;
    int ldxs;
};

// Encode pass over one operand.  // One operand X with rows r (i of op(A), or j of op(B)) and steps p:
// element (r, p) at X[p + r ld] when kcontig, else X[r + p ld].
struct EncOperand {
    const void* X;
    int64_t ld;
    int rows, K, kcontig;
    int vec;             // 16-byte loads allowed (base and ld aligned)
    int panels, chunks;  // panel = output-tile extent; chunk = kLowpChunk steps
    int ichunks;         // chunks per verification interval (XR, XM: one set per interval)
    uint16_t* XS;        // bf16 pieces: XS[(3 panel + s) K + p] (NULL: not written)
    uint8_t* XS8;        // e4m3 pieces with scales 2^(7 - 4 t):
                         // XS8[(8 panel + t) K + p] (NULL: not written)
    float* XRp;          // partial |x| row sums: XRp[chunk rows + r]
    float* XMp;          // partial panel maxima: XMp[panel chunks + chunk]
    float* XR;           // finalised per interval t (steps of chunks t ichunks ..):
                         // XR[t rows + r] = sum_p |x(r, p)| (rounded up)
    float* XM;           // XM[t panels + panel] = max_p sum_{r in panel} |x(r, p)|
};
struct EncArgs {
    EncOperand op[2];
};

constexpr int kLowpTile = 128;   // output tile extent (rows and columns)
constexpr int kFp8Pieces = 8;    // e4m3 pieces of a panel sum (wide fp8 protected)
constexpr int kLowpBK = 64;      // k-block
constexpr int kLowpChunk = 64;   // k steps per encode block

// mode 0: plain; mode 1: protected.  sta/stb: storage types (FTG_BF16 or
// FTG_F8_E4M3); FP8 x FP8 runs on the fp8 MFMA, any other mix on the bf16 one.
hipError_t launch_lowp_gemm(const LowpArgs& a, ftg_dtype sta, ftg_dtype stb, int ta, int tb, int mode,
                            hipStream_t s);
hipError_t launch_lowp_encode(const EncArgs& e, ftg_dtype st, int grid_x, int finish_x, hipStream_t s);
// k-major copy P[p + r ldp] of an operand with contiguous rows X[r + p ld]
// (eb = element bytes, ldp a multiple of 16, P 16-byte aligned; vec: X rows
// allow 16-byte loads)
hipError_t launch_lowp_pack(const void* X, int64_t ld, int64_t rows, int64_t K, int eb, void* P, int64_t ldp,
                            int vec, hipStream_t s);
hipError_t launch_sscale(float* C, int64_t m, int64_t n, int64_t ldc, float beta, hipStream_t s);

template <typename STA, typename STB, bool F8MMA, int MODE>
hipError_t launch_lowp_t(const LowpArgs& a, int ta, int tb, hipStream_t s);

void lowp_tile_shape(ftg_dtype t, int id, int* bm, int* bn, int* bk);
// tile configuration 2: workgroups of 2 x 2 checksum tiles (256 x 256 outputs),
// k-contiguous operands with 16-byte rows and K a multiple of the k-block
constexpr int kLowpWideTile = 2;
bool lowp_wide_ok(const LowpArgs& a, ftg_dtype t, int mode);
hipError_t launch_lowp_wide(const LowpArgs& a, ftg_dtype t, int mode, hipStream_t s);
int lowp_heuristic_tile(ftg_dtype t, int64_t m, int64_t n, int64_t k);

}  // namespace ftg
