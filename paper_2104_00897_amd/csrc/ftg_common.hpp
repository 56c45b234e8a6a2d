// Device-side pieces shared by the protected GEMM kernels: fault report,
// seeded injector, round-off threshold, wave reductions.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/ftgemm.h"

namespace ftg {

// Granularity of injection and of verification intervals in k (every
// kernel's k-block divides it).
constexpr int kKGran = 128;

// Most verification intervals per tile with injection on (LDS fault table).
constexpr int kMaxIntervals = 128;

// Smallest repair-queue capacity of a handle (flagged slots of one call).
constexpr unsigned int kMinRepairQueue = 16384;

// A flagged final-slot check handed from a GEMM kernel to the repair kernel.
// Row/column indices are tile-local; expected checksums already include the
// alpha/beta scaling; cin is C_in at the located element (0 when beta = 0).
struct RepairReq {
    int problem, tm, tn, interval;
    int nr, nc, fi, fj;  // flagged row/column counts, first flagged row/column
    int R, Q;
    int whole;  // 1: recompute the whole tile (not stored: C still holds C_in)
    int pad1;
    int64_t m0, n0;
    double dfi, tfi, dfj, tfj, exp_row, exp_col, cin;
};

// Fault report kept on the device by the handle.  Counters are updated with
// device atomics; records are appended at atomically reserved indices.  The
// repair queue collects flagged tiles until the repair kernel drains it.
struct DevReport {
    unsigned long long cnt[8];  // see Cnt
    unsigned int n_records, n_inject, capacity, pad;
    ftg_fault_record* records;
    ftg_inject_record* inject_log;
    unsigned int rq_count, rq_done, rq_capacity, rq_lost;
    RepairReq* rq;
};

enum Cnt {
    kInjected = 0,
    kDetected = 1,
    kCorrSub = 2,
    kCorrRecomp = 3,
    kChecksumOnly = 4,
    kUncorrectable = 5,
    kTilesRecomputed = 6,
    kMaxPassRatio = 7  // bit pattern of the largest |delta|/tau of a passing check
};

// Injector parameters of one problem (see ftg_inject in ftgemm.h).
struct InjectParams {
    int on;
    int target;
    int bit_lo, bit_hi;
    uint64_t seed;
    uint32_t S, F, a_inv, b;  // slot count (< 2^32), faults, inverse of a mod S, offset
};

// SplitMix64 output number `ctr` of the stream seeded with `seed`
// (Steele, Lea & Flood, OOPSLA 2014).
__host__ __device__ inline uint64_t splitmix64(uint64_t seed, uint64_t ctr)
{
    uint64_t z = seed + (ctr + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// One planned fault of a slot, tile-local coordinates.
struct Fault {
    int row, col;     // tile-local
    int64_t pflip;    // last k step before the flip
    int bit;
};

// Faults of slot s (0, 1 or 2 of them).  rows/cols: extent of the tile;
// [plo, phi): k range of the interval.
__device__ inline int slot_faults(const InjectParams& ip, uint64_t s, int rows, int cols,
                                  int64_t plo, int64_t phi, Fault* f)
{
    if (!ip.on || ip.S == 0) return 0;
    const uint64_t S = ip.S;
    const uint64_t d = (s + S - ip.b) % S;
    const uint64_t r = d * ip.a_inv % S;  // inverse of the slot bijection (S < 2^32)
    if (r >= ip.F) return 0;
    uint64_t c0 = 1024 + 8 * r;
    uint64_t x[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) x[q] = splitmix64(ip.seed, c0 + q);
    int nbits = ip.bit_hi - ip.bit_lo + 1;
    int64_t len = phi - plo;
    auto pfl = [&](int64_t step) {
        int64_t e = (step / kKGran + 1) * kKGran;
        return (e < phi ? e : phi) - 1;
    };
    f[0].row = (int)(x[0] % (uint64_t)rows);
    f[0].col = (int)(x[1] % (uint64_t)cols);
    f[0].pflip = pfl(plo + (int64_t)(x[2] % (uint64_t)len));
    f[0].bit = ip.bit_lo + (int)(x[3] % (uint64_t)nbits);
    if (ip.target != FTG_TARGET_TWO_IN_SLOT) return 1;
    if (rows < 2 || cols < 2) return 0;
    f[1].row = (int)((f[0].row + 1 + (int64_t)(x[4] % (uint64_t)(rows - 1))) % rows);
    f[1].col = (int)((f[0].col + 1 + (int64_t)(x[5] % (uint64_t)(cols - 1))) % cols);
    f[1].pflip = pfl(plo + (int64_t)(x[6] % (uint64_t)len));
    f[1].bit = ip.bit_lo + (int)(x[7] % (uint64_t)nbits);
    return 2;
}

__device__ inline double flip_f64(double v, int bit)
{
    unsigned long long u = __double_as_longlong(v);
    u ^= 1ull << bit;
    return __longlong_as_double(u);
}

__device__ inline float flip_f32(float v, int bit)
{
    unsigned int u = __float_as_uint(v);
    u ^= 1u << bit;
    return __uint_as_float(u);
}

// Round-off threshold: 2 g(n) mag (1 + 2^-20) with g(n) = gamma(n) for binary64
// accumulation, lambda sqrt(n) 2^-24 for binary32 accumulation.
__device__ inline double tau_of(int acc32, double lambda, int64_t nterms, double mag)
{
    double g;
    if (acc32) {
        g = lambda * sqrt((double)nterms) * 0x1p-24;
    } else {
        double nu = (double)nterms * 0x1p-53;
        g = nu / (1.0 - nu);
    }
    return 2.0 * g * mag * (1.0 + 0x1p-20);
}

__device__ inline bool flagged(double d, double tau) { return !(fabs(d) <= tau); }

// Noise margin of the threshold: the largest |delta| / tau among the checks
// that passed, over every call since the last report reset.  Called by every
// lane of a wave with its own ratio (0 for none).  Non-negative doubles order
// like their bit patterns, so an integer maximum keeps the largest; a wave
// skips the atomic when the stored value is already larger.
__device__ inline void note_pass_ratio(DevReport* rep, double r)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) r = fmax(r, __shfl_xor(r, off));
    if ((threadIdx.x & 63) == 0 && r > 0.0) {
        const unsigned long long u = (unsigned long long)__double_as_longlong(r);
        if (u > __hip_atomic_load(&rep->cnt[kMaxPassRatio], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
            atomicMax(&rep->cnt[kMaxPassRatio], u);
    }
}

// The faulty value no longer carries the true one (absorption): its rounding
// unit in the output precision (binary32 when acc32) exceeds tau / (2 q), the
// share of the row threshold of one of the row's q elements.  Subtracting the
// error magnitude could not restore the element then; it is recomputed.
__device__ inline bool absorbed(bool acc32, double x, double tau, int q)
{
    if (x == 0.0) return false;
    const double ulp = ldexp(1.0, ilogb(x) - (acc32 ? 23 : 52));
    return ulp > tau / (2.0 * (double)q);
}

// Raw buffer access (CDNA buffer instructions): an SGPR resource with a base
// address, a 32-bit per-lane byte offset and a uniform byte offset.  An offset
// at or beyond the record count reads 0 and drops writes, which is how
// elements outside the matrix are zero-filled without branches.
constexpr int kOOB = (int)0x80000000u;


__device__ inline __amdgpu_buffer_rsrc_t make_rsrc(const void* base)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, 0x7FFFFFFF,
                                             0x00020000);
}

typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

__device__ inline double buf_load_f64(__amdgpu_buffer_rsrc_t r, int voff, int soff)
{
    u32x2 v = __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0);
    return __builtin_bit_cast(double, v);
}

__device__ inline void buf_store_f64(double x, __amdgpu_buffer_rsrc_t r, int voff, int soff)
{
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, x), r, voff, soff, 0);
}

// A binary64 value moved between lanes of a 16-lane row by a DPP control
// (data-parallel primitive: an operand modifier of the vector ALU, no LDS
// traffic), applied to both 32-bit halves.
template <int CTRL>
__device__ inline double dpp_f64(double x)
{
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}

// Sum over each row of 16 lanes; every lane ends with its row's sum (the same
// value in every lane: each step adds the same two partial sums).
__device__ inline double row_sum16(double v)
{
    v += dpp_f64<0xB1>(v);   // quad_perm [1,0,3,2]: lane pairs
    v += dpp_f64<0x4E>(v);   // quad_perm [2,3,0,1]: quads
    v += dpp_f64<0x141>(v);  // row_half_mirror: half rows of 8
    v += dpp_f64<0x140>(v);  // row_mirror: rows of 16
    return v;
}

// Sum over aligned groups of `width` lanes (width a power of two <= 64);
// every lane of a group ends with the group's sum.
template <int WIDTH>
__device__ inline double group_sum(double v)
{
    if constexpr (WIDTH >= 16) {
        v = row_sum16(v);
#pragma unroll
        for (int off = 16; off < WIDTH; off <<= 1) v += __shfl_xor(v, off);
    } else {
#pragma unroll
        for (int off = WIDTH / 2; off > 0; off >>= 1) v += __shfl_xor(v, off);
    }
    return v;
}

// Sum over the four lane quarters (lanes l, l^16, l^32, l^48).
__device__ inline double quarter_sum(double v)
{
    v += __shfl_xor(v, 16);
    v += __shfl_xor(v, 32);
    return v;
}

__device__ inline void push_record(DevReport* rep, int problem, int tm, int tn, int interval,
                                   int64_t row, int64_t col, int kind, double delta, double tau)
{
    unsigned int idx = atomicAdd(&rep->n_records, 1u);
    if (idx < rep->capacity) {
        ftg_fault_record r;
        r.problem = problem;
        r.tile_m = tm;
        r.tile_n = tn;
        r.interval = interval;
        r.row = row;
        r.col = col;
        r.kind = kind;
        r.reserved = 0;
        r.delta = delta;
        r.tau = tau;
        rep->records[idx] = r;
    }
}

__device__ inline void push_inject(DevReport* rep, int problem, int tm, int tn, int interval,
                                   int64_t row, int64_t col, int64_t pflip, int bit, int target,
                                   double oldv, double newv)
{
    atomicAdd(&rep->cnt[kInjected], 1ull);
    unsigned int idx = atomicAdd(&rep->n_inject, 1u);
    if (idx < rep->capacity) {
        ftg_inject_record r;
        r.problem = problem;
        r.tile_m = tm;
        r.tile_n = tn;
        r.interval = interval;
        r.row = row;
        r.col = col;
        r.pflip = pflip;
        r.bit = bit;
        r.target = target;
        r.old_val = oldv;
        r.new_val = newv;
        rep->inject_log[idx] = r;
    }
}

// Appends a repair request (one thread).  A full queue must not lose a fault
// silently: the slot is then counted and recorded as uncorrectable (its tile
// keeps what the kernel stored, or C_in for an unstored whole-tile request),
// rq_lost counts it, and the report read returns FTG_ERR_UNCORRECTED.
__device__ inline bool push_repair(DevReport* rep, const RepairReq& r)
{
    const unsigned int idx = atomicAdd(&rep->rq_count, 1u);
    if (idx < rep->rq_capacity) {
        rep->rq[idx] = r;
        return true;
    }
    atomicAdd(&rep->rq_lost, 1u);
    atomicAdd(&rep->cnt[kDetected], 1ull);
    atomicAdd(&rep->cnt[kUncorrectable], 1ull);
    push_record(rep, r.problem, r.tm, r.tn, r.interval, -1, -1, FTG_KIND_UNCORRECTABLE,
                r.nr ? r.dfi : r.dfj, r.nr ? r.tfi : r.tfj);
    return false;
}

// Workgroup id -> tile id.  Consecutive workgroup ids are spread round-robin
// over the 8 XCDs (each with its own L2); remap so that every XCD receives a
// contiguous range of the tile order, then walk tiles in groups of `group`
// tile rows so neighbouring tiles share A row panels and B column panels.
__device__ inline void tile_of_block(int bid, int nblocks, int tiles_m, int tiles_n, int group,
                                     int* tm, int* tn)
{
    int per = nblocks / 8;
    int t = bid;
    if (bid < per * 8) t = (bid % 8) * per + bid / 8;
    int width = group * tiles_n;
    int gid = t / width;
    int first = gid * group;
    int gsz = tiles_m - first < group ? tiles_m - first : group;
    int in = t % width;
    *tm = first + in % gsz;
    *tn = in / gsz;
}

}  // namespace ftg
