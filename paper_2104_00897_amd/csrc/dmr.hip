// Level-1 and Level-2 routines protected by duplicated computation (DMR),
// the scheme FT-BLAS applies to its memory-bound routines (§4): DSCAL,
// DNRM2, DGEMV and DTRSV.
//
// Every floating-point operation runs twice.  The second run works on copies
// of its operands that the compiler cannot prove equal to the originals, so
// it emits its own instructions.  The two results are compared bit for bit
// at every verification step: a group of 8 operations per lane (the paper
// compares once per unrolled iteration, §4.3).  A mismatch recomputes the
// step, twice, from the operands still held in registers (the paper's
// in-register checkpoint, §4.4) and compares again.  Agreement corrects the
// step (FTG_KIND_RECOMPUTE); a second mismatch is reported uncorrectable.
// Loads and stores are not duplicated: memory lies outside the sphere of
// replication (§4.1).  Reductions across lanes, waves and workgroups are
// duplicated and compared the same way.
//
// On MI355X these routines are bound by HBM bandwidth: a few flops per
// 8-byte element, against about 10 binary64 flops per byte that the vector
// units deliver at 8 TB/s.  So the duplicate fills issue slots that would
// otherwise idle (the argument of §4.2 for the CPU).
#include <hip/hip_runtime.h>
#include <limits.h>
#include <stdint.h>

#include <type_traits>

#include "ftg_common.hpp"
#include "ftg_kernels.hpp"

namespace ftg {

namespace {

constexpr int kThreads = 256;
constexpr int kU = 8;                  // operations per lane between two comparisons
constexpr int kVecStep = 64 * kU;      // DSCAL/DNRM2: elements per wave step
constexpr int kVecMaxBlocks = 2048;
constexpr int kGnRows = 64;            // DGEMV without transpose: rows per workgroup (one per lane)
constexpr int kGtCols = 4;             // DGEMV transposed: output elements per workgroup (one per wave)
constexpr int kGtStep = 64 * kU;       // DGEMV transposed: rows per wave step
constexpr int kGvTarget = 2048;        // DGEMV: workgroups aimed at per launch
constexpr int kTrsvB = 128;            // DTRSV: order of the diagonal blocks
constexpr int kTrsvLd = kTrsvB + 1;    // LDS leading dimension of a staged block

// Blue's scaling for binary64 (Blue, ACM TOMS 1978; thresholds as derived by
// Anderson, ACM TOMS 2017): the squares of magnitudes in [tsml, tbig]
// neither overflow nor lose accuracy to underflow.  Larger magnitudes are
// summed scaled by sbig, smaller ones by ssml (all powers of two, so the
// scaling is exact).
constexpr double kTsml = 0x1p-511, kTbig = 0x1p486, kSsml = 0x1p537, kSbig = 0x1p-538;

// A copy of x that the compiler cannot prove equal to x: an operation on it
// is issued again rather than shared with the same operation on x.
__device__ __forceinline__ double dup(double x)
{
    asm volatile("" : "+v"(x));
    return x;
}

__device__ __forceinline__ bool differ(double a, double b)
{
    return __double_as_longlong(a) != __double_as_longlong(b);
}

template <typename T>
__host__ __device__ __forceinline__ T imin(T a, T b) { return a < b ? a : b; }

// First planned step after `after` whose fault belongs to thread `owner`.
__device__ __forceinline__ int next_fault(const DmrPlan& p, int64_t owner, int after)
{
    int best = INT_MAX;
    for (int q = 0; q < p.n; ++q)
        if (p.f[q].owner == owner && p.f[q].step > after && p.f[q].step < best) best = p.f[q].step;
    return best;
}

// Flips the planned bit of the step's first result (FTG_TARGET_ACC and
// FTG_TARGET_TWO_IN_SLOT) or of its duplicate (FTG_TARGET_CHECKSUM) and logs
// it when `log`.  Returns the bit to flip again in the recomputation (the
// fault persists under FTG_TARGET_TWO_IN_SLOT), else -1.
__device__ __forceinline__ int apply_fault(const DmrPlan& p, const DmrFault& f, double& v1, double& v2, DevReport* rep, bool log,
                           int tm, int64_t row, int64_t col, int step)
{
    double old, now;
    if (p.target == FTG_TARGET_CHECKSUM) {
        old = v2;
        v2 = flip_f64(v2, f.bit);
        now = v2;
    } else {
        old = v1;
        v1 = flip_f64(v1, f.bit);
        now = v1;
    }
    if (log) push_inject(rep, 0, tm, -1, step, row, col, step, f.bit, p.target, old, now);
    return p.target == FTG_TARGET_TWO_IN_SLOT ? f.bit : -1;
}

// Counts and records a detected mismatch: corrected by the recomputation
// (`fixed`) or not.  delta: the difference of the two mismatching copies.
__device__ void note_repair(DevReport* rep, bool fixed, int tm, int64_t row, int64_t col, int step, double a,
                            double b)
{
    atomicAdd(&rep->cnt[kDetected], 1ull);
    atomicAdd(&rep->cnt[fixed ? kCorrRecomp : kUncorrectable], 1ull);
    push_record(rep, 0, tm, -1, step, row, col, fixed ? FTG_KIND_RECOMPUTE : FTG_KIND_UNCORRECTABLE, a - b, 0.0);
}

// ------------------------------------------------------------------ DSCAL
// Wave w takes the runs of 512 elements w, w + nwaves, ...; lane l of a run
// starting at c0 holds the 8 elements vec_elem(c0, l, s), s < 8: elements
// 64 apart, each access of a wave a coalesced 512-byte run; or (V2, DNRM2 on
// a contiguous, 16-byte aligned x) pairs of neighbours 128 apart, each access
// a 1 KB run of 16-byte pieces.  Measured, DNRM2 reads faster in pairs and
// DSCAL (which also writes) one element at a time.

template <bool V2>
__device__ __forceinline__ int64_t vec_elem(int64_t c0, int lane, int s)
{
    return V2 ? c0 + 128 * (s >> 1) + 2 * lane + (s & 1) : c0 + lane + 64 * s;
}

template <bool UNIT, bool V2>
__device__ __forceinline__ void vec_load(const double* __restrict__ x, int64_t n, int64_t inc, int64_t c0, int lane,
                                         double* v)
{
    if (V2 && c0 + kVecStep <= n) {
#pragma unroll
        for (int u = 0; u < kU / 2; ++u) {
            const double2 p = *reinterpret_cast<const double2*>(x + c0 + 128 * u + 2 * lane);
            v[2 * u] = p.x;
            v[2 * u + 1] = p.y;
        }
    } else {
#pragma unroll
        for (int s = 0; s < kU; ++s) {
            const int64_t i = vec_elem<V2>(c0, lane, s);
            v[s] = i < n ? x[UNIT ? i : i * inc] : 0.0;
        }
    }
}

template <bool UNIT, bool V2>
__device__ __forceinline__ void vec_store(double* __restrict__ x, int64_t n, int64_t inc, int64_t c0, int lane,
                                          const double* v)
{
    if (V2 && c0 + kVecStep <= n) {
#pragma unroll
        for (int u = 0; u < kU / 2; ++u)
            *reinterpret_cast<double2*>(x + c0 + 128 * u + 2 * lane) = make_double2(v[2 * u], v[2 * u + 1]);
    } else {
#pragma unroll
        for (int s = 0; s < kU; ++s) {
            const int64_t i = vec_elem<V2>(c0, lane, s);
            if (i < n) x[UNIT ? i : i * inc] = v[s];
        }
    }
}

// Planned faults of one step of one lane, packed 7 bits per element u (bit
// 6: a fault; bits 0..5: the bit to flip).
__device__ __forceinline__ uint64_t step_faults(const DmrPlan& p, int64_t me, int step)
{
    uint64_t pk = 0;
    for (int q = 0; q < p.n; ++q)
        if (p.f[q].owner == me && p.f[q].step == step) pk |= (uint64_t)(64 | p.f[q].bit) << (7 * p.f[q].sub);
    return pk;
}

// A DSCAL step that leaves the common path -- planned faults, or a
// mismatch there -- done again from memory (x is not yet overwritten):
// product and duplicate of each element, the planned flips, comparison,
// recomputation of a mismatching element, records, stores.  Out of line, so
// that the common path keeps few registers.  Returns the mismatches found.
template <bool UNIT>
__device__ __noinline__ int scal_slow_step(double* __restrict__ x, int64_t n, int64_t inc, double alpha, int64_t c0,
                                           int lane, int step, uint64_t pk, int target, DevReport* rep)
{
    int found = 0;
#pragma unroll 1
    for (int u = 0; u < kU; ++u) {
        const int64_t i = vec_elem<false>(c0, lane, u);
        if (i >= n) break;
        const double v = x[UNIT ? i : i * inc];
        double r = alpha * v, d = alpha * dup(v);
        int again = -1;
        const int fb = (int)((pk >> (7 * u)) & 127);
        if (fb & 64) {
            DmrPlan one;
            one.target = target;
            DmrFault f;
            f.bit = fb & 63;
            again = apply_fault(one, f, r, d, rep, true, -1, i, -1, step);
        }
        if (differ(r, d)) {
            double r1 = alpha * dup(v);
            const double r2 = alpha * dup(v);
            if (again >= 0) r1 = flip_f64(r1, again);
            note_repair(rep, !differ(r1, r2), -1, i, -1, step, r, d);
            r = r1;
            ++found;
        }
        x[UNIT ? i : i * inc] = r;
    }
    return found;
}

template <bool DMR, bool UNIT, bool V2>
__global__ __launch_bounds__(kThreads) void scal_kernel(double* __restrict__ x, int64_t n, int64_t inc,
                                                        double alpha, int64_t nwaves, DmrPlan plan,
                                                        DevReport* rep)
{
    const int lane = threadIdx.x & 63;
    const int64_t w = (int64_t)blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6);
    const int64_t me = w * 64 + lane;
    const int64_t stride = nwaves * kVecStep;
    int next = INT_MAX;
    if (DMR && plan.n) next = next_fault(plan, me, -1);
    // protected: the next step's elements are loaded before this step's are
    // checked, scaled and stored, so every wave keeps loads in flight while it
    // works (measured: 3% faster protected, 4% slower unprotected, which
    // therefore loads each step at its start)
    constexpr bool PF = DMR;
    double v[kU];
    if (PF && w * kVecStep < n) vec_load<UNIT, V2>(x, n, inc, w * kVecStep, lane, v);
    int step = 0;
    for (int64_t c0 = w * kVecStep; c0 < n; c0 += stride, ++step) {
        double vn[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) vn[u] = 0.0;
        if (PF && c0 + stride < n) vec_load<UNIT, V2>(x, n, inc, c0 + stride, lane, vn);
        if (!PF) vec_load<UNIT, V2>(x, n, inc, c0, lane, v);
        if (DMR && step == next) {
            const uint64_t pk = step_faults(plan, me, step);
            next = next_fault(plan, me, step);
            scal_slow_step<UNIT>(x, n, inc, alpha, c0, lane, step, pk, plan.target, rep);
        } else {
            double r[kU];
#pragma unroll
            for (int u = 0; u < kU; ++u) r[u] = alpha * v[u];
            bool bad = false;
            if constexpr (DMR) {
                // each product against its duplicate, as it is formed
#pragma unroll
                for (int u = 0; u < kU; ++u) bad |= differ(r[u], alpha * dup(v[u]));
                if (bad) {
                    // a mismatch that the step's recomputation does not show again was
                    // transient: the recomputed (stored) values are the corrected ones
                    if (scal_slow_step<UNIT>(x, n, inc, alpha, c0, lane, step, 0, 0, rep) == 0)
                        note_repair(rep, true, -1, vec_elem<false>(c0, lane, 0), -1, step, 0.0, 0.0);
                }
            }
            if (!bad) vec_store<UNIT, V2>(x, n, inc, c0, lane, r);
        }
        if (PF) {
#pragma unroll
            for (int u = 0; u < kU; ++u) v[u] = vn[u];
        }
    }
}

// ------------------------------------------------------------------ DNRM2
// Sums of squares of the small, medium and big elements (Blue's scaling).
struct Sq3 {
    double s, m, b;
};

__device__ __forceinline__ int sq_class(double v)
{
    const double ax = fabs(v);
    return ax > kTbig ? 2 : (ax < kTsml ? 0 : 1);  // NaN: medium
}

__device__ __forceinline__ void sq_add(double v, Sq3& a)
{
    const double ax = fabs(v);
    const bool big = ax > kTbig, sml = ax < kTsml;
    const double y = v * (big ? kSbig : (sml ? kSsml : 1.0));
    const double t = fma(y, y, big ? a.b : (sml ? a.s : a.m));
    a.b = big ? t : a.b;
    a.s = sml ? t : a.s;
    a.m = (big || sml) ? a.m : t;
}

__device__ __forceinline__ bool differ3(const Sq3& a, const Sq3& b)
{
    return differ(a.s, b.s) | differ(a.m, b.m) | differ(a.b, b.b);
}

__device__ __forceinline__ Sq3 dup3(const Sq3& a) { return Sq3{dup(a.s), dup(a.m), dup(a.b)}; }

__device__ __forceinline__ Sq3 wave_sum3(const Sq3& a)
{
    return Sq3{group_sum<64>(a.s), group_sum<64>(a.m), group_sum<64>(a.b)};
}

__device__ __forceinline__ Sq3 add3(const Sq3& a, const Sq3& b) { return Sq3{a.s + b.s, a.m + b.m, a.b + b.b}; }

// Flips bit `bit` of the accumulator of class `cls`.
__device__ __forceinline__ void flip3(Sq3& a, int cls, int bit)
{
    if (cls == 0) a.s = flip_f64(a.s, bit);
    else if (cls == 1) a.m = flip_f64(a.m, bit);
    else a.b = flip_f64(a.b, bit);
}

// The norm from the three sums (the combination step of Blue's algorithm).
__device__ double sq_norm(const Sq3& a)
{
    if (a.b > 0.0) {
        double b = a.b;
        if (a.m > 0.0 || a.m != a.m) b = b + (a.m * kSbig) * kSbig;
        return sqrt(b) * 0x1p538;  // 1 / sbig
    }
    if (a.s > 0.0) {
        if (a.m > 0.0 || a.m != a.m) {
            const double ym = sqrt(a.m), ys = sqrt(a.s) * 0x1p-537;  // 1 / ssml
            const double lo = ys > ym ? ym : ys, hi = ys > ym ? ys : ym;
            const double q = lo / hi;
            return sqrt(hi * hi * (1.0 + q * q));
        }
        return sqrt(a.s) * 0x1p-537;
    }
    return sqrt(a.m);
}

// Workgroup sums of the three accumulators (duplicated across lanes, then
// across the four waves); thread 0 gets the result.
template <bool DMR>
__device__ Sq3 block_sum3(Sq3 a1, Sq3 a2, DevReport* rep, int step)
{
    __shared__ double red[kThreads / 64][3];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    Sq3 t1 = wave_sum3(a1);
    if constexpr (DMR) {
        const Sq3 t2 = wave_sum3(dup3(a2));
        if (differ3(t1, t2)) {
            const Sq3 r1 = wave_sum3(dup3(a1)), r2 = wave_sum3(dup3(a1));
            if (lane == 0) note_repair(rep, !differ3(r1, r2), -1, -1, -1, step, t1.m, t2.m);
            t1 = r1;
        }
    }
    if (lane == 0) {
        red[wv][0] = t1.s;
        red[wv][1] = t1.m;
        red[wv][2] = t1.b;
    }
    __syncthreads();
    Sq3 b1{0.0, 0.0, 0.0};
    if (threadIdx.x == 0) {
        for (int q = 0; q < kThreads / 64; ++q) b1 = add3(b1, Sq3{red[q][0], red[q][1], red[q][2]});
        if constexpr (DMR) {
            Sq3 b2{0.0, 0.0, 0.0};
            for (int q = 0; q < kThreads / 64; ++q) b2 = add3(b2, dup3(Sq3{red[q][0], red[q][1], red[q][2]}));
            if (differ3(b1, b2)) {
                Sq3 r1{0.0, 0.0, 0.0}, r2{0.0, 0.0, 0.0};
                for (int q = 0; q < kThreads / 64; ++q) {
                    r1 = add3(r1, dup3(Sq3{red[q][0], red[q][1], red[q][2]}));
                    r2 = add3(r2, dup3(Sq3{red[q][0], red[q][1], red[q][2]}));
                }
                note_repair(rep, !differ3(r1, r2), -1, -1, -1, step, b1.m, b2.m);
                b1 = r1;
            }
        }
    }
    return b1;
}

struct Sq3N {
    Sq3 a;
    int found;
};

// A DNRM2 step that leaves the common path (planned faults, or a mismatch
// there), done again from memory starting from the verified sums `chk`:
// both copies, the planned flips (of the sum that took the element),
// comparison, recomputation of both copies from chk on a mismatch, record.
// Returns the step's sums and the mismatches found.  Out of line, so that
// the common path keeps few registers.
template <bool UNIT, bool V2>
__device__ __noinline__ Sq3N nrm2_slow_step(const double* __restrict__ x, int64_t n, int64_t inc, int64_t c0,
                                            int lane, int step, Sq3 chk, uint64_t pk, int target, DevReport* rep)
{
    // one element at a time, reloaded where needed: few registers
    auto at = [&](int u) {
        const int64_t i = vec_elem<V2>(c0, lane, u);
        return i < n ? x[UNIT ? i : i * inc] : 0.0;
    };
    Sq3 a1 = chk, a2 = chk;
#pragma unroll 1
    for (int u = 0; u < kU; ++u) {
        const double v = at(u);
        sq_add(v, a1);
        sq_add(dup(v), a2);
    }
    int again = -1, again_cls = 0;
#pragma unroll 1
    for (int u = 0; u < kU; ++u) {
        const int fb = (int)((pk >> (7 * u)) & 127);
        if (!(fb & 64)) continue;
        const int cls = sq_class(at(u));  // the sum that took the element
        double t1 = cls == 0 ? a1.s : (cls == 1 ? a1.m : a1.b);
        double t2 = cls == 0 ? a2.s : (cls == 1 ? a2.m : a2.b);
        DmrPlan one;
        one.target = target;
        DmrFault f;
        f.bit = fb & 63;
        const int g = apply_fault(one, f, t1, t2, rep, true, -1, vec_elem<V2>(c0, lane, u), -1, step);
        if (cls == 0) {
            a1.s = t1;
            a2.s = t2;
        } else if (cls == 1) {
            a1.m = t1;
            a2.m = t2;
        } else {
            a1.b = t1;
            a2.b = t2;
        }
        if (g >= 0) {
            again = g;
            again_cls = cls;
        }
    }
    Sq3N out{a1, 0};
    if (differ3(a1, a2)) {
        Sq3 r1 = chk, r2 = chk;
#pragma unroll 1
        for (int u = 0; u < kU; ++u) {
            const double v = at(u);
            sq_add(dup(v), r1);
            sq_add(dup(v), r2);
        }
        if (again >= 0) flip3(r1, again_cls, again);
        note_repair(rep, !differ3(r1, r2), -1, vec_elem<V2>(c0, lane, 0), -1, step, a1.s + a1.m + a1.b,
                    a2.s + a2.m + a2.b);
        out.a = r1;
        out.found = 1;
    }
    return out;
}

// Per-workgroup sums of squares of the elements (same element order as
// DSCAL), three doubles per workgroup into part.
template <bool DMR, bool UNIT, bool V2>
__global__ __launch_bounds__(kThreads) void nrm2_part_kernel(const double* __restrict__ x, int64_t n, int64_t inc,
                                                             int64_t nwaves, double* __restrict__ part,
                                                             DmrPlan plan, DevReport* rep)
{
    const int lane = threadIdx.x & 63;
    const int64_t w = (int64_t)blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6);
    const int64_t me = w * 64 + lane;
    int next = INT_MAX;
    if (DMR && plan.n) next = next_fault(plan, me, -1);
    Sq3 a1{0.0, 0.0, 0.0}, a2{0.0, 0.0, 0.0};
    // protected: the next step's elements are loaded before this step's are
    // added (as in DSCAL), so loads stay in flight while the duplicated sums run
    constexpr bool PF = DMR;
    const int64_t stride = nwaves * kVecStep;
    double v[kU];
    if (PF && w * kVecStep < n) vec_load<UNIT, V2>(x, n, inc, w * kVecStep, lane, v);
    int step = 0;
    for (int64_t c0 = w * kVecStep; c0 < n; c0 += stride, ++step) {
        double vn[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) vn[u] = 0.0;
        if (PF && c0 + stride < n) vec_load<UNIT, V2>(x, n, inc, c0 + stride, lane, vn);
        if (DMR && step == next) {
            const uint64_t pk = step_faults(plan, me, step);
            next = next_fault(plan, me, step);
            a1 = nrm2_slow_step<UNIT, V2>(x, n, inc, c0, lane, step, a1, pk, plan.target, rep).a;
            a2 = a1;
#pragma unroll
            for (int u = 0; u < kU; ++u) v[u] = vn[u];
            continue;
        }
        if (!PF) vec_load<UNIT, V2>(x, n, inc, c0, lane, v);
        const Sq3 chk = a1;
#pragma unroll
        for (int u = 0; u < kU; ++u) sq_add(v[u], a1);
        if constexpr (DMR) {
#pragma unroll
            for (int u = 0; u < kU; ++u) sq_add(dup(v[u]), a2);
            if (differ3(a1, a2)) {
                const Sq3N r = nrm2_slow_step<UNIT, V2>(x, n, inc, c0, lane, step, chk, 0, 0, rep);
                // not seen again by the recomputation: a transient mismatch, corrected by it
                if (r.found == 0) note_repair(rep, true, -1, vec_elem<V2>(c0, lane, 0), -1, step, 0.0, 0.0);
                a1 = r.a;
                a2 = r.a;
            }
        }
        if (PF) {
#pragma unroll
            for (int u = 0; u < kU; ++u) v[u] = vn[u];
        }
    }
    const Sq3 b = block_sum3<DMR>(a1, a2, rep, -1);
    if (threadIdx.x == 0) {
        part[3 * blockIdx.x + 0] = b.s;
        part[3 * blockIdx.x + 1] = b.m;
        part[3 * blockIdx.x + 2] = b.b;
    }
}

// Sums the workgroups' partial sums and forms the norm (one workgroup).
template <bool DMR>
__global__ __launch_bounds__(kThreads) void nrm2_final_kernel(const double* __restrict__ part, int nparts,
                                                              double* __restrict__ out, DevReport* rep)
{
    Sq3 a1{0.0, 0.0, 0.0}, a2{0.0, 0.0, 0.0};
    for (int p = threadIdx.x; p < nparts; p += kThreads) {
        const Sq3 v{part[3 * p], part[3 * p + 1], part[3 * p + 2]};
        a1 = add3(a1, v);
        if constexpr (DMR) a2 = add3(a2, dup3(v));
    }
    if constexpr (DMR) {
        if (differ3(a1, a2)) {
            Sq3 r1{0.0, 0.0, 0.0}, r2{0.0, 0.0, 0.0};
            for (int p = threadIdx.x; p < nparts; p += kThreads) {
                const Sq3 v{part[3 * p], part[3 * p + 1], part[3 * p + 2]};
                r1 = add3(r1, dup3(v));
                r2 = add3(r2, dup3(v));
            }
            note_repair(rep, !differ3(r1, r2), -1, -1, -1, -1, a1.m, a2.m);
            a1 = r1;
            a2 = r1;
        }
    }
    const Sq3 b = block_sum3<DMR>(a1, a2, rep, -1);
    if (threadIdx.x == 0) {
        double r = sq_norm(b);
        if constexpr (DMR) {
            const double r2 = sq_norm(dup3(b));
            if (differ(r, r2)) {
                const double q1 = sq_norm(dup3(b)), q2 = sq_norm(dup3(b));
                note_repair(rep, !differ(q1, q2), -1, -1, -1, -1, r, r2);
                r = q1;
            }
        }
        *out = r;
    }
}

// ------------------------------------------------------------------ DGEMV
// One launch over a stored panel of A.  Without transpose (gemv_n_kernel)
// the panel is rows x cols with rows the output elements; transposed
// (gemv_t_kernel) it is rows x cols with cols the outputs.  The reduction
// dimension is cut into chunks of `width`; with one chunk the launch writes
// y := alpha s + beta y, otherwise every chunk's sums go to part[c ldp + i]
// and gemv_reduce_kernel finishes.
struct Gv {
    const double* A;
    int64_t lda;
    int64_t rows, cols;
    const double* x;  // element 0 of the reduction vector
    int64_t incx;
    double* y;        // element 0 of the output vector
    int64_t incy;
    double alpha, beta;
    double* part;
    int64_t ldp;
    int64_t width;    // chunk width along the reduction
    int64_t bout;     // workgroups along the outputs
    int direct;       // 1: write y; 0: write partial sums
    DevReport* rep;
};

__device__ __forceinline__ double axpby(double alpha, double t, double beta, double yv)
{
    return beta == 0.0 ? alpha * t : fma(alpha, t, beta * yv);
}

template <bool DMR>
__device__ double out_value(const Gv& g, double t, double yv, int64_t row)
{
    double o1 = axpby(g.alpha, t, g.beta, yv);
    if constexpr (DMR) {
        const double o2 = axpby(g.alpha, dup(t), g.beta, dup(yv));
        if (differ(o1, o2)) {
            const double r1 = axpby(g.alpha, dup(t), g.beta, dup(yv));
            const double r2 = axpby(g.alpha, dup(t), g.beta, dup(yv));
            note_repair(g.rep, !differ(r1, r2), -1, row, -1, -1, o1, o2);
            o1 = r1;
        }
    }
    return o1;
}

// y_i := alpha sum_j A(i, j) x_j + beta y_i.  Workgroup (rb, c): rows
// rb*64 + lane, one per lane; wave wv takes a quarter of chunk c's columns,
// 8 columns per step (8 coalesced 512-byte column segments in flight per
// wave); the four waves' sums meet in LDS.
template <bool DMR, bool XUNIT>
__global__ __launch_bounds__(kThreads) void gemv_n_kernel(Gv g, DmrPlan plan)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t rb = blockIdx.x % g.bout, c = blockIdx.x / g.bout;
    const int64_t i = rb * kGnRows + lane;
    const bool valid = i < g.rows;
    const int64_t wcols = g.width / 4;
    const int64_t j0w = c * g.width + wv * wcols;
    const int64_t j1w = imin(g.cols, j0w + wcols);
    const double* Ai = g.A + (valid ? i : 0);  // lanes past the last row read row 0 and store nothing
    const int64_t me = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    int next = INT_MAX;
    if (DMR && plan.n) next = next_fault(plan, me, -1);
    double acc1 = 0.0, acc2 = 0.0;
    int step = 0;
    for (int64_t j0 = j0w; j0 < j1w; j0 += kU, ++step) {
        const int64_t cnt = j1w - j0;
        double a[kU], xv[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const bool in = u < cnt;
            const int64_t j = in ? j0 + u : j0;
            const double av = Ai[j * g.lda];
            const double xx = XUNIT ? g.x[j] : g.x[j * g.incx];
            a[u] = in ? av : 0.0;
            xv[u] = in ? xx : 0.0;
        }
        const double chk = acc1;
#pragma unroll
        for (int u = 0; u < kU; ++u) acc1 = fma(a[u], xv[u], acc1);
        if constexpr (DMR) {
#pragma unroll
            for (int u = 0; u < kU; ++u) acc2 = fma(dup(a[u]), xv[u], acc2);
            int again = -1;
            if (step == next) {
                for (int q = 0; q < plan.n; ++q) {
                    const DmrFault f = plan.f[q];
                    if (f.owner == me && f.step == step)
                        again = apply_fault(plan, f, acc1, acc2, g.rep, true, -1, i, j0, step);
                }
                next = next_fault(plan, me, step);
            }
            if (differ(acc1, acc2)) {
                double r1 = chk, r2 = chk;
#pragma unroll
                for (int u = 0; u < kU; ++u) r1 = fma(dup(a[u]), xv[u], r1);
#pragma unroll
                for (int u = 0; u < kU; ++u) r2 = fma(dup(a[u]), xv[u], r2);
                if (again >= 0) r1 = flip_f64(r1, again);
                note_repair(g.rep, !differ(r1, r2), -1, i, j0, step, acc1, acc2);
                acc1 = r1;
                acc2 = r1;
            }
        }
    }
    __shared__ double red[kThreads];
    red[threadIdx.x] = acc1;
    __syncthreads();
    if (wv != 0) return;
    double t1 = ((red[lane] + red[64 + lane]) + red[128 + lane]) + red[192 + lane];
    if constexpr (DMR) {
        const double t2 = ((dup(red[lane]) + dup(red[64 + lane])) + dup(red[128 + lane])) + dup(red[192 + lane]);
        if (differ(t1, t2)) {
            const double r1 = ((dup(red[lane]) + dup(red[64 + lane])) + dup(red[128 + lane])) + dup(red[192 + lane]);
            const double r2 = ((dup(red[lane]) + dup(red[64 + lane])) + dup(red[128 + lane])) + dup(red[192 + lane]);
            note_repair(g.rep, !differ(r1, r2), -1, i, -1, -1, t1, t2);
            t1 = r1;
        }
    }
    if (!valid) return;
    if (!g.direct) {
        g.part[c * g.ldp + i] = t1;
        return;
    }
    const double yv = g.beta != 0.0 ? g.y[i * g.incy] : 0.0;
    g.y[i * g.incy] = out_value<DMR>(g, t1, yv, i);
}

// y_j := alpha sum_i A(i, j) x_i + beta y_j.  Workgroup (jb, c): wave wv
// computes output jb*4 + wv over chunk c's rows; lane l of a step starting
// at r0 adds rows r0 + l + 64 u (u < 8), then the wave's lanes are summed.
template <bool DMR, bool XUNIT>
__global__ __launch_bounds__(kThreads) void gemv_t_kernel(Gv g, DmrPlan plan)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t jb = blockIdx.x % g.bout, c = blockIdx.x / g.bout;
    const int64_t j = jb * kGtCols + wv;
    if (j >= g.cols) return;  // whole waves; no barrier follows
    const int64_t r0w = c * g.width, r1w = imin(g.rows, r0w + g.width);
    const double* Aj = g.A + j * g.lda;
    const int64_t me = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    int next = INT_MAX;
    if (DMR && plan.n) next = next_fault(plan, me, -1);
    double acc1 = 0.0, acc2 = 0.0;
    int step = 0;
    for (int64_t r0 = r0w; r0 < r1w; r0 += kGtStep, ++step) {
        double a[kU], xv[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const int64_t ii = r0 + lane + 64 * u;
            const bool in = ii < r1w;
            const int64_t ic = in ? ii : r0w;
            const double av = Aj[ic];
            const double xx = XUNIT ? g.x[ic] : g.x[ic * g.incx];
            a[u] = in ? av : 0.0;
            xv[u] = in ? xx : 0.0;
        }
        const double chk = acc1;
#pragma unroll
        for (int u = 0; u < kU; ++u) acc1 = fma(a[u], xv[u], acc1);
        if constexpr (DMR) {
#pragma unroll
            for (int u = 0; u < kU; ++u) acc2 = fma(dup(a[u]), xv[u], acc2);
            int again = -1;
            if (step == next) {
                for (int q = 0; q < plan.n; ++q) {
                    const DmrFault f = plan.f[q];
                    if (f.owner == me && f.step == step)
                        again = apply_fault(plan, f, acc1, acc2, g.rep, true, -1, r0 + lane, j, step);
                }
                next = next_fault(plan, me, step);
            }
            if (differ(acc1, acc2)) {
                double r1 = chk, r2 = chk;
#pragma unroll
                for (int u = 0; u < kU; ++u) r1 = fma(dup(a[u]), xv[u], r1);
#pragma unroll
                for (int u = 0; u < kU; ++u) r2 = fma(dup(a[u]), xv[u], r2);
                if (again >= 0) r1 = flip_f64(r1, again);
                note_repair(g.rep, !differ(r1, r2), -1, r0 + lane, j, step, acc1, acc2);
                acc1 = r1;
                acc2 = r1;
            }
        }
    }
    double t1 = group_sum<64>(acc1);
    if constexpr (DMR) {
        const double t2 = group_sum<64>(dup(acc2));
        if (differ(t1, t2)) {
            const double r1 = group_sum<64>(dup(acc1));
            const double r2 = group_sum<64>(dup(acc1));
            if (lane == 0) note_repair(g.rep, !differ(r1, r2), -1, -1, j, -1, t1, t2);
            t1 = r1;
        }
    }
    if (lane != 0) return;
    if (!g.direct) {
        g.part[c * g.ldp + j] = t1;
        return;
    }
    const double yv = g.beta != 0.0 ? g.y[j * g.incy] : 0.0;
    g.y[j * g.incy] = out_value<DMR>(g, t1, yv, j);
}

// y_i := alpha sum_c part[c ldp + i] + beta y_i over the chunks.
template <bool DMR>
__global__ __launch_bounds__(kThreads) void gemv_reduce_kernel(Gv g, int64_t len, int64_t nparts)
{
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i >= len) return;
    double t1 = 0.0, t2 = 0.0;
    for (int64_t c = 0; c < nparts; ++c) {
        const double p = g.part[c * g.ldp + i];
        t1 += p;
        if constexpr (DMR) t2 += dup(p);
    }
    if constexpr (DMR) {
        if (differ(t1, t2)) {
            double r1 = 0.0, r2 = 0.0;
            for (int64_t c = 0; c < nparts; ++c) {
                const double p = g.part[c * g.ldp + i];
                r1 += dup(p);
                r2 += dup(p);
            }
            note_repair(g.rep, !differ(r1, r2), -1, i, -1, -1, t1, t2);
            t1 = r1;
        }
    }
    const double yv = g.beta != 0.0 ? g.y[i * g.incy] : 0.0;
    g.y[i * g.incy] = out_value<DMR>(g, t1, yv, i);
}

// ------------------------------------------------------------------ DTRSV
// Blocked DTRSV (§3.2: the update by the solved part is a DGEMV, the small
// diagonal part a substitution) in one launch: one workgroup per block of
// 128 rows, taken in solve order from a ticket counter.  Workgroup q
//   - stages its block's triangle of op(A) in LDS;
//   - for every block j solved before it, in solve order, loads its part of
//     the block row of op(A) against block j (the loads leave before the
//     wait), waits until block j is published, reads x_j and adds the
//     products (duplicated, compared every 8 multiply-adds);
//   - forms the right-hand side x_i - sum and substitutes (below);
//   - writes its unknowns, then publishes them (release fence, flag store).
// Tickets follow the order in which workgroups start, so every block a
// workgroup waits for belongs to a workgroup already running, and no wait
// can keep its producer from running.  Waits are bounded all the same: one
// that runs out records an uncorrectable fault and goes on, so every
// workgroup ends.
//
// Substitution (wave 0, two rows per lane): x_k = r_k / a_kk -- a
// multiplication by the reciprocal formed while staging, as the paper's
// packing stores them (§3.3.3) -- then every row takes the term a_ik x_k.
// Both copies run side by side and x_k is compared as it is formed.  A
// mismatch recomputes r_k from the staged right-hand side and the unknowns
// solved so far, in the order of the original updates, so a corrected x_k
// is bitwise the one a fault-free run forms.
struct Tc {
    const double* A;
    int64_t lda;
    double* x;             // element 0
    int64_t incx;
    int64_t n;
    int nblk;
    int lower, trans, unit;
    unsigned int* sync;    // [0] ticket counter, [1 + b] block b published (zeroed before the launch)
    int spin_limit;
    DevReport* rep;
};

__device__ __forceinline__ double readlane_f64(double v, int l)
{
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
    return __hiloint2double(hi, lo);
}

// The block's triangle of op(A) into M[k kTrsvLd + i] = op(A)(r0 + i, r0 + k)
// (0 outside the triangle and past nb; 1 on a unit diagonal, not read), 16
// loads in flight per thread, consecutive threads reading consecutive
// elements of a column of A.
__device__ __forceinline__ void stage_tri(double* M, const Tc& t, int64_t r0, int nb)
{
    constexpr int kBatch = 16;
    for (int e0 = 0; e0 < kTrsvB * kTrsvB; e0 += kThreads * kBatch) {
        double v[kBatch];
#pragma unroll
        for (int b = 0; b < kBatch; ++b) {
            const int e = e0 + b * kThreads + (int)threadIdx.x;
            const int i = t.trans ? e / kTrsvB : e % kTrsvB;
            const int k = t.trans ? e % kTrsvB : e / kTrsvB;
            const bool tri = i < nb && k < nb && (t.lower ? i >= k : i <= k);
            const bool one = tri && i == k && t.unit;
            v[b] = one ? 1.0 : 0.0;
            if (tri && !one) v[b] = t.trans ? t.A[(r0 + k) + (r0 + i) * t.lda] : t.A[(r0 + i) + (r0 + k) * t.lda];
        }
#pragma unroll
        for (int b = 0; b < kBatch; ++b) {
            const int e = e0 + b * kThreads + (int)threadIdx.x;
            const int i = t.trans ? e / kTrsvB : e % kTrsvB;
            const int k = t.trans ? e % kTrsvB : e / kTrsvB;
            M[k * kTrsvLd + i] = v[b];
        }
    }
}

// Wave 0: solves the staged block for the right-hand side rhs (reciprocal
// diagonal dr) and writes the unknowns to x.  Lane l holds rows l and l + 64
// (halves 0 and 1).  The solve runs as two phases, one per half in solve
// order (a lower block solves half 0 first, an upper one half 1); in the
// first phase the other half's rows take every term too, in the second they
// are done.  A step is a multiply, a broadcast (readlane) and one or two
// multiply-adds per lane.  Steps go in unrolled chunks of 16 whose columns of
// M sit in registers (the next chunk's are read while a chunk runs); a
// chunk's unknowns reach LDS together at its end.  The chunk loop itself is
// not unrolled: it runs once per block, on a cold instruction cache.
template <bool DMR>
__device__ __forceinline__ void substitute(const double* M, const double* rhs, const double* dr, double* xs,
                                           const Tc& t, int64_t r0, int nb, int block, const DmrPlan& plan)
{
    const int lane = threadIdx.x;
    double r1[2] = {rhs[lane], rhs[lane + 64]};
    double r2[2] = {r1[0], r1[1]};
    const double d[2] = {dr[lane], dr[lane + 64]};
    // rows of this block with a planned substitution fault (bit k of fm[k / 64])
    uint64_t fm[2] = {0, 0};
    if constexpr (DMR) {
        for (int f = 0; f < plan.n; ++f)
            if (plan.f[f].owner == block && plan.f[f].sub == 1) fm[plan.f[f].step >> 6] |= 1ull << (plan.f[f].step & 63);
    }
    auto col = [&](int q) { return t.lower ? q : nb - 1 - q; };  // row solved at step q
    constexpr int kStep = 16;
    int done = 0;  // steps before the phase
    auto phase = [&](auto hc, auto oc) __attribute__((always_inline)) {
        constexpr int H = decltype(hc)::value;    // the half solved in this phase
        constexpr bool UO = decltype(oc)::value;  // the other half still takes terms
        const int nh = nb - 64 * H < 0 ? 0 : (nb - 64 * H > 64 ? 64 : nb - 64 * H);
        auto krow = [&](int i) { return t.lower ? 64 * H + i : 64 * H + nh - 1 - i; };  // row of the phase's step i
        double mh[kStep], mo[kStep];
        auto load_chunk = [&](int i0, double* a, double* b) __attribute__((always_inline)) {
#pragma unroll
            for (int j = 0; j < kStep; ++j) {
                const int kj = krow(i0 + j < nh ? i0 + j : nh - 1);
                a[j] = M[kj * kTrsvLd + lane + 64 * H];
                if (UO) b[j] = M[kj * kTrsvLd + lane + 64 * (1 - H)];
            }
        };
        if (nh > 0) load_chunk(0, mh, mo);
        for (int i0 = 0; i0 < nh; i0 += kStep) {
            double nmh[kStep], nmo[kStep];
            load_chunk(i0 + kStep < nh ? i0 + kStep : i0, nmh, nmo);
            double xv[kStep];
            // the chunk's steps compare the two copies of each unknown into one
            // flag, checked at the chunk's end (a branch per step would
            // serialise the two copies); a flagged chunk is done again from the
            // rows as they were at its start
            const double ck0 = r1[0], ck1 = r1[1];
            bool bad = false;
            uint32_t planned = 0;  // steps of the chunk with a planned fault (bit j)
#pragma unroll
            for (int j = 0; j < kStep; ++j) {
                xv[j] = 0.0;
                if (i0 + j >= nh) continue;  // uniform
                const int k = krow(i0 + j);
                double x1 = readlane_f64(r1[H] * d[H], k & 63);
                if constexpr (DMR) {
                    double x2 = readlane_f64(r2[H] * dup(d[H]), k & 63);
                    if ((fm[H] >> (k & 63)) & 1) {
                        planned |= 1u << j;
                        for (int f = 0; f < plan.n; ++f) {
                            const DmrFault ff = plan.f[f];
                            if (ff.owner == block && ff.step == k && ff.sub == 1)
                                apply_fault(plan, ff, x1, x2, t.rep, lane == 0, block, r0 + k, -1, 1);
                        }
                    }
                    bad |= differ(x1, x2);
                    r2[H] = fma(-dup(mh[j]), x2, r2[H]);
                    if (UO) r2[1 - H] = fma(-dup(mo[j]), x2, r2[1 - H]);
                }
                xv[j] = x1;
                r1[H] = fma(-mh[j], x1, r1[H]);
                if (UO) r1[1 - H] = fma(-mo[j], x1, r1[1 - H]);
            }
            if (lane == 0) {
#pragma unroll
                for (int j = 0; j < kStep; ++j)
                    if (i0 + j < nh) xs[krow(i0 + j)] = xv[j];
            }
            if (DMR && bad) {
                // the chunk again from its start, one step at a time, reading the
                // columns from LDS and writing each unknown there as it is formed
                r1[0] = r2[0] = ck0;
                r1[1] = r2[1] = ck1;
                int found = 0;
#pragma unroll 1
                for (int j = 0; j < kStep && i0 + j < nh; ++j) {
                    const int k = krow(i0 + j);
                    const double mhj = M[k * kTrsvLd + lane + 64 * H];
                    const double moj = UO ? M[k * kTrsvLd + lane + 64 * (1 - H)] : 0.0;
                    double x1 = readlane_f64(r1[H] * d[H], k & 63);
                    double x2 = readlane_f64(r2[H] * dup(d[H]), k & 63);
                    int again = -1;
                    if (((planned >> j) & 1) && plan.target == FTG_TARGET_TWO_IN_SLOT) {
                        // a fault that persists strikes the recomputation too
                        for (int f = 0; f < plan.n; ++f)
                            if (plan.f[f].owner == block && plan.f[f].step == k && plan.f[f].sub == 1) again = plan.f[f].bit;
                        if (again >= 0) x1 = flip_f64(x1, again);
                    }
                    if (differ(x1, x2)) {
                        // r_k again from the staged right-hand side and the solved
                        // unknowns, in solve order
                        ++found;
                        const int pos = done + i0 + j;
                        double y1 = rhs[k], y2 = rhs[k];
                        for (int s2 = 0; s2 < pos; ++s2) {
                            const int ks = col(s2);
                            const double mv = M[ks * kTrsvLd + k], xq = xs[ks];
                            y1 = fma(-dup(mv), xq, y1);
                            y2 = fma(-dup(mv), xq, y2);
                        }
                        y1 = y1 * dup(dr[k]);
                        y2 = y2 * dup(dr[k]);
                        if (again >= 0) y1 = flip_f64(y1, again);
                        if (lane == 0) note_repair(t.rep, !differ(y1, y2), block, r0 + k, -1, 1, x1, x2);
                        x1 = y1;
                        x2 = y1;
                    } else if ((planned >> j) & 1) {
                        // a planned fault the chunk check caught and the
                        // recomputation no longer shows
                        ++found;
                        if (lane == 0) note_repair(t.rep, true, block, r0 + k, -1, 1, 0.0, 0.0);
                    }
                    if (lane == 0) xs[k] = x1;
                    r2[H] = fma(-dup(mhj), x2, r2[H]);
                    if (UO) r2[1 - H] = fma(-dup(moj), x2, r2[1 - H]);
                    r1[H] = fma(-mhj, x1, r1[H]);
                    if (UO) r1[1 - H] = fma(-moj, x1, r1[1 - H]);
                }
                // a mismatch that the recomputation does not show again was
                // transient: the recomputed unknowns are the corrected ones
                if (found == 0 && lane == 0) note_repair(t.rep, true, block, r0 + krow(i0), -1, 1, 0.0, 0.0);
            }
#pragma unroll
            for (int j = 0; j < kStep; ++j) {
                mh[j] = nmh[j];
                if (UO) mo[j] = nmo[j];
            }
        }
        done += nh;
    };
    if (t.lower) {
        phase(std::integral_constant<int, 0>{}, std::true_type{});
        phase(std::integral_constant<int, 1>{}, std::false_type{});
    } else {
        phase(std::integral_constant<int, 1>{}, std::true_type{});
        phase(std::integral_constant<int, 0>{}, std::false_type{});
    }
    // xs was written by lane 0 of this wave; LDS accesses of a wave complete in order
    if (lane < nb) t.x[(r0 + lane) * t.incx] = xs[lane];
    if (lane + 64 < nb) t.x[(r0 + lane + 64) * t.incx] = xs[lane + 64];
}

template <bool DMR>
__global__ __launch_bounds__(kThreads, 1) void trsv_chain_kernel(Tc t, DmrPlan plan)
{
    __shared__ double M[kTrsvB * kTrsvLd];
    __shared__ double rhs[kTrsvB], xs[kTrsvB], dr[kTrsvB], xj[kTrsvB];
    __shared__ double red[kThreads];
    __shared__ int s_ticket, s_late;
    const int tid = threadIdx.x;
    if (tid == 0) {
        s_ticket = (int)atomicAdd(&t.sync[0], 1u);
        s_late = 0;
    }
    __syncthreads();
    const int q = s_ticket;  // position in solve order
    const int block = t.lower ? q : t.nblk - 1 - q;
    const int64_t r0 = (int64_t)block * kTrsvB;
    const int nb = (int)imin<int64_t>(kTrsvB, t.n - r0);
    // this block's own entries of x: no other workgroup writes them
    const double xi = tid < nb ? t.x[(r0 + tid) * t.incx] : 0.0;
    stage_tri(M, t, r0, nb);

    // products of the block row with the solved blocks: thread (i, h) takes
    // row i and columns 16 c + 8 h + u (u < 8) of each chunk c of 16 columns
    const int i = t.trans ? tid >> 1 : tid & (kTrsvB - 1);
    const int h = t.trans ? tid & 1 : tid >> 7;
    const bool rowok = i < nb;
    const int64_t gi = r0 + (rowok ? i : 0);
    double acc1 = 0.0, acc2 = 0.0;
    for (int p = 0; p < q; ++p) {
        const int j = t.lower ? p : t.nblk - 1 - p;
        const int64_t c0 = (int64_t)j * kTrsvB;
        const int nbj = (int)imin<int64_t>(kTrsvB, t.n - c0);
        double a[8][kU];
#pragma unroll
        for (int cc = 0; cc < 8; ++cc)
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                const int c = cc * 16 + h * kU + u;
                const bool ok = rowok && c < nbj;
                const int64_t gc = c0 + (c < nbj ? c : 0);
                const double v = t.trans ? t.A[gc + gi * t.lda] : t.A[gi + gc * t.lda];
                a[cc][u] = ok ? v : 0.0;
            }
        if (tid == 0) {
            int spins = 0;
            while (__hip_atomic_load(&t.sync[1 + j], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == 0u) {
                __builtin_amdgcn_s_sleep(2);
                if (++spins >= t.spin_limit) {
                    s_late = 1;
                    break;
                }
            }
        }
        __syncthreads();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        if (tid < kTrsvB) xj[tid] = tid < nbj ? t.x[(c0 + tid) * t.incx] : 0.0;
        __syncthreads();
#pragma unroll
        for (int cc = 0; cc < 8; ++cc) {
            const double chk = acc1;
#pragma unroll
            for (int u = 0; u < kU; ++u) acc1 = fma(a[cc][u], xj[cc * 16 + h * kU + u], acc1);
            if constexpr (DMR) {
#pragma unroll
                for (int u = 0; u < kU; ++u) acc2 = fma(dup(a[cc][u]), xj[cc * 16 + h * kU + u], acc2);
                if (differ(acc1, acc2)) {
                    double r1 = chk, r2 = chk;
#pragma unroll
                    for (int u = 0; u < kU; ++u) r1 = fma(dup(a[cc][u]), xj[cc * 16 + h * kU + u], r1);
#pragma unroll
                    for (int u = 0; u < kU; ++u) r2 = fma(dup(a[cc][u]), xj[cc * 16 + h * kU + u], r2);
                    note_repair(t.rep, !differ(r1, r2), block, gi, c0 + cc * 16 + h * kU, p, acc1, acc2);
                    acc1 = r1;
                    acc2 = r1;
                }
            }
        }
        __syncthreads();  // xj is rewritten for the next block
    }
    red[tid] = acc1;
    __syncthreads();
    // right-hand side r_i = x_i - (both halves of the products), reciprocal diagonal
    if (tid < kTrsvB) {
        double q1 = 0.0, s1 = 0.0;
        if (tid < nb) {
            const double pa = t.trans ? red[2 * tid] : red[tid];
            const double pb = t.trans ? red[2 * tid + 1] : red[tid + kTrsvB];
            const double dg = M[tid * kTrsvLd + tid];
            q1 = 1.0 / dg;
            const int64_t g = r0 + tid;
            s1 = xi - (pa + pb);
            if constexpr (DMR) {
                double s2 = xi - (dup(pa) + dup(pb));
                const double q2 = 1.0 / dup(dg);
                if (differ(q1, q2)) {
                    const double a1 = 1.0 / dup(dg), a2 = 1.0 / dup(dg);
                    note_repair(t.rep, !differ(a1, a2), block, g, -1, 0, q1, q2);
                    q1 = a1;
                }
                int again = -1;
                for (int f = 0; f < plan.n; ++f) {
                    const DmrFault ff = plan.f[f];
                    if (ff.owner == block && ff.step == tid && ff.sub == 0)
                        again = apply_fault(plan, ff, s1, s2, t.rep, true, block, g, -1, 0);
                }
                if (differ(s1, s2)) {
                    double r1 = xi - (dup(pa) + dup(pb));
                    const double r2 = xi - (dup(pa) + dup(pb));
                    if (again >= 0) r1 = flip_f64(r1, again);
                    note_repair(t.rep, !differ(r1, r2), block, g, -1, 0, s1, s2);
                    s1 = r1;
                }
            }
        }
        dr[tid] = q1;
        rhs[tid] = s1;
    }
    __syncthreads();
    if (tid >= 64) return;
    substitute<DMR>(M, rhs, dr, xs, t, r0, nb, block, plan);
    // publish: the unknowns' stores complete and become visible device-wide before the flag
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    if (tid == 0) {
        __hip_atomic_store(&t.sync[1 + block], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        if (s_late) {
            // a wait ran out: the products used whatever x held then
            atomicAdd(&t.rep->cnt[kDetected], 1ull);
            atomicAdd(&t.rep->cnt[kUncorrectable], 1ull);
            push_record(t.rep, 0, block, -1, 0, r0, -1, FTG_KIND_UNCORRECTABLE, 0.0, 0.0);
        }
    }
}

__global__ void zero_u32_kernel(unsigned int* p, int64_t count)
{
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count; e += (int64_t)gridDim.x * blockDim.x)
        p[e] = 0u;
}

int64_t vec_blocks(int64_t n)
{
    int64_t b = (n + kVecStep * (kThreads / 64) - 1) / (kVecStep * (kThreads / 64));
    return b < 1 ? 1 : (b > kVecMaxBlocks ? kVecMaxBlocks : b);
}

// Thread and step of element i of a DSCAL/DNRM2 launch with `nwaves` waves.
void map_vec(DmrPlan& plan, int64_t nwaves, bool v2)
{
    for (int q = 0; q < plan.n; ++q) {
        DmrFault& f = plan.f[q];
        // the element's place in its run c0 = c * 512 (see vec_elem)
        const int64_t c = f.unit / kVecStep, r = f.unit % kVecStep;
        f.owner = (c % nwaves) * 64 + (v2 ? (r % 128) / 2 : r % 64);
        f.step = (int)(c / nwaves);
        f.sub = (int)(v2 ? 2 * (r / 128) + r % 2 : r / 64);
    }
}

// Shape of a DGEMV launch: workgroups along the outputs, chunk width and
// count along the reduction (aiming at kGvTarget workgroups, at most
// max_chunks chunks).
struct GvShape {
    int64_t bout, width, chunks;
};

GvShape gv_shape(int trans, int64_t rows, int64_t cols, int64_t target, int64_t max_chunks)
{
    GvShape s;
    const int64_t red = trans ? rows : cols;          // reduction length
    const int64_t gran = trans ? kGtStep : 4 * kU;    // chunk width granularity
    s.bout = trans ? (cols + kGtCols - 1) / kGtCols : (rows + kGnRows - 1) / kGnRows;
    int64_t want = (target + s.bout - 1) / s.bout;
    const int64_t most = (red + gran - 1) / gran;
    if (want > most) want = most;
    if (want > max_chunks) want = max_chunks;
    if (want < 1) want = 1;
    s.width = ((red + want - 1) / want + gran - 1) / gran * gran;
    s.chunks = (red + s.width - 1) / s.width;
    return s;
}

// Thread and step of DGEMV unit u (see dmr_units_gemv).
void map_gemv(DmrPlan& plan, int trans, int64_t rows, int64_t cols, const GvShape& sh)
{
    for (int q = 0; q < plan.n; ++q) {
        DmrFault& f = plan.f[q];
        if (!trans) {
            const int64_t i = f.unit % rows, j0 = (f.unit / rows) * kU;
            const int64_t c = j0 / sh.width, wcols = sh.width / 4;
            const int64_t wv = (j0 - c * sh.width) / wcols;
            const int64_t step = (j0 - c * sh.width - wv * wcols) / kU;
            const int64_t bid = c * sh.bout + i / kGnRows;
            f.owner = bid * kThreads + wv * 64 + i % kGnRows;
            f.step = (int)step;
        } else {
            const int64_t j = f.unit % cols, rest = f.unit / cols;
            const int64_t lane = rest % 64, r0 = (rest / 64) * kGtStep;  // the lane's first row is r0 + lane
            const int64_t c = r0 / sh.width;
            const int64_t bid = c * sh.bout + j / kGtCols;
            f.owner = bid * kThreads + (j % kGtCols) * 64 + lane;
            f.step = (int)((r0 - c * sh.width) / kGtStep);
        }
        f.sub = 0;
    }
}

template <bool DMR>
hipError_t gemv_launch(int trans, const Gv& g, int64_t grid, const DmrPlan& plan, bool xunit, hipStream_t s)
{
    if (!trans) {
        if (xunit) hipLaunchKernelGGL((gemv_n_kernel<DMR, true>), dim3((unsigned)grid), dim3(kThreads), 0, s, g, plan);
        else hipLaunchKernelGGL((gemv_n_kernel<DMR, false>), dim3((unsigned)grid), dim3(kThreads), 0, s, g, plan);
    } else {
        if (xunit) hipLaunchKernelGGL((gemv_t_kernel<DMR, true>), dim3((unsigned)grid), dim3(kThreads), 0, s, g, plan);
        else hipLaunchKernelGGL((gemv_t_kernel<DMR, false>), dim3((unsigned)grid), dim3(kThreads), 0, s, g, plan);
    }
    return hipGetLastError();
}

}  // namespace

int64_t dmr_units_vec(int64_t n) { return n; }

// Without transpose: (output row i, group of 8 consecutive columns g) as
// u = i + m g.  Transposed: (output column j, lane group: the rows
// 512 t + l + 64 u, u < 8, that one lane adds between two comparisons, for
// every (t, l) with 512 t + l < m) as u = j + n (64 t + l).
int64_t dmr_units_gemv(int trans, int64_t m, int64_t n)
{
    if (!trans) return m * ((n + kU - 1) / kU);
    const int64_t groups = (m / kGtStep) * 64 + imin<int64_t>(64, m % kGtStep);
    return n * groups;
}

int64_t dmr_units_trsv(int64_t n) { return n; }

size_t dmr_nrm2_work_bytes(int64_t n) { return (size_t)vec_blocks(n) * 3 * sizeof(double); }

size_t dmr_gemv_work_bytes(int trans, int64_t m, int64_t n)
{
    const GvShape sh = gv_shape(trans, m, n, kGvTarget, INT64_MAX);
    return sh.chunks > 1 ? (size_t)sh.chunks * (size_t)(trans ? n : m) * sizeof(double) : 0;
}

size_t dmr_trsv_work_bytes(int64_t n) { return n > 0 ? (size_t)((n + kTrsvB - 1) / kTrsvB + 1) * sizeof(unsigned int) : 0; }

hipError_t launch_dmr_scal(double* x, int64_t n, int64_t inc, double alpha, bool dmr, DmrPlan plan, DevReport* rep,
                           hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const int64_t blocks = vec_blocks(n), nwaves = blocks * (kThreads / 64);
    map_vec(plan, nwaves, false);
    const dim3 grid((unsigned)blocks), blk(kThreads);
    auto go = [&](auto kern) { hipLaunchKernelGGL(kern, grid, blk, 0, s, x, n, inc, alpha, nwaves, plan, rep); };
    if (dmr) {
        if (inc == 1) go(scal_kernel<true, true, false>);
        else go(scal_kernel<true, false, false>);
    } else {
        if (inc == 1) go(scal_kernel<false, true, false>);
        else go(scal_kernel<false, false, false>);
    }
    return hipGetLastError();
}

hipError_t launch_dmr_nrm2(const double* x, int64_t n, int64_t inc, double* out, double* work, bool dmr,
                           DmrPlan plan, DevReport* rep, hipStream_t s)
{
    const int64_t blocks = vec_blocks(n), nwaves = blocks * (kThreads / 64);
    const bool v2 = inc == 1 && (reinterpret_cast<uintptr_t>(x) & 15) == 0;
    map_vec(plan, nwaves, v2);
    const dim3 grid((unsigned)blocks), blk(kThreads);
    auto go = [&](auto kern) { hipLaunchKernelGGL(kern, grid, blk, 0, s, x, n, inc, nwaves, work, plan, rep); };
    if (dmr) {
        if (v2) go(nrm2_part_kernel<true, true, true>);
        else if (inc == 1) go(nrm2_part_kernel<true, true, false>);
        else go(nrm2_part_kernel<true, false, false>);
        hipLaunchKernelGGL((nrm2_final_kernel<true>), dim3(1), blk, 0, s, work, (int)blocks, out, rep);
    } else {
        if (v2) go(nrm2_part_kernel<false, true, true>);
        else if (inc == 1) go(nrm2_part_kernel<false, true, false>);
        else go(nrm2_part_kernel<false, false, false>);
        hipLaunchKernelGGL((nrm2_final_kernel<false>), dim3(1), blk, 0, s, work, (int)blocks, out, rep);
    }
    return hipGetLastError();
}

hipError_t launch_dmr_gemv(int trans, int64_t m, int64_t n, double alpha, const double* A, int64_t lda,
                           const double* x, int64_t incx, double beta, double* y, int64_t incy, double* work,
                           bool dmr, DmrPlan plan, DevReport* rep, hipStream_t s)
{
    const GvShape sh = gv_shape(trans, m, n, kGvTarget, INT64_MAX);
    map_gemv(plan, trans, m, n, sh);
    Gv g;
    g.A = A;
    g.lda = lda;
    g.rows = m;
    g.cols = n;
    g.x = x;
    g.incx = incx;
    g.y = y;
    g.incy = incy;
    g.alpha = alpha;
    g.beta = beta;
    g.part = work;
    g.ldp = trans ? n : m;
    g.width = sh.width;
    g.bout = sh.bout;
    g.direct = sh.chunks == 1;
    g.rep = rep;
    const int64_t grid = sh.bout * sh.chunks;
    hipError_t e = dmr ? gemv_launch<true>(trans, g, grid, plan, incx == 1, s)
                       : gemv_launch<false>(trans, g, grid, plan, incx == 1, s);
    if (e != hipSuccess || g.direct) return e;
    const int64_t len = trans ? n : m;
    const unsigned rgrid = (unsigned)((len + kThreads - 1) / kThreads);
    if (dmr) hipLaunchKernelGGL((gemv_reduce_kernel<true>), dim3(rgrid), dim3(kThreads), 0, s, g, len, sh.chunks);
    else hipLaunchKernelGGL((gemv_reduce_kernel<false>), dim3(rgrid), dim3(kThreads), 0, s, g, len, sh.chunks);
    return hipGetLastError();
}

hipError_t launch_dmr_trsv(int lower, int trans, int unit, int64_t n, const double* A, int64_t lda, double* x,
                           int64_t incx, double* work, bool dmr, DmrPlan plan, DevReport* rep, hipStream_t s)
{
    for (int q = 0; q < plan.n; ++q) {
        plan.f[q].owner = plan.f[q].unit / kTrsvB;
        plan.f[q].step = (int)(plan.f[q].unit % kTrsvB);
    }
    const int64_t nblk = (n + kTrsvB - 1) / kTrsvB;
    unsigned int* sync = reinterpret_cast<unsigned int*>(work);
    // a fill kernel, not a memset, so that the call can be captured in a graph
    const int64_t zb = imin<int64_t>((nblk + 1 + 255) / 256, 1024);
    hipLaunchKernelGGL(zero_u32_kernel, dim3((unsigned)zb), dim3(256), 0, s, sync, nblk + 1);
    Tc t;
    t.A = A;
    t.lda = lda;
    t.x = x;
    t.incx = incx;
    t.n = n;
    t.nblk = (int)nblk;
    t.lower = lower;
    t.trans = trans;
    t.unit = unit;
    t.sync = sync;
    t.spin_limit = 1 << 22;
    t.rep = rep;
    if (dmr) hipLaunchKernelGGL((trsv_chain_kernel<true>), dim3((unsigned)nblk), dim3(kThreads), 0, s, t, plan);
    else hipLaunchKernelGGL((trsv_chain_kernel<false>), dim3((unsigned)nblk), dim3(kThreads), 0, s, t, plan);
    return hipGetLastError();
}

}  // namespace ftg
