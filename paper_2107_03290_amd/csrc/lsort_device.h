// Device-side building blocks of the LearnedSort 2.0 kernels (gfx950, wave64):
// key words, the sampler, the model, block scans.
//
// Floating point: the model is evaluated in FP64 exactly as written (the
// library is compiled with -ffp-contract=off; the single fused multiply-add
// is explicit), so predictions are bit-identical to any IEEE-754 FP64
// evaluation of the same formulas.
#pragma once
#include "lsort_internal.h"

#pragma clang fp contract(off)

namespace lsort {

// ------------------------------------------------------- global pointers --

// Key and range pointers are read from descriptors in memory, so the compiler
// cannot tell which address space they point into and accesses through them
// become flat instructions.  On gfx9 a flat access also counts against the
// LDS wait counter: every wait for an LDS result would then also wait for the
// keys in flight (the next tile's prefetch) and for earlier stores.  Every
// buffer the library hands to a kernel is device (global) memory, so such
// pointers are cast to the global address space before use.
template <class T>
using gptr = __attribute__((address_space(1))) T*;

template <class T>
__device__ __forceinline__ gptr<T> as_global(T* p)
{
    return (gptr<T>)p;
}

constexpr uint64_t kSign = 0x8000000000000000ull;
constexpr uint64_t kSkipBit = 0x8000000000000000ull;
constexpr uint32_t kNoScatter = 1u;
constexpr uint32_t kFlagNonMonotone = 0x4u;   // LS_FLAG_NONMONOTONE
// s_waitcnt operand: vmcnt(0), expcnt and lgkmcnt left at their maximum
constexpr int kWaitVmcnt0 = 0x0F70;

// ------------------------------------------------------------------ keys --

// IEEE-754 totalOrder as an unsigned word: negative keys are bit-inverted,
// non-negative keys get the sign bit set.
__device__ __forceinline__ uint64_t to_ord(uint64_t raw, uint32_t dt)
{
    if (dt != kF64)
        return raw;
    return (raw & kSign) ? ~raw : (raw | kSign);
}

__device__ __forceinline__ uint64_t from_ord(uint64_t o, uint32_t dt)
{
    if (dt != kF64)
        return o;
    return (o & kSign) ? (o & ~kSign) : ~o;
}

// Value seen by the model: the double itself, or the u64 rounded to nearest.
__device__ __forceinline__ double key_value(uint64_t raw, uint32_t dt)
{
    return dt == kF64 ? __longlong_as_double((long long)raw) : (double)raw;
}

__device__ __forceinline__ bool nonfinite(uint64_t raw, uint32_t dt)
{
    return dt == kF64 && ((raw >> 52) & 0x7ffu) == 0x7ffu;
}

__device__ __forceinline__ double ord_value(uint64_t o, uint32_t dt)
{
    return key_value(from_ord(o, dt), dt);
}

// ---------------------------------------------------------------- sampler --

// SplitMix64 (Steele, Lea, Flood 2014): output t of the stream whose state
// starts at `seed` is the state after t+1 golden-gamma increments, mixed.
__device__ __forceinline__ uint64_t splitmix64_at(uint64_t seed, uint64_t t)
{
    uint64_t z = seed + (t + 1u) * 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ uint64_t sample_index(uint64_t seed, uint64_t t, uint64_t n)
{
    return __umul64hi(splitmix64_at(seed, t), n);
}

// ------------------------------------------------------------------ model --

// Device model layout at offset o of the pool (doubles):
//   [xmin, xmax, rs, m'], then per leaf k the segment starting at its knot
//   {X_k, y_k, s_k, yhi_k} (an empty leaf has X_k = +inf), then L uint32
//   "previous knot" indices (kNoPrev: none).
// In LDS the segments are double2 pairs {X, y}, {s, yhi}; entry L is a
// constant-zero segment that stands for "below the first knot".
// Root coordinate of a value: the totalOrder word of the double, as a number.
__device__ __forceinline__ double root_coord(double x)
{
    const uint64_t b = (uint64_t)__double_as_longlong(x);
    return __ull2double_rn((b >> 63) ? ~b : (b | kSign));
}

// A model as partition kernels use it, from LDS.  Knots 0..L-1 are the leaf
// knots, knot L the start knot at the sample minimum.
struct SModel {
    double r0, rs, lm1;
    uint32_t L;
    const double2* seg;     // 2 (L + 1) entries: {X, ylo}, {s, yhi}
    const double* ym;       // L + 1 mid-ranks at the knots
    const uint16_t* prev;   // L entries, L for none
};

// Copy a model into LDS (all threads participate; caller syncs).
__device__ __forceinline__ void load_model(SModel& M, const double* pool, uint64_t off, uint32_t L, void* lds)
{
    const double* g = pool + off;
    double2* seg = reinterpret_cast<double2*>(lds);
    double* ym = reinterpret_cast<double*>(seg + 2 * (L + 1));
    uint16_t* prev = reinterpret_cast<uint16_t*>(ym + (L + 1));
    const double2* gs = reinterpret_cast<const double2*>(g + kModelSeg);
    for (uint32_t i = threadIdx.x; i < 2 * (L + 1); i += blockDim.x)
        seg[i] = gs[i];
    const double* gym = g + model_ym_off(L);
    for (uint32_t i = threadIdx.x; i <= L; i += blockDim.x)
        ym[i] = gym[i];
    const uint32_t* gp = reinterpret_cast<const uint32_t*>(g + model_prev_off(L));
    for (uint32_t i = threadIdx.x; i < L; i += blockDim.x) {
        const uint32_t p = gp[i];
        prev[i] = (uint16_t)(p == kNoPrev ? L : p);
    }
    M.r0 = root_coord(g[0]);
    M.rs = g[2];
    M.L = L;
    M.lm1 = (double)(L - 1u);
    M.seg = seg;
    M.ym = ym;
    M.prev = prev;
}

// F(x), the model's estimate of the fraction of keys below x: the segment of
// the largest knot not above x; the knot's mid-rank at the knot itself; 0
// below the sample minimum; non-finite keys map to 0 or 1 by sign.
template <uint32_t DT>
__device__ __forceinline__ double model_F(const SModel& M, uint64_t raw)
{
    const double x = key_value(raw, DT);
    const double r = DT == kF64 ? __ull2double_rn(to_ord(raw, kF64)) : root_coord(x);
    const double t = (r - M.r0) * M.rs;
    const uint32_t k = t >= 1.0 ? (t >= M.lm1 ? M.L - 1u : (uint32_t)t) : 0u;
    uint32_t j = k;
    double2 a = M.seg[2 * k];         // {X, ylo}
    double2 b = M.seg[2 * k + 1];     // {s, yhi}
    // Keep the whole segment loaded here: otherwise the compiler moves the
    // loads of ylo, s and yhi past the branch (they are dead on its taken
    // side), and the common path pays a second dependent LDS round trip.
    asm volatile("" : "+v"(a.y), "+v"(b.x), "+v"(b.y));
    if (x < a.x) {                    // below this leaf's knot: previous knot
        j = M.prev[k];
        a = M.seg[2 * j];
        b = M.seg[2 * j + 1];
    }
    double F = __fma_rn(x - a.x, b.x, a.y);
    F = F < a.y ? a.y : F;
    F = F > b.y ? b.y : F;
    F = b.x == 0.0 ? a.y : F;
    if (x == a.x)
        F = M.ym[j];
    if (j == M.L && !(x >= a.x))      // below the sample minimum
        F = 0.0;
    if (DT == kF64 && nonfinite(raw, kF64))
        F = (raw & kSign) ? 0.0 : 1.0;
    return F;
}

// Bucket of a model task: clamp(floor(F * scale) - offset, 0, fanout - 1);
// F * scale <= fanout^2 < 2^31, so 32-bit integers are exact.
template <uint32_t DT>
__device__ __forceinline__ uint32_t model_bucket(const SModel& M, uint64_t raw, double scale, int32_t offset,
                                                 uint32_t fanout, uint32_t flags)
{
    const double v = model_F<DT>(M, raw) * scale;
    int32_t q = (int32_t)v - offset;
    q = q < 0 ? 0 : q;
    q = q > (int32_t)fanout - 1 ? (int32_t)fanout - 1 : q;
    uint32_t b = (uint32_t)q;
    if (flags & kFlagNonMonotone)        // test hook: break monotonicity on purpose
        b = (raw & 1u) ? (b + fanout / 2u) % fanout : b;
    return b;
}

template <uint32_t DT>
__device__ __forceinline__ uint32_t msd_bucket(uint64_t raw, uint32_t shift, uint32_t fanout)
{
    return (uint32_t)((to_ord(raw, DT) >> shift) & (uint64_t)(fanout - 1u));
}

// ------------------------------------------------------------ task lists --

// The task of a round that owns chunk `chunk` (tasks are laid out with
// increasing chunk0).
__device__ __forceinline__ uint32_t find_task(const Task* tasks, uint32_t ntasks, uint32_t chunk)
{
    uint32_t lo = 0, hi = ntasks;
    while (hi - lo > 1) {
        uint32_t mid = (lo + hi) >> 1;
        if (tasks[mid].chunk0 <= chunk) lo = mid; else hi = mid;
    }
    return lo;
}

// ------------------------------------------------------ workgroup order --

// Workgroups of a launch are handed to the eight XCDs in turn (workgroup b
// runs on XCD b mod 8), and each XCD has its own L2.  xcd_order maps b to a
// work index so that every XCD gets one contiguous range of work items:
// neighbouring items, whose outputs meet in shared cache lines, then run on
// the same XCD.  A bijection of [0, grid).
__device__ __forceinline__ uint32_t xcd_order(uint32_t b, uint32_t grid)
{
    const uint32_t x = b & 7u, j = b >> 3, q = grid >> 3, r = grid & 7u;
    return x * q + (x < r ? x : r) + j;
}

// ------------------------------------------------------- LDS bitonic sort --

// Ascending bitonic network over N = 2^logN (16 <= N <= 16 * NT) words in
// LDS, stored at base_pad(i).  Each thread keeps 16 elements in registers:
// the 16 indices that differ only in a window of 4 index bits.  Up to four
// consecutive stages of the network touch only bits inside one window, so
// each LDS round trip runs four stages in registers; a phase of the network
// needs ceil(p/4) round trips.  All NT threads call it; the words must be in
// LDS and synchronised on entry, and are sorted and synchronised on exit.
// PAD = false: the words sit at plain indices (more bank conflicts).
__host__ __device__ __forceinline__ uint32_t base_pad(uint32_t i) { return i + (i >> 4); }

// LDS word of element i: padded (one spare word per 16 against bank
// conflicts) or plain.
template <bool PAD>
__device__ __forceinline__ uint32_t lds_at(uint32_t i) { return PAD ? base_pad(i) : i; }

// element index of register m of thread t, the 4 register bits at [lo, lo+4)
__device__ __forceinline__ uint32_t base_idx(uint32_t t, uint32_t lo, uint32_t m)
{
    const uint32_t low = t & ((1u << lo) - 1u);
    return low | (m << lo) | ((t >> lo) << (lo + 4));
}

__device__ __forceinline__ void cmpex(uint64_t& a, uint64_t& b, bool up)
{
    const bool sw = (a > b) == up;
    const uint64_t x = sw ? b : a;
    const uint64_t y = sw ? a : b;
    a = x;
    b = y;
}

// Stages on register bits top..0 (top <= 3) with one direction.
__device__ __forceinline__ void reg_stages(uint64_t (&r)[16], uint32_t top, bool up)
{
#pragma unroll
    for (int rb = 3; rb >= 0; --rb) {
        if ((uint32_t)rb <= top) {
#pragma unroll
            for (int m = 0; m < 16; ++m)
                if (!(m & (1 << rb)))
                    cmpex(r[m], r[m | (1 << rb)], up);
        }
    }
}

template <uint32_t NT, bool PAD = true>
__device__ void lds_bitonic(uint64_t* s, uint32_t logN)
{
    const uint32_t t = threadIdx.x;
    const bool act = t < ((1u << logN) >> 4);
    uint64_t r[16];
    // phases 1..4: the 16 consecutive elements of each thread
    if (act) {
#pragma unroll
        for (int m = 0; m < 16; ++m)
            r[m] = s[lds_at<PAD>(16 * t + m)];
#pragma unroll
        for (int p = 1; p <= 4; ++p) {
#pragma unroll
            for (int rb = p - 1; rb >= 0; --rb) {
#pragma unroll
                for (int m = 0; m < 16; ++m) {
                    if (!(m & (1 << rb))) {
                        const uint32_t idx = 16u * t + (uint32_t)m;
                        const bool up = ((idx >> p) & 1u) == 0 || (uint32_t)p == logN;
                        cmpex(r[m], r[m | (1 << rb)], up);
                    }
                }
            }
        }
#pragma unroll
        for (int m = 0; m < 16; ++m)
            s[lds_at<PAD>(16 * t + m)] = r[m];
    }
    __syncthreads();
    // phases 5..logN: stages on bits p-1 .. 0 in windows of four bits
    for (uint32_t p = 5; p <= logN; ++p) {
        int32_t bit = (int32_t)p - 1;
        while (bit >= 0) {
            const uint32_t lo = bit >= 3 ? (uint32_t)bit - 3 : 0u;
            if (act) {
                const uint32_t i0 = base_idx(t, lo, 0);
                const bool up = p == logN || ((i0 >> p) & 1u) == 0;
#pragma unroll
                for (int m = 0; m < 16; ++m)
                    r[m] = s[lds_at<PAD>(base_idx(t, lo, (uint32_t)m))];
                reg_stages(r, (uint32_t)bit - lo, up);
#pragma unroll
                for (int m = 0; m < 16; ++m)
                    s[lds_at<PAD>(base_idx(t, lo, (uint32_t)m))] = r[m];
            }
            __syncthreads();
            bit = (int32_t)lo - 1;
        }
    }
}

// ------------------------------------------------------------ block scans --

// Exclusive prefix of the per-wave totals wsum[0..nw) in place, with the
// grand total in wsum[nw]; done by wave 0 with shuffles.  Call between two
// barriers of the whole block.
template <typename T, typename Op>
__device__ __forceinline__ void wave_totals_scan(T* wsum, uint32_t nw, T ident, Op op)
{
    if (threadIdx.x < 64) {
        const uint32_t lane = threadIdx.x;
        T v = lane < nw ? wsum[lane] : ident;
#pragma unroll
        for (uint32_t d = 1; d < 16; d <<= 1) {
            const T y = __shfl_up(v, d, 64);
            if (lane >= d)
                v = op(y, v);
        }
        T ex = __shfl_up(v, 1, 64);
        if (lane == 0)
            ex = ident;
        if (lane < nw)
            wsum[lane] = ex;
        if (lane + 1 == nw)
            wsum[nw] = v;
    }
}

struct AddU32 {
    __device__ uint32_t operator()(uint32_t a, uint32_t b) const { return a + b; }
};

// Exclusive scan of in[0..n) (LDS, u32) into out[0..n) (may be the same
// array); returns the total.  wsum: LDS scratch of blockDim/64 + 1 entries;
// at most 16 waves.
__device__ inline uint32_t block_scan_u32(const uint32_t* in, uint32_t* out, uint32_t n, uint32_t* wsum)
{
    const uint32_t nt = blockDim.x;
    const uint32_t per = (n + nt - 1) / nt;
    const uint32_t lo = min(n, threadIdx.x * per), hi = min(n, lo + per);
    uint32_t s = 0;
    for (uint32_t i = lo; i < hi; ++i)
        s += in[i];
    const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
    uint32_t x = s;
#pragma unroll
    for (uint32_t d = 1; d < 64; d <<= 1) {
        uint32_t y = __shfl_up(x, d, 64);
        if (lane >= d)
            x += y;
    }
    if (lane == 63)
        wsum[wave] = x;
    __syncthreads();
    wave_totals_scan<uint32_t>(wsum, nt / 64, 0u, AddU32());
    __syncthreads();
    uint32_t base = wsum[wave] + x - s;
    for (uint32_t i = lo; i < hi; ++i) {
        uint32_t v = in[i];
        out[i] = base;
        base += v;
    }
    uint32_t total = wsum[nt / 64];
    __syncthreads();
    return total;
}

__device__ inline uint32_t block_scan_u32(uint32_t* a, uint32_t n, uint32_t* wsum)
{
    return block_scan_u32(a, a, n, wsum);
}

// K exclusive scans of a[k][0..n) in place (LDS, u32) sharing the three
// barriers of one; totals[k] receives each grand total.  wsum: K rows of
// blockDim/64 + 1 entries; at most 16 waves.
template <uint32_t K>
__device__ inline void block_scan_u32_multi(uint32_t* const (&a)[K], uint32_t n, uint32_t (*wsum)[17],
                                            uint32_t (&totals)[K])
{
    const uint32_t nt = blockDim.x;
    const uint32_t per = (n + nt - 1) / nt;
    const uint32_t lo = min(n, threadIdx.x * per), hi = min(n, lo + per);
    const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
    uint32_t s[K], x[K];
#pragma unroll
    for (uint32_t k = 0; k < K; ++k) {
        s[k] = 0;
        for (uint32_t i = lo; i < hi; ++i)
            s[k] += a[k][i];
        x[k] = s[k];
#pragma unroll
        for (uint32_t d = 1; d < 64; d <<= 1) {
            const uint32_t y = __shfl_up(x[k], d, 64);
            if (lane >= d)
                x[k] += y;
        }
        if (lane == 63)
            wsum[k][wave] = x[k];
    }
    __syncthreads();
#pragma unroll
    for (uint32_t k = 0; k < K; ++k)
        wave_totals_scan<uint32_t>(wsum[k], nt / 64, 0u, AddU32());
    __syncthreads();
#pragma unroll
    for (uint32_t k = 0; k < K; ++k) {
        uint32_t base = wsum[k][wave] + x[k] - s[k];
        for (uint32_t i = lo; i < hi; ++i) {
            const uint32_t v = a[k][i];
            a[k][i] = base;
            base += v;
        }
        totals[k] = wsum[k][nt / 64];
    }
    __syncthreads();
}

// Sum / maximum over the 64 lanes of a wave (every lane gets the result).
template <typename T>
__device__ __forceinline__ T wave_sum(T v)
{
#pragma unroll
    for (uint32_t d = 32; d > 0; d >>= 1)
        v += __shfl_xor(v, d, 64);
    return v;
}

template <typename T>
__device__ __forceinline__ T wave_max(T v)
{
#pragma unroll
    for (uint32_t d = 32; d > 0; d >>= 1) {
        const T y = __shfl_xor(v, d, 64);
        v = y > v ? y : v;
    }
    return v;
}

// Generic exclusive block scan (LDS, in place) with an associative operator;
// returns the reduction of all n entries.  wsum: blockDim/64 + 1 entries.
template <typename T, typename Op>
__device__ T block_scan_op(T* a, uint32_t n, T ident, Op op, T* wsum)
{
    const uint32_t nt = blockDim.x;
    const uint32_t per = (n + nt - 1) / nt;
    const uint32_t lo = min(n, threadIdx.x * per), hi = min(n, lo + per);
    T s = ident;
    for (uint32_t i = lo; i < hi; ++i)
        s = op(s, a[i]);
    const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
    T x = s;
#pragma unroll
    for (uint32_t d = 1; d < 64; d <<= 1) {
        T y = __shfl_up(x, d, 64);
        if (lane >= d)
            x = op(y, x);
    }
    // exclusive prefix within the wave
    T ex = __shfl_up(x, 1, 64);
    if (lane == 0)
        ex = ident;
    if (lane == 63)
        wsum[wave] = x;
    __syncthreads();
    wave_totals_scan<T>(wsum, nt / 64, ident, op);
    __syncthreads();
    T base = op(wsum[wave], ex);
    for (uint32_t i = lo; i < hi; ++i) {
        T v = a[i];
        a[i] = base;
        base = op(base, v);
    }
    T total = wsum[nt / 64];
    __syncthreads();
    return total;
}

struct MaxI32 {
    __device__ int32_t operator()(int32_t a, int32_t b) const { return a > b ? a : b; }
};
struct MinI32 {
    __device__ int32_t operator()(int32_t a, int32_t b) const { return a < b ? a : b; }
};
struct AddU64 {
    __device__ uint64_t operator()(uint64_t a, uint64_t b) const { return a + b; }
};

}  // namespace lsort
