// LearnedSort 2.0 hot path for gfx950: sampling, model training, bucket
// histogram, prefix scan, classification, scatter, LDS base case, fills and
// the touch-up check.  Every kernel runs wave64; LDS holds the model, the
// per-bucket counters and the staged tile.
//
// Floating point: the model is evaluated in FP64 exactly as written (the
// library is compiled with -ffp-contract=off; the single fused multiply-add
// is explicit), so predictions are bit-identical to any IEEE-754 FP64
// evaluation of the same formulas.
#include "lsort_internal.h"

#pragma clang fp contract(off)

namespace lsort {

constexpr uint64_t kSign = 0x8000000000000000ull;
constexpr uint64_t kSkipBit = 0x8000000000000000ull;
constexpr uint32_t kNoScatter = 1u;
constexpr uint32_t kFlagNonMonotone = 0x4u;   // LS_FLAG_NONMONOTONE

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
//   [xmin, xmax, rs, m'] X[L] y[L] yhi[L] s[L] then L uint32 "previous knot".
struct SModel {
    double xmin, rs, lm1;
    uint32_t L;
    const double* X;
    const double* y;
    const double* yhi;
    const double* s;
    const uint16_t* prev;
};

// Copy a model into LDS (all threads participate).
__device__ __forceinline__ void load_model(SModel& M, const double* pool, uint64_t off, uint32_t L,
                                           double* lds, uint16_t* lprev)
{
    const double* g = pool + off;
    for (uint32_t i = threadIdx.x; i < 4 * L; i += blockDim.x)
        lds[i] = g[4 + i];
    const uint32_t* gp = reinterpret_cast<const uint32_t*>(g + 4 + 4 * (size_t)L);
    for (uint32_t i = threadIdx.x; i < L; i += blockDim.x)
        lprev[i] = (uint16_t)gp[i];
    M.xmin = g[0];
    M.rs = g[2];
    M.L = L;
    M.lm1 = (double)(L - 1u);
    M.X = lds;
    M.y = lds + L;
    M.yhi = lds + 2 * L;
    M.s = lds + 3 * L;
    M.prev = lprev;
}

// F(x): fraction of the sample below x, interpolated linearly from the
// largest knot not above x (knots: leaf minima of the sample).
__device__ __forceinline__ double model_F(const SModel& M, uint64_t raw, uint32_t dt)
{
    if (nonfinite(raw, dt))
        return (raw & kSign) ? 0.0 : 1.0;
    const double x = key_value(raw, dt);
    const double t = (x - M.xmin) * M.rs;
    uint32_t k;
    if (!(t >= 1.0))
        k = 0;
    else if (t >= M.lm1)
        k = M.L - 1u;
    else
        k = (uint32_t)t;
    uint32_t j = (x >= M.X[k]) ? k : (uint32_t)M.prev[k];
    if (j == kNoPrev)
        return 0.0;
    const double s = M.s[j];
    const double y = M.y[j];
    if (s == 0.0)
        return y;
    double F = __fma_rn(x - M.X[j], s, y);
    F = F < y ? y : F;
    const double yh = M.yhi[j];
    return F > yh ? yh : F;
}

__device__ __forceinline__ uint32_t bucket_of(const Task& T, const SModel& M, uint64_t raw, uint32_t flags)
{
    if (T.kind == kMsd)
        return (uint32_t)((to_ord(raw, T.dtype) >> T.shift) & (uint64_t)(T.fanout - 1u));
    const double v = model_F(M, raw, T.dtype) * T.scale;
    int64_t q = (int64_t)v - T.offset;
    q = q < 0 ? 0 : q;
    q = q > (int64_t)T.fanout - 1 ? (int64_t)T.fanout - 1 : q;
    uint32_t b = (uint32_t)q;
    if (flags & kFlagNonMonotone)        // test hook: break monotonicity on purpose
        b = (raw & 1u) ? (b + T.fanout / 2u) % T.fanout : b;
    return b;
}

// ------------------------------------------------------------ block scans --

// Exclusive scan of a[0..n) (LDS, u32) in place; returns the total.
// wsum: LDS scratch of blockDim/64 + 1 entries.
__device__ uint32_t block_scan_u32(uint32_t* a, uint32_t n, uint32_t* wsum)
{
    const uint32_t nt = blockDim.x;
    const uint32_t per = (n + nt - 1) / nt;
    const uint32_t lo = min(n, threadIdx.x * per), hi = min(n, lo + per);
    uint32_t s = 0;
    for (uint32_t i = lo; i < hi; ++i)
        s += a[i];
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
    if (threadIdx.x == 0) {
        uint32_t run = 0;
        for (uint32_t w = 0; w < nt / 64; ++w) {
            uint32_t v = wsum[w];
            wsum[w] = run;
            run += v;
        }
        wsum[nt / 64] = run;
    }
    __syncthreads();
    uint32_t base = wsum[wave] + x - s;
    for (uint32_t i = lo; i < hi; ++i) {
        uint32_t v = a[i];
        a[i] = base;
        base += v;
    }
    uint32_t total = wsum[nt / 64];
    __syncthreads();
    return total;
}

// ----------------------------------------------------------- model training --

constexpr uint32_t kSampleBlock = 2048;   // samples per training block

__device__ __forceinline__ uint32_t find_job(const ModelJob* jobs, uint32_t njobs, uint32_t blk)
{
    uint32_t lo = 0, hi = njobs;
    while (hi - lo > 1) {
        uint32_t mid = (lo + hi) >> 1;
        if (jobs[mid].block0 <= blk) lo = mid; else hi = mid;
    }
    return lo;
}

__global__ void k_train_init(const ModelJob* jobs, uint32_t njobs, uint64_t* minmax, uint32_t* lcnt,
                             uint64_t* lmin)
{
    const ModelJob J = jobs[blockIdx.x];
    if (threadIdx.x == 0) {
        minmax[2 * blockIdx.x] = ~0ull;
        minmax[2 * blockIdx.x + 1] = 0;
    }
    for (uint32_t k = threadIdx.x; k < J.leaves; k += blockDim.x) {
        lcnt[J.leaf_off + k] = 0;
        lmin[J.leaf_off + k] = ~0ull;
    }
}

// Gather the sample (order-preserving words) and reduce its finite range.
__global__ __launch_bounds__(256) void k_train_sample(const ModelJob* jobs, uint32_t njobs,
                                                      uint64_t* sample, uint64_t* minmax)
{
    __shared__ uint32_t s_job;
    __shared__ uint64_t s_lo[4], s_hi[4];
    if (threadIdx.x == 0)
        s_job = find_job(jobs, njobs, blockIdx.x);
    __syncthreads();
    const uint32_t j = s_job;
    const ModelJob J = jobs[j];
    const uint64_t t0 = (uint64_t)(blockIdx.x - J.block0) * kSampleBlock;
    uint64_t lo = ~0ull, hi = 0;
    for (uint32_t i = threadIdx.x; i < kSampleBlock; i += blockDim.x) {
        uint64_t t = t0 + i;
        if (t >= J.m)
            break;
        uint64_t raw = J.src[sample_index(J.seed, t, J.n)];
        uint64_t o = to_ord(raw, J.dtype);
        sample[J.sample_off + t] = o;
        if (!nonfinite(raw, J.dtype)) {
            lo = o < lo ? o : lo;
            hi = o > hi ? o : hi;
        }
    }
    for (uint32_t d = 32; d > 0; d >>= 1) {
        uint64_t a = __shfl_xor(lo, d, 64), b = __shfl_xor(hi, d, 64);
        lo = a < lo ? a : lo;
        hi = b > hi ? b : hi;
    }
    if ((threadIdx.x & 63u) == 0) {
        s_lo[threadIdx.x >> 6] = lo;
        s_hi[threadIdx.x >> 6] = hi;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (uint32_t w = 1; w < blockDim.x / 64; ++w) {
            lo = s_lo[w] < lo ? s_lo[w] : lo;
            hi = s_hi[w] > hi ? s_hi[w] : hi;
        }
        if (lo != ~0ull) {
            atomicMin((unsigned long long*)&minmax[2 * j], (unsigned long long)lo);
            atomicMax((unsigned long long*)&minmax[2 * j + 1], (unsigned long long)hi);
        }
    }
}

__device__ __forceinline__ void root_params(const uint64_t* minmax, uint32_t j, uint32_t dt, uint32_t L,
                                            double& xmin, double& xmax, double& rs, bool& any)
{
    uint64_t lo = minmax[2 * j], hi = minmax[2 * j + 1];
    any = lo != ~0ull;
    xmin = any ? ord_value(lo, dt) : 0.0;
    xmax = any ? ord_value(hi, dt) : 0.0;
    rs = (xmax > xmin) ? (double)L / (xmax - xmin) : 0.0;
}

__device__ __forceinline__ uint32_t root_leaf(double x, double xmin, double rs, uint32_t L)
{
    double t = (x - xmin) * rs;
    if (!(t >= 1.0))
        return 0;
    if (t >= (double)(L - 1u))
        return L - 1u;
    return (uint32_t)t;
}

// Per-leaf sample counts and minima, aggregated in LDS first.
__global__ __launch_bounds__(256) void k_train_leaves(const ModelJob* jobs, uint32_t njobs,
                                                      const uint64_t* sample, const uint64_t* minmax,
                                                      uint32_t* lcnt, uint64_t* lmin)
{
    __shared__ uint32_t s_job;
    __shared__ uint32_t c[kMaxLeaves];
    __shared__ unsigned long long mn[kMaxLeaves];
    if (threadIdx.x == 0)
        s_job = find_job(jobs, njobs, blockIdx.x);
    __syncthreads();
    const uint32_t j = s_job;
    const ModelJob J = jobs[j];
    const uint32_t L = J.leaves;
    for (uint32_t k = threadIdx.x; k < L; k += blockDim.x) {
        c[k] = 0;
        mn[k] = ~0ull;
    }
    double xmin, xmax, rs;
    bool any;
    root_params(minmax, j, J.dtype, L, xmin, xmax, rs, any);
    __syncthreads();
    const uint64_t t0 = (uint64_t)(blockIdx.x - J.block0) * kSampleBlock;
    for (uint32_t i = threadIdx.x; i < kSampleBlock; i += blockDim.x) {
        uint64_t t = t0 + i;
        if (t >= J.m)
            break;
        uint64_t o = sample[J.sample_off + t];
        uint64_t raw = from_ord(o, J.dtype);
        if (nonfinite(raw, J.dtype))
            continue;
        uint32_t k = root_leaf(key_value(raw, J.dtype), xmin, rs, L);
        atomicAdd(&c[k], 1u);
        atomicMin(&mn[k], (unsigned long long)o);
    }
    __syncthreads();
    for (uint32_t k = threadIdx.x; k < L; k += blockDim.x) {
        if (c[k]) {
            atomicAdd(&lcnt[J.leaf_off + k], c[k]);
            atomicMin((unsigned long long*)&lmin[J.leaf_off + k], mn[k]);
        }
    }
}

// Fit: knots at leaf minima with exact eCDF values, segments to the next knot.
__global__ __launch_bounds__(256) void k_train_fit(const ModelJob* jobs, const uint64_t* minmax,
                                                   const uint32_t* lcnt, const uint64_t* lmin,
                                                   double* models)
{
    __shared__ uint64_t below[kMaxLeaves];
    __shared__ uint16_t nxt[kMaxLeaves];
    __shared__ uint16_t prv[kMaxLeaves];
    __shared__ uint64_t s_total;
    const uint32_t j = blockIdx.x;
    const ModelJob J = jobs[j];
    const uint32_t L = J.leaves;
    const uint32_t* cnt = lcnt + J.leaf_off;
    if (threadIdx.x == 0) {
        uint64_t run = 0;
        uint32_t last = kNoPrev;
        for (uint32_t k = 0; k < L; ++k) {
            below[k] = run;
            run += cnt[k];
            prv[k] = (uint16_t)last;
            if (cnt[k])
                last = k;
        }
        s_total = run;
        uint32_t nx = kNoPrev;
        for (uint32_t k = L; k-- > 0;) {
            nxt[k] = (uint16_t)nx;
            if (cnt[k])
                nx = k;
        }
    }
    __syncthreads();
    const uint64_t mfin = s_total;
    double xmin, xmax, rs;
    bool any;
    root_params(minmax, j, J.dtype, L, xmin, xmax, rs, any);
    double* g = models + J.model_off;
    double* X = g + 4;
    double* y = X + L;
    double* yhi = y + L;
    double* s = yhi + L;
    uint32_t* prev = reinterpret_cast<uint32_t*>(s + L);
    if (threadIdx.x == 0) {
        g[0] = mfin ? xmin : 0.0;
        g[1] = mfin ? xmax : 0.0;
        g[2] = mfin ? rs : 0.0;
        g[3] = (double)mfin;
    }
    const double inf = __longlong_as_double(0x7ff0000000000000ll);
    for (uint32_t k = threadIdx.x; k < L; k += blockDim.x) {
        if (!mfin) {
            X[k] = inf;
            y[k] = 0.0;
            yhi[k] = 0.0;
            s[k] = 0.0;
            prev[k] = kNoPrev;
            continue;
        }
        const double yk = (double)below[k] / (double)mfin;
        // the previous knot below any key of leaf k that lies under X_k
        prev[k] = prv[k];
        if (!cnt[k]) {
            X[k] = inf;
            y[k] = yk;
            yhi[k] = yk;
            s[k] = 0.0;
            continue;
        }
        const double Xk = ord_value(lmin[J.leaf_off + k], J.dtype);
        double Xh = xmax, yh = 1.0;
        if (nxt[k] != kNoPrev) {
            const uint32_t q = nxt[k];
            Xh = ord_value(lmin[J.leaf_off + q], J.dtype);
            yh = (double)below[q] / (double)mfin;
        }
        double sl = (yh - yk) / (Xh - Xk);
        if (!(sl > 0.0) || __builtin_isinf(sl))
            sl = 0.0;
        X[k] = Xk;
        y[k] = yk;
        yhi[k] = yh;
        s[k] = sl;
    }
}

hipError_t launch_train(const ModelJob* d_jobs, uint32_t njobs, uint32_t total_blocks, uint64_t* d_sample,
                        uint64_t* d_minmax, uint32_t* d_lcnt, uint64_t* d_lmin, double* d_models,
                        hipStream_t st)
{
    if (!njobs)
        return hipSuccess;
    k_train_init<<<njobs, 256, 0, st>>>(d_jobs, njobs, d_minmax, d_lcnt, d_lmin);
    k_train_sample<<<total_blocks, 256, 0, st>>>(d_jobs, njobs, d_sample, d_minmax);
    k_train_leaves<<<total_blocks, 256, 0, st>>>(d_jobs, njobs, d_sample, d_minmax, d_lcnt, d_lmin);
    k_train_fit<<<njobs, 256, 0, st>>>(d_jobs, d_minmax, d_lcnt, d_lmin, d_models);
    return hipGetLastError();
}

// ------------------------------------------------------- partition rounds --

__device__ __forceinline__ uint32_t find_task(const Task* tasks, uint32_t ntasks, uint32_t chunk)
{
    uint32_t lo = 0, hi = ntasks;
    while (hi - lo > 1) {
        uint32_t mid = (lo + hi) >> 1;
        if (tasks[mid].chunk0 <= chunk) lo = mid; else hi = mid;
    }
    return lo;
}

__global__ void k_round_init(uint64_t* bstat, uint32_t nbuckets)
{
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nbuckets) {
        bstat[2 * i] = ~0ull;
        bstat[2 * i + 1] = 0;
    }
}

hipError_t launch_round_init(uint64_t* d_bstat, uint32_t nbuckets, hipStream_t st)
{
    if (nbuckets)
        k_round_init<<<(nbuckets + 255) / 256, 256, 0, st>>>(d_bstat, nbuckets);
    return hipGetLastError();
}

// Bucket sizes per (bucket, chunk) plus per-bucket min/max of the key words
// (Alg. 1 S_B, and the all-equal test of Alg. 2).
constexpr uint32_t kHistThreads = 256;
constexpr uint32_t kHistUnroll = 8;

__global__ __launch_bounds__(kHistThreads) void k_hist(const Task* tasks, uint32_t ntasks, uint64_t chunk,
                                                       const double* models, uint32_t* cnt, uint64_t* bstat,
                                                       uint32_t flags)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ uint32_t s_task;
    if (threadIdx.x == 0)
        s_task = find_task(tasks, ntasks, blockIdx.x);
    __syncthreads();
    const Task T = tasks[s_task];
    const uint32_t f = T.fanout;
    unsigned long long* mn = reinterpret_cast<unsigned long long*>(smem);
    unsigned long long* mx = mn + f;
    uint32_t* h = reinterpret_cast<uint32_t*>(mx + f);
    double* mlds = reinterpret_cast<double*>(smem + (size_t)f * 20 + ((f & 1u) ? 4 : 0));
    for (uint32_t b = threadIdx.x; b < f; b += blockDim.x) {
        h[b] = 0;
        mn[b] = ~0ull;
        mx[b] = 0;
    }
    SModel M{};
    if (T.kind != kMsd)
        load_model(M, models, T.model, T.leaves, mlds, reinterpret_cast<uint16_t*>(mlds + 4 * T.leaves));
    __syncthreads();
    const uint32_t lc = blockIdx.x - T.chunk0;
    const uint64_t lo = (uint64_t)lc * chunk;
    const uint64_t hi = min(T.n, lo + chunk);
    const uint64_t* src = (T.src ? T.scratch : T.keys) + T.start;
    for (uint64_t base = lo; base < hi; base += (uint64_t)kHistThreads * kHistUnroll) {
        uint64_t raw[kHistUnroll];
#pragma unroll
        for (uint32_t u = 0; u < kHistUnroll; ++u) {
            uint64_t i = base + u * kHistThreads + threadIdx.x;
            raw[u] = i < hi ? src[i] : 0;
        }
#pragma unroll
        for (uint32_t u = 0; u < kHistUnroll; ++u) {
            uint64_t i = base + u * kHistThreads + threadIdx.x;
            if (i < hi) {
                uint32_t b = bucket_of(T, M, raw[u], flags);
                uint64_t o = to_ord(raw[u], T.dtype);
                atomicAdd(&h[b], 1u);
                atomicMin(&mn[b], (unsigned long long)o);
                atomicMax(&mx[b], (unsigned long long)o);
            }
        }
    }
    __syncthreads();
    for (uint32_t b = threadIdx.x; b < f; b += blockDim.x) {
        cnt[T.cnt_off + (uint64_t)b * T.nchunks + lc] = h[b];
        if (h[b]) {
            atomicMin((unsigned long long*)&bstat[2 * ((uint64_t)T.bucket_off + b)], mn[b]);
            atomicMax((unsigned long long*)&bstat[2 * ((uint64_t)T.bucket_off + b) + 1], mx[b]);
        }
    }
}

static size_t model_lds_bytes(uint32_t L) { return (size_t)L * 34 + 16; }

hipError_t launch_hist(const Task* d_tasks, uint32_t ntasks, uint32_t total_chunks, uint64_t chunk,
                       const double* d_models, uint32_t* d_cnt, uint64_t* d_bstat, uint32_t max_fanout,
                       uint32_t max_leaves, uint32_t flags, hipStream_t st)
{
    size_t smem = (size_t)max_fanout * 20 + 8 + model_lds_bytes(max_leaves);
    k_hist<<<total_chunks, kHistThreads, smem, st>>>(d_tasks, ntasks, chunk, d_models, d_cnt, d_bstat, flags);
    return hipGetLastError();
}

// Exclusive scan of u32 counts into u64 positions: block sums, a scan of the
// block sums, then each block rescans with its offset.
constexpr uint32_t kScanBlock = 4096;

__global__ __launch_bounds__(256) void k_scan_reduce(const uint32_t* in, uint64_t n, uint64_t* sums)
{
    __shared__ uint64_t ws[4];
    uint64_t base = (uint64_t)blockIdx.x * kScanBlock;
    uint64_t s = 0;
    for (uint32_t i = threadIdx.x; i < kScanBlock; i += 256) {
        uint64_t k = base + i;
        if (k < n)
            s += in[k];
    }
    for (uint32_t d = 32; d > 0; d >>= 1)
        s += __shfl_xor(s, d, 64);
    if ((threadIdx.x & 63u) == 0)
        ws[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0)
        sums[blockIdx.x] = ws[0] + ws[1] + ws[2] + ws[3];
}

__global__ __launch_bounds__(1024) void k_scan_top(uint64_t* sums, uint32_t nb)
{
    __shared__ uint64_t ws[17];
    const uint32_t per = (nb + 1023) / 1024;
    const uint32_t lo = min(nb, threadIdx.x * per), hi = min(nb, lo + per);
    uint64_t s = 0;
    for (uint32_t i = lo; i < hi; ++i)
        s += sums[i];
    const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
    uint64_t x = s;
    for (uint32_t d = 1; d < 64; d <<= 1) {
        uint64_t y = __shfl_up(x, d, 64);
        if (lane >= d)
            x += y;
    }
    if (lane == 63)
        ws[wave] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t run = 0;
        for (uint32_t w = 0; w < 16; ++w) {
            uint64_t v = ws[w];
            ws[w] = run;
            run += v;
        }
    }
    __syncthreads();
    uint64_t b = ws[wave] + x - s;
    for (uint32_t i = lo; i < hi; ++i) {
        uint64_t v = sums[i];
        sums[i] = b;
        b += v;
    }
}

__global__ __launch_bounds__(256) void k_scan_down(const uint32_t* in, uint64_t n, const uint64_t* sums,
                                                   uint64_t* out)
{
    __shared__ uint64_t ws[5];
    const uint64_t base = (uint64_t)blockIdx.x * kScanBlock;
    constexpr uint32_t per = kScanBlock / 256;
    uint32_t v[per];
    uint64_t s = 0;
#pragma unroll
    for (uint32_t i = 0; i < per; ++i) {
        uint64_t k = base + (uint64_t)threadIdx.x * per + i;
        v[i] = k < n ? in[k] : 0u;
        s += v[i];
    }
    const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
    uint64_t x = s;
    for (uint32_t d = 1; d < 64; d <<= 1) {
        uint64_t y = __shfl_up(x, d, 64);
        if (lane >= d)
            x += y;
    }
    if (lane == 63)
        ws[wave] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t run = sums[blockIdx.x];
        for (uint32_t w = 0; w < 4; ++w) {
            uint64_t t = ws[w];
            ws[w] = run;
            run += t;
        }
    }
    __syncthreads();
    uint64_t b = ws[wave] + x - s;
#pragma unroll
    for (uint32_t i = 0; i < per; ++i) {
        uint64_t k = base + (uint64_t)threadIdx.x * per + i;
        if (k < n)
            out[k] = b;
        b += v[i];
    }
}

size_t scan_tmp_entries(uint64_t n) { return (size_t)((n + kScanBlock - 1) / kScanBlock) + 1; }

hipError_t launch_scan(const uint32_t* d_in, uint64_t* d_out, uint64_t n, uint64_t* d_tmp, hipStream_t st)
{
    uint32_t nb = (uint32_t)((n + kScanBlock - 1) / kScanBlock);
    if (!nb)
        return hipSuccess;
    k_scan_reduce<<<nb, 256, 0, st>>>(d_in, n, d_tmp);
    k_scan_top<<<1, 1024, 0, st>>>(d_tmp, nb);
    k_scan_down<<<nb, 256, 0, st>>>(d_in, n, d_tmp, d_out);
    return hipGetLastError();
}

// Classify every bucket of a task: empty, all-equal (filled with its value,
// never moved again), small (grouped with its neighbours for the LDS base
// case) or over-full (a task of the next round).
enum : uint8_t { kEmpty = 0, kSmall = 1, kFillB = 2, kBig = 3 };

__global__ __launch_bounds__(256) void k_classify(const Task* tasks, const uint64_t* pos, const uint64_t* bstat,
                                                  uint32_t base_cap, uint32_t param_fanout, Task* next,
                                                  Group* groups, Fill* fills, uint8_t* skip,
                                                  uint32_t* task_flags, RoundCtl* ctl)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const Task T = tasks[blockIdx.x];
    const uint32_t f = T.fanout;
    uint64_t* bst = reinterpret_cast<uint64_t*>(smem);     // bucket start (task-relative)
    uint64_t* bsz = bst + f;                                // bucket size
    uint32_t* item = reinterpret_cast<uint32_t*>(bsz + f);  // per bucket: list slot
    uint32_t* gsize = item + f;                             // group size by leader bucket
    uint8_t* kind = reinterpret_cast<uint8_t*>(gsize + f);
    __shared__ uint32_t s_ng, s_nt, s_nf, s_nfb, s_gb, s_tb, s_fb, s_noprog;
    __shared__ unsigned long long s_fkeys;
    const uint32_t fill_min = base_cap / 8u > 2u ? base_cap / 8u : 2u;
    for (uint32_t b = threadIdx.x; b < f; b += blockDim.x) {
        uint64_t s0 = pos[T.cnt_off + (uint64_t)b * T.nchunks] - T.cnt_base;
        uint64_t s1 = (b + 1 < f) ? pos[T.cnt_off + (uint64_t)(b + 1) * T.nchunks] - T.cnt_base : T.n;
        uint64_t sz = s1 - s0;
        uint64_t lo = bstat[2 * ((uint64_t)T.bucket_off + b)];
        uint64_t hi = bstat[2 * ((uint64_t)T.bucket_off + b) + 1];
        uint8_t k;
        if (sz == 0)
            k = kEmpty;
        else if (lo == hi && sz >= fill_min)
            k = kFillB;
        else if (lo != hi && sz > base_cap)
            k = kBig;
        else
            k = kSmall;
        bst[b] = s0;
        bsz[b] = sz;
        kind[b] = k;
        skip[(uint64_t)T.bucket_off + b] = (k == kFillB);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        // Greedy walk: runs of small buckets up to base_cap keys form groups.
        uint32_t ng = 0, nt = 0, nf = 0, nfb = 0, noprog = 0;
        uint64_t fkeys = 0, gkeys = 0;
        int32_t open = -1;
        uint64_t osz = 0;
        for (uint32_t b = 0; b < f; ++b) {
            uint8_t k = kind[b];
            if (k == kEmpty)
                continue;
            if (k == kSmall) {
                gkeys += bsz[b];
                if (open >= 0 && osz + bsz[b] <= base_cap) {
                    osz += bsz[b];
                    item[b] = ~0u;
                    continue;
                }
                if (open >= 0)
                    gsize[open] = (uint32_t)osz;
                open = (int32_t)b;
                osz = bsz[b];
                item[b] = ng++;
                continue;
            }
            if (open >= 0) {
                gsize[open] = (uint32_t)osz;
                open = -1;
            }
            if (k == kFillB) {
                item[b] = nf;
                nf += (uint32_t)((bsz[b] + kFillPiece - 1) / kFillPiece);
                nfb += 1;
                fkeys += bsz[b];
            } else {
                item[b] = nt++;
                if (bsz[b] == T.n)
                    noprog = 1;
            }
        }
        if (open >= 0)
            gsize[open] = (uint32_t)osz;
        s_ng = ng;
        s_nt = nt;
        s_nf = nf;
        s_nfb = nfb;
        s_fkeys = fkeys;
        s_noprog = noprog;
        s_gb = ng ? atomicAdd(&ctl->ngroups, ng) : 0;
        s_tb = nt ? atomicAdd(&ctl->ntasks, nt) : 0;
        s_fb = nf ? atomicAdd(&ctl->nfill, nf) : 0;
        if (nfb) {
            atomicAdd(&ctl->nfillbuckets, nfb);
            atomicAdd((unsigned long long*)&ctl->fillkeys, (unsigned long long)fkeys);
        }
        if (gkeys)
            atomicAdd((unsigned long long*)&ctl->group_keys, (unsigned long long)gkeys);
        if (noprog)
            atomicAdd((unsigned long long*)&ctl->stall_keys, (unsigned long long)T.n);
        task_flags[blockIdx.x] = noprog ? kNoScatter : 0u;
    }
    __syncthreads();
    const uint32_t noprog = s_noprog;
    // Where the keys of this round's buckets live after the scatter.
    uint64_t* moved = (T.src ? T.keys : T.scratch) + T.start;
    const uint32_t lf = 31u - __clz(param_fanout);
    for (uint32_t b = threadIdx.x; b < f; b += blockDim.x) {
        uint8_t k = kind[b];
        if (k == kSmall && item[b] != ~0u) {
            Group G;
            G.src = moved + bst[b];
            G.dst = T.keys + T.start + bst[b];
            G.start = T.start + bst[b];
            G.n = gsize[b];
            G.dtype = T.dtype;
            groups[s_gb + item[b]] = G;
        } else if (k == kFillB) {
            uint64_t raw = from_ord(bstat[2 * ((uint64_t)T.bucket_off + b)], T.dtype);
            uint64_t sz = bsz[b];
            uint32_t np = (uint32_t)((sz + kFillPiece - 1) / kFillPiece);
            for (uint32_t p = 0; p < np; ++p) {
                Fill F;
                uint64_t off = (uint64_t)p * kFillPiece;
                F.dst = T.keys + T.start + bst[b] + off;
                F.raw = raw;
                F.start = T.start + bst[b] + off;
                F.n = (uint32_t)min((uint64_t)kFillPiece, sz - off);
                F.dtype = T.dtype;
                fills[s_fb + item[b] + p] = F;
            }
        } else if (k == kBig) {
            Task C = T;
            C.start = T.start + bst[b];
            C.n = bsz[b];
            C.src = noprog ? T.src : 1u - T.src;
            C.level = T.level + 1;
            C.chunk0 = C.nchunks = C.bucket_off = 0;
            C.cnt_off = C.cnt_base = 0;
            const uint64_t lo = bstat[2 * ((uint64_t)T.bucket_off + b)];
            const uint64_t hi = bstat[2 * ((uint64_t)T.bucket_off + b) + 1];
            const bool stalled = noprog || (T.kind == kLocal && bsz[b] > T.n - T.n / 8u);
            if (T.kind == kGlobal) {
                C.kind = kGlobalL1;
                C.scale = (double)f * (double)f;
                C.offset = (int64_t)b * (int64_t)f;
            } else if (T.kind == kLocal && stalled) {
                // no model progress: split on the highest differing bit
                uint32_t d = 63u - (uint32_t)__clzll((long long)(lo ^ hi));
                uint32_t bits = lf < d + 1 ? lf : d + 1;
                bits = bits ? bits : 1;
                C.kind = kMsd;
                C.fanout = 1u << bits;
                C.shift = d + 1 - bits;
                C.scale = 0.0;
                C.offset = 0;
                atomicAdd(&ctl->fallbacks, 1u);
            } else {
                C.kind = kLocal;       // model trained on the range before the next round
                C.fanout = param_fanout;
                C.scale = (double)param_fanout;
                C.offset = 0;
            }
            next[s_tb + item[b]] = C;
        }
    }
}

hipError_t launch_classify(const Task* d_tasks, uint32_t ntasks, const uint64_t* d_pos, const uint64_t* d_bstat,
                           uint32_t base_cap, uint32_t param_fanout, Task* d_next, Group* d_groups, Fill* d_fills,
                           uint8_t* d_skip, uint32_t* d_task_flags, RoundCtl* d_ctl, uint32_t max_fanout,
                           hipStream_t st)
{
    size_t smem = (size_t)max_fanout * (8 + 8 + 4 + 4 + 1) + 16;
    k_classify<<<ntasks, 256, smem, st>>>(d_tasks, d_pos, d_bstat, base_cap, param_fanout, d_next, d_groups,
                                          d_fills, d_skip, d_task_flags, d_ctl);
    return hipGetLastError();
}

// Scatter: stage one tile in LDS ordered by bucket, then write each bucket's
// run at its cursor so consecutive lanes write consecutive addresses.
constexpr uint32_t kScatterThreads = 256;

template <uint32_t KPT>
__global__ __launch_bounds__(kScatterThreads) void k_scatter(const Task* tasks, uint32_t ntasks, uint64_t chunk,
                                                             const double* models, const uint64_t* pos,
                                                             const uint8_t* skip, const uint32_t* task_flags,
                                                             uint32_t flags)
{
    constexpr uint32_t TILE = KPT * kScatterThreads;
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ uint32_t s_task;
    __shared__ uint32_t wsum[kScatterThreads / 64 + 1];
    if (threadIdx.x == 0)
        s_task = find_task(tasks, ntasks, blockIdx.x);
    __syncthreads();
    const uint32_t ti = s_task;
    if (task_flags[ti] & kNoScatter)
        return;
    const Task T = tasks[ti];
    const uint32_t f = T.fanout;
    uint64_t* stage = reinterpret_cast<uint64_t*>(smem);
    uint64_t* cur = stage + TILE;
    uint32_t* tcnt = reinterpret_cast<uint32_t*>(cur + f);
    uint32_t* tstart = tcnt + f;
    uint16_t* sb = reinterpret_cast<uint16_t*>(tstart + f);
    double* mlds = reinterpret_cast<double*>(smem + (size_t)TILE * 10 + (size_t)f * 16 + 16);
    const uint32_t lc = blockIdx.x - T.chunk0;
    for (uint32_t b = threadIdx.x; b < f; b += blockDim.x) {
        uint64_t c = pos[T.cnt_off + (uint64_t)b * T.nchunks + lc] - T.cnt_base;
        cur[b] = skip[(uint64_t)T.bucket_off + b] ? (c | kSkipBit) : c;
        tcnt[b] = 0;
    }
    SModel M{};
    if (T.kind != kMsd)
        load_model(M, models, T.model, T.leaves, mlds, reinterpret_cast<uint16_t*>(mlds + 4 * T.leaves));
    __syncthreads();
    const uint64_t lo = (uint64_t)lc * chunk;
    const uint64_t hi = min(T.n, lo + chunk);
    const uint64_t* src = (T.src ? T.scratch : T.keys) + T.start;
    uint64_t* dst = (T.src ? T.keys : T.scratch) + T.start;
    for (uint64_t base = lo; base < hi; base += TILE) {
        uint64_t raw[KPT];
        uint32_t bk[KPT];
        uint32_t rk[KPT];
#pragma unroll
        for (uint32_t u = 0; u < KPT; ++u) {
            uint64_t i = base + u * kScatterThreads + threadIdx.x;
            raw[u] = i < hi ? src[i] : 0;
        }
#pragma unroll
        for (uint32_t u = 0; u < KPT; ++u) {
            uint64_t i = base + u * kScatterThreads + threadIdx.x;
            bk[u] = ~0u;
            if (i < hi) {
                uint32_t b = bucket_of(T, M, raw[u], flags);
                if (!(cur[b] & kSkipBit)) {
                    bk[u] = b;
                    rk[u] = atomicAdd(&tcnt[b], 1u);
                }
            }
        }
        __syncthreads();
        for (uint32_t b = threadIdx.x; b < f; b += blockDim.x)
            tstart[b] = tcnt[b];
        __syncthreads();
        const uint32_t ntile = block_scan_u32(tstart, f, wsum);
#pragma unroll
        for (uint32_t u = 0; u < KPT; ++u) {
            if (bk[u] != ~0u) {
                uint32_t p = tstart[bk[u]] + rk[u];
                stage[p] = raw[u];
                sb[p] = (uint16_t)bk[u];
            }
        }
        __syncthreads();
        for (uint32_t p = threadIdx.x; p < ntile; p += kScatterThreads) {
            uint32_t b = sb[p];
            dst[cur[b] + (p - tstart[b])] = stage[p];
        }
        __syncthreads();
        for (uint32_t b = threadIdx.x; b < f; b += blockDim.x) {
            cur[b] += tcnt[b];
            tcnt[b] = 0;
        }
        __syncthreads();
    }
}

hipError_t launch_scatter(const Task* d_tasks, uint32_t ntasks, uint32_t total_chunks, uint64_t chunk,
                          const double* d_models, const uint64_t* d_pos, const uint8_t* d_skip,
                          const uint32_t* d_task_flags, uint32_t tile, uint32_t max_fanout, uint32_t max_leaves,
                          uint32_t flags, hipStream_t st)
{
    size_t smem = (size_t)tile * 10 + (size_t)max_fanout * 16 + 16 + model_lds_bytes(max_leaves);
    switch (tile) {
    case 1024:
        k_scatter<4><<<total_chunks, kScatterThreads, smem, st>>>(d_tasks, ntasks, chunk, d_models, d_pos, d_skip,
                                                                  d_task_flags, flags);
        break;
    case 2048:
        k_scatter<8><<<total_chunks, kScatterThreads, smem, st>>>(d_tasks, ntasks, chunk, d_models, d_pos, d_skip,
                                                                  d_task_flags, flags);
        break;
    case 4096:
        k_scatter<16><<<total_chunks, kScatterThreads, smem, st>>>(d_tasks, ntasks, chunk, d_models, d_pos, d_skip,
                                                                   d_task_flags, flags);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ------------------------------------------------------------- base case --

// Sort one group (<= base_cap keys) in LDS: bitonic network over the next
// power of two, padded with the largest word.
constexpr uint32_t kBaseThreads = 512;

__global__ __launch_bounds__(kBaseThreads) void k_base(const Group* groups)
{
    extern __shared__ __align__(16) unsigned char smem[];
    uint64_t* s = reinterpret_cast<uint64_t*>(smem);
    const Group G = groups[blockIdx.x];
    const uint32_t n = G.n;
    uint32_t N = 2;
    while (N < n)
        N <<= 1;
    for (uint32_t i = threadIdx.x; i < N; i += kBaseThreads)
        s[i] = i < n ? to_ord(G.src[i], G.dtype) : ~0ull;
    __syncthreads();
    for (uint32_t k = 2; k <= N; k <<= 1) {
        for (uint32_t j = k >> 1; j > 0; j >>= 1) {
            for (uint32_t i = threadIdx.x; i < N; i += kBaseThreads) {
                uint32_t l = i ^ j;
                if (l > i) {
                    uint64_t a = s[i], b = s[l];
                    bool up = (i & k) == 0;
                    if ((a > b) == up) {
                        s[i] = b;
                        s[l] = a;
                    }
                }
            }
            __syncthreads();
        }
    }
    for (uint32_t i = threadIdx.x; i < n; i += kBaseThreads)
        G.dst[i] = from_ord(s[i], G.dtype);
}

hipError_t launch_base(const Group* d_groups, uint32_t ngroups, uint32_t base_cap, hipStream_t st)
{
    if (!ngroups)
        return hipSuccess;
    uint32_t N = 2;
    while (N < base_cap)
        N <<= 1;
    k_base<<<ngroups, kBaseThreads, (size_t)N * 8, st>>>(d_groups);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_fill(const Fill* fills)
{
    const Fill F = fills[blockIdx.x];
    for (uint32_t i = threadIdx.x; i < F.n; i += 256)
        F.dst[i] = F.raw;
}

hipError_t launch_fill(const Fill* d_fills, uint32_t nfill, hipStream_t st)
{
    if (nfill)
        k_fill<<<nfill, 256, 0, st>>>(d_fills);
    return hipGetLastError();
}

// Touch-up check (Alg. 2's final pass): every final range is sorted by
// construction, so only the seam with the preceding range can be out of
// order.  `full` also rechecks every adjacent pair inside the groups.
__global__ __launch_bounds__(256) void k_touchup(const Group* groups, uint32_t ngroups, const Fill* fills,
                                                 uint32_t nfill, RoundCtl* ctl)
{
    uint32_t i = blockIdx.x * 256 + threadIdx.x;
    const uint64_t* p;
    uint64_t start;
    uint32_t dt;
    if (i < ngroups) {
        p = groups[i].dst;
        start = groups[i].start;
        dt = groups[i].dtype;
    } else if (i < ngroups + nfill) {
        p = fills[i - ngroups].dst;
        start = fills[i - ngroups].start;
        dt = fills[i - ngroups].dtype;
    } else {
        return;
    }
    if (start > 0 && to_ord(p[-1], dt) > to_ord(p[0], dt))
        atomicAdd(&ctl->violations, 1u);
}

__global__ __launch_bounds__(256) void k_touchup_full(const Group* groups, RoundCtl* ctl)
{
    const Group G = groups[blockIdx.x];
    uint32_t bad = 0;
    for (uint32_t i = threadIdx.x + 1; i < G.n; i += 256)
        bad += to_ord(G.dst[i - 1], G.dtype) > to_ord(G.dst[i], G.dtype);
    if (bad)
        atomicAdd(&ctl->violations, bad);
}

hipError_t launch_touchup(const Group* d_groups, uint32_t ngroups, const Fill* d_fills, uint32_t nfill, int full,
                          RoundCtl* d_ctl, hipStream_t st)
{
    uint32_t items = ngroups + nfill;
    if (items)
        k_touchup<<<(items + 255) / 256, 256, 0, st>>>(d_groups, ngroups, d_fills, nfill, d_ctl);
    if (full && ngroups)
        k_touchup_full<<<ngroups, 256, 0, st>>>(d_groups, d_ctl);
    return hipGetLastError();
}

}  // namespace lsort
