// Model training on the device (Sec. 6.1: two layers, 1% sample; the
// procedure itself is reading R14 of the model):
//   k_train_runs       gather each job's sample as order-preserving words in
//                      runs of kSampleBlock, count its non-finite words, and
//                      sort each run in LDS
//   k_train_merge      merge passes: every word moves to its rank in the
//                      merged pair of runs (its index plus its count in the
//                      other run), so a pass is one gather-free scatter
//   k_train_modes      per leaf: its most repeated value (longest run of equal
//                      values, the smallest on ties) and its first sample
//   k_train_fit        knots (the most repeated value of a leaf when it holds
//                      2+ copies and 1/L of the sample, else the leaf's
//                      smallest value), mid-ranks, segments; tables to zero
//   k_train_small      all of the above in one workgroup per job, when every
//                      sample fits one run (the sample and tables in LDS)
// The per-leaf tables (best, first) and the per-job non-finite counts start
// and end at zero.
#include "lsort_device.h"

#pragma clang fp contract(off)

namespace lsort {

constexpr uint64_t kOrdNegInf = 0x000fffffffffffffull;   // order word of -inf
constexpr uint64_t kOrdPosInf = 0xfff0000000000000ull;   // order word of +inf

// Job of training block blk (jobs sorted by block0).
__device__ __forceinline__ uint32_t find_job(const ModelJob* jobs, uint32_t njobs, uint32_t blk)
{
    uint32_t lo = 0, hi = njobs;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (jobs[mid].block0 <= blk) lo = mid; else hi = mid;
    }
    return lo;
}

// Job owning sample word g (jobs sorted by sample_off).
__device__ __forceinline__ uint32_t find_job_of(const ModelJob* jobs, uint32_t njobs, uint64_t g)
{
    uint32_t lo = 0, hi = njobs;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (jobs[mid].sample_off <= g) lo = mid; else hi = mid;
    }
    return lo;
}

// Finite part [lo, hi) of a job's sorted sample: its non-finite words sit
// at both ends, nf[0] of them up to -inf's word and nf[1] from +inf's.
__device__ __forceinline__ void finite_range(const uint64_t* nf, uint64_t m, uint64_t& lo, uint64_t& hi)
{
    lo = nf[0];
    hi = m - nf[1];
}

// First index in [a, b) whose value exceeds x (values non-decreasing).
__device__ inline uint64_t value_upper(const uint64_t* S, uint64_t a, uint64_t b, double x, uint32_t dt)
{
    while (a < b) {
        const uint64_t mid = (a + b) >> 1;
        if (ord_value(S[mid], dt) > x) b = mid; else a = mid + 1;
    }
    return a;
}

struct Root {
    double xmin, xmax, r0, rs;
};

// Root of a sample whose finite values run from xmin to xmax.
__device__ inline Root root_from(double xmin, double xmax, uint32_t L)
{
    Root R;
    R.xmin = xmin;
    R.xmax = xmax;
    R.r0 = root_coord(R.xmin);
    const double r1 = root_coord(R.xmax);
    R.rs = r1 > R.r0 ? (double)L / (r1 - R.r0) : 0.0;
    return R;
}

__device__ inline Root root_of(const uint64_t* S, uint64_t lo, uint64_t hi, uint32_t dt, uint32_t L)
{
    return root_from(ord_value(S[lo], dt), ord_value(S[hi - 1], dt), L);
}

__device__ __forceinline__ uint32_t root_leaf(double x, const Root& R, uint32_t L)
{
    const double t = (root_coord(x) - R.r0) * R.rs;
    if (!(t >= 1.0))
        return 0;
    if (t >= (double)(L - 1u))
        return L - 1u;
    return (uint32_t)t;
}

// Gather one run of up to kSampleBlock sample words (16 independent loads
// per lane) into LDS, count the non-finite ones (f64), sort the run.
__global__ __launch_bounds__(256) void k_train_runs(const ModelJob* jobs, uint32_t njobs, uint64_t* sample,
                                                    uint64_t* nf, const LiveCounts* live)
{
    if (live) {
        if (blockIdx.x >= live->blocks)
            return;
        njobs = live->njobs;
    }
    extern __shared__ __align__(16) unsigned char smem[];
    uint64_t* s = reinterpret_cast<uint64_t*>(smem);
    __shared__ uint32_t s_job;
    __shared__ uint32_t s_nf[2];
    if (threadIdx.x == 0) {
        s_job = find_job(jobs, njobs, blockIdx.x);
        s_nf[0] = s_nf[1] = 0;
    }
    __syncthreads();
    const uint32_t j = s_job;
    const ModelJob J = jobs[j];
    const uint64_t t0 = (uint64_t)(blockIdx.x - J.block0) * kSampleBlock;
    if (t0 >= J.m)
        return;
    const uint32_t n = (uint32_t)min((uint64_t)kSampleBlock, J.m - t0);
    uint32_t logN = 4;
    while ((1u << logN) < n)
        ++logN;
    constexpr uint32_t U = kSampleBlock / 256;
    uint64_t raw[U];
#pragma unroll
    for (uint32_t u = 0; u < U; ++u) {
        const uint32_t i = u * 256 + threadIdx.x;
        raw[u] = i < n ? as_global<const uint64_t>(J.src)[sample_index(J.seed, t0 + i, J.n)] : 0;
    }
    uint32_t neg = 0, pos = 0;
#pragma unroll
    for (uint32_t u = 0; u < U; ++u) {
        const uint32_t i = u * 256 + threadIdx.x;
        if (i < (1u << logN)) {
            const uint64_t w = i < n ? to_ord(raw[u], J.dtype) : ~0ull;
            s[base_pad(i)] = w;
            if (i < n && J.dtype == kF64) {
                neg += w <= kOrdNegInf;
                pos += w >= kOrdPosInf;
            }
        }
    }
    if (neg)
        atomicAdd(&s_nf[0], neg);
    if (pos)
        atomicAdd(&s_nf[1], pos);
    __syncthreads();
    if (threadIdx.x == 0) {
        if (s_nf[0])
            atomicAdd((unsigned long long*)&nf[2 * j], (unsigned long long)s_nf[0]);
        if (s_nf[1])
            atomicAdd((unsigned long long*)&nf[2 * j + 1], (unsigned long long)s_nf[1]);
    }
    lds_bitonic<256>(s, logN);
    uint64_t* run = sample + J.sample_off + t0;
    for (uint32_t i = threadIdx.x; i < n; i += 256)
        run[i] = s[base_pad(i)];
}

// One merge pass: runs of w words (sorted) become runs of 2w.  A word of the
// left run lands after the right run's smaller words, a word of the right run
// after the left run's words not above it, so equal words keep their order.
__global__ __launch_bounds__(256) void k_train_merge(const ModelJob* jobs, uint32_t njobs, const uint64_t* src,
                                                     uint64_t* dst, uint64_t w, uint64_t total, const LiveCounts* live)
{
    if (live) {
        njobs = live->njobs;
        total = live->samples;
    }
    const uint64_t g = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    if (g >= total)
        return;
    const ModelJob J = jobs[find_job_of(jobs, njobs, g)];
    const uint64_t t = g - J.sample_off;
    if (t >= J.m)
        return;
    const uint64_t* S = src + J.sample_off;
    const uint64_t p0 = t / (2 * w) * (2 * w);
    const uint64_t a1 = min(p0 + w, J.m), b1 = min(p0 + 2 * w, J.m);
    const uint64_t x = S[t];
    uint64_t pos;
    if (t < a1) {
        uint64_t lo = a1, hi = b1;                 // right-run words below x
        while (lo < hi) {
            const uint64_t mid = (lo + hi) >> 1;
            if (S[mid] < x) lo = mid + 1; else hi = mid;
        }
        pos = t + (lo - a1);
    } else {
        uint64_t lo = p0, hi = a1;                 // left-run words not above x
        while (lo < hi) {
            const uint64_t mid = (lo + hi) >> 1;
            if (S[mid] <= x) lo = mid + 1; else hi = mid;
        }
        pos = (t - a1) + lo;
    }
    dst[J.sample_off + pos] = x;
}

// The runs of equal values among the finite sample words [a, a + nv) (word
// a + i has value val(i + 1); val(0) is the word before a, NaN when a is the
// first finite word): each lane walks kSampleBlock / 256 consecutive words,
// and a run that reaches past the lane's range is searched for among the
// block's words, then past them with beyond(x).  Per leaf the longest run
// goes to s_best as (length << 32 | ~start) and the first run to s_first as
// (~start << 32 | length), starts relative to lo.
template <typename Val, typename Beyond>
__device__ __forceinline__ void modes_runs(const Val& val, uint32_t nv, uint64_t a, uint64_t lo, const Root& R,
                                           uint32_t L, unsigned long long* s_best, unsigned long long* s_first,
                                           const Beyond& beyond)
{
    constexpr uint32_t kPer = kSampleBlock / 256;
    const uint32_t r0 = threadIdx.x * kPer;
    const uint32_t r1 = min(r0 + kPer, nv);
    for (uint32_t i = r0; i < r1;) {
        const double x = val[i + 1];
        uint32_t e = i + 1;
        while (e < r1 && val[e + 1] == x)
            ++e;
        if (!(val[i] == x)) {                          // a run starts here (NaN before lo)
            uint64_t end = a + e;
            if (e == r1) {
                uint32_t l = r1, h = nv;
                while (l < h) {
                    const uint32_t mid = (l + h) >> 1;
                    if (val[mid + 1] > x) h = mid; else l = mid + 1;
                }
                end = l < nv ? a + l : beyond(x);
            }
            const uint32_t k = root_leaf(x, R, L);
            const uint64_t rel = a + i - lo, len = end - (a + i);
            atomicMax(&s_best[k], (unsigned long long)((len << 32) | (0xffffffffull - rel)));
            atomicMax(&s_first[k], (unsigned long long)(((0xffffffffull - rel) << 32) | len));
        }
        i = e;
    }
}

// Per leaf: the longest run of equal values as (length << 32 | ~start) and
// the first run as (~start << 32 | length), both reduced with atomicMax in
// LDS before the global atomics.  The block's sorted words are staged in LDS
// and each lane walks 16 consecutive ones; only a run that reaches past the
// lane's range is searched for in global memory.
__global__ __launch_bounds__(256) void k_train_modes(const ModelJob* jobs, uint32_t njobs, const uint64_t* sorted,
                                                     uint64_t* best, uint64_t* firstc, const uint64_t* nf,
                                                     const LiveCounts* live)
{
    if (live) {
        if (blockIdx.x >= live->blocks)
            return;
        njobs = live->njobs;
    }
    __shared__ uint32_t s_job;
    __shared__ unsigned long long s_best[kMaxLeaves], s_first[kMaxLeaves];
    __shared__ double s_val[kSampleBlock + 1];
    __shared__ uint64_t s_lo, s_hi;
    if (threadIdx.x == 0) {
        s_job = find_job(jobs, njobs, blockIdx.x);
        uint64_t lo, hi;
        finite_range(nf + 2 * s_job, jobs[s_job].m, lo, hi);
        s_lo = lo;
        s_hi = hi;
    }
    __syncthreads();
    const ModelJob J = jobs[s_job];
    const uint32_t L = J.leaves;
    const uint64_t lo = s_lo, hi = s_hi;
    const uint64_t t0 = (uint64_t)(blockIdx.x - J.block0) * kSampleBlock;
    const uint64_t a = max(t0, lo), b = min(t0 + kSampleBlock, hi);
    if (a >= b)
        return;                                        // the whole block leaves together
    const uint64_t* S = sorted + J.sample_off;
    // s_val[i] = value of word a - 1 + i (i = 0 is the word before the range)
    const uint32_t nv = (uint32_t)(b - a);
    for (uint32_t i = threadIdx.x; i <= nv; i += 256) {
        const uint64_t t = a + i - 1;
        s_val[i] = (i == 0 && a == lo) ? __longlong_as_double(0x7ff8000000000000ll) : ord_value(S[t], J.dtype);
    }
    for (uint32_t k = threadIdx.x; k < L; k += 256) {
        s_best[k] = 0;
        s_first[k] = 0;
    }
    const Root R = root_of(S, lo, hi, J.dtype, L);
    __syncthreads();
    modes_runs(s_val, nv, a, lo, R, L, s_best, s_first,
               [&](double x) { return value_upper(S, a + nv, hi, x, J.dtype); });
    __syncthreads();
    for (uint32_t k = threadIdx.x; k < L; k += 256) {
        if (s_best[k]) {
            atomicMax((unsigned long long*)&best[J.leaf_off + k], s_best[k]);
            atomicMax((unsigned long long*)&firstc[J.leaf_off + k], s_first[k]);
        }
    }
}

// Knots and segments of one model from its leaf tables: best(k) and
// first(k) as the runs kernel leaves them (0: empty leaf), val(i) the i-th
// finite sample value (i < mfin).  prv / nxt: the exclusive max / reversed
// min scans of the non-empty leaves; run0: length of the first run; kB / kd:
// LDS scratch of L entries.
template <typename Best, typename First, typename Val>
__device__ __forceinline__ void fit_model(uint32_t L, uint64_t mfin, uint64_t run0, int32_t first_leaf,
                                          const int32_t* prv, const int32_t* nxt, uint32_t* kB, uint32_t* kd,
                                          double* g, const Best& best, const First& first, const Val& val)
{
    double2* seg = reinterpret_cast<double2*>(g + kModelSeg);     // {X, ylo}, {s, yhi}
    double* gym = g + model_ym_off(L);
    double* gy = g + model_y_off(L);
    double* gy1 = g + model_y1_off(L);
    uint32_t* prev = reinterpret_cast<uint32_t*>(g + model_prev_off(L));
    const double inf = __longlong_as_double(0x7ff0000000000000ll);
    if (mfin == 0) {
        for (uint32_t k = threadIdx.x; k <= L; k += blockDim.x) {
            seg[2 * k] = make_double2(inf, 0.0);
            seg[2 * k + 1] = make_double2(0.0, 0.0);
            gym[k] = 0.0;
            gy[k] = 0.0;
            gy1[k] = 0.0;
            if (k < L)
                prev[k] = kNoPrev;
        }
        if (threadIdx.x == 0)
            g[0] = g[1] = g[2] = g[3] = 0.0;
        return;
    }
    const Root R = root_from(val(0), val(mfin - 1), L);
    const double mf = (double)mfin, m2 = (double)(2 * mfin);
    for (uint32_t k = threadIdx.x; k < L; k += blockDim.x) {
        const uint64_t key = best(k);
        if (!key)
            continue;
        const uint64_t len = key >> 32;
        if (len >= 2 && len * L >= mfin) {
            kB[k] = (uint32_t)(0xffffffffull - (key & 0xffffffffull));
            kd[k] = (uint32_t)len;
        } else {
            const uint64_t fr = first(k);
            kB[k] = (uint32_t)(0xffffffffull - (fr >> 32));
            kd[k] = (uint32_t)(fr & 0xffffffffull);
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        g[0] = R.xmin;
        g[1] = R.xmax;
        g[2] = R.rs;
        g[3] = mf;
    }
    // knot k (k == L: the start knot at the sample minimum) and the
    // segment above it
    for (uint32_t k = threadIdx.x; k <= L; k += blockDim.x) {
        uint64_t B = 0, d = 0;
        bool knot = true;
        int32_t q;                                // next non-empty leaf
        if (k < L) {
            knot = best(k) != 0;
            B = knot ? kB[k] : 0;
            d = knot ? kd[k] : 0;
            q = nxt[L - 1 - k];
            prev[k] = prv[k] < 0 ? kNoPrev : (uint32_t)prv[k];
        } else {
            d = run0;
            q = first_leaf;
        }
        if (!knot) {
            // empty leaf: constant at the sample count below it
            const uint64_t nb = q != 0x7fffffff ? 0xffffffffull - (first((uint32_t)q) >> 32) : mfin;
            const double v = (double)nb / mf;
            seg[2 * k] = make_double2(inf, v);
            seg[2 * k + 1] = make_double2(0.0, v);
            gym[k] = v;
            gy[k] = v;
            gy1[k] = v;
            continue;
        }
        const double X = k < L ? val(B) : R.xmin;
        const double ylo = (double)(2 * (B + d) - 1) / m2;
        double Xh = R.xmax, yh = 1.0;
        if (q != 0x7fffffff) {
            const uint64_t Bq = kB[q];
            Xh = val(Bq);
            yh = (double)(2 * Bq + 1) / m2;
        }
        double sl = (yh - ylo) / (Xh - X);
        if (!(sl > 0.0) || __builtin_isinf(sl))
            sl = 0.0;
        seg[2 * k] = make_double2(X, ylo);
        seg[2 * k + 1] = make_double2(sl, yh);
        gym[k] = (double)(2 * B + d) / m2;
        gy[k] = (double)B / mf;
        gy1[k] = (double)(B + d) / mf;
    }
}

// Knots and segments of one job's model (one block per job).
__global__ __launch_bounds__(256) void k_train_fit(const ModelJob* jobs, const uint64_t* sorted, uint64_t* best,
                                                   uint64_t* firstc, uint64_t* nf, double* models,
                                                   const LiveCounts* live)
{
    if (live && blockIdx.x >= live->njobs)
        return;
    __shared__ int32_t prv[kMaxLeaves];
    __shared__ int32_t nxt[kMaxLeaves];      // reversed index
    __shared__ uint32_t kB[kMaxLeaves], kd[kMaxLeaves];   // knot: sample values below it, its copies
    __shared__ int32_t ws32[17];
    __shared__ uint64_t s_lo, s_hi, s_run0;
    const ModelJob J = jobs[blockIdx.x];
    if (J.m <= kSampleBlock)
        return;     // trained in LDS by k_train_small
    const uint32_t L = J.leaves;
    const uint64_t* S = sorted + J.sample_off;
    if (threadIdx.x == 0) {
        uint64_t lo, hi;
        finite_range(nf + 2 * blockIdx.x, J.m, lo, hi);
        s_lo = lo;
        s_hi = hi;
        // the run of the smallest finite value is leaf 0's first run
        s_run0 = hi > lo ? (firstc[J.leaf_off] & 0xffffffffull) : 0;
    }
    const uint64_t* bt = best + J.leaf_off;
    for (uint32_t k = threadIdx.x; k < L; k += blockDim.x) {
        const bool ne = bt[k] != 0;
        prv[k] = ne ? (int32_t)k : -1;
        nxt[L - 1 - k] = ne ? (int32_t)k : 0x7fffffff;
    }
    __syncthreads();
    block_scan_op<int32_t>(prv, L, -1, MaxI32(), ws32);
    const int32_t first_leaf = block_scan_op<int32_t>(nxt, L, 0x7fffffff, MinI32(), ws32);
    const uint64_t lo = s_lo, hi = s_hi;
    fit_model(L, hi - lo, s_run0, first_leaf, prv, nxt, kB, kd, models + J.model_off,
              [&](uint32_t k) { return bt[k]; }, [&](uint32_t k) { return firstc[J.leaf_off + k]; },
              [&](uint64_t i) { return ord_value(S[lo + i], J.dtype); });
    __syncthreads();
    // leave the tables at zero for the next training call
    for (uint32_t k = threadIdx.x; k < L; k += blockDim.x) {
        best[J.leaf_off + k] = 0;
        firstc[J.leaf_off + k] = 0;
    }
    if (threadIdx.x == 0) {
        nf[2 * blockIdx.x] = 0;
        nf[2 * blockIdx.x + 1] = 0;
    }
}

// Values of the sorted sample words held in LDS for modes_runs: entry i is
// the value of word a + i - 1, entry 0 NaN (a is the first finite word).
struct LdsRunVals {
    const uint64_t* w;
    uint64_t a;
    uint32_t dt;
    __device__ double operator[](uint32_t i) const
    {
        return i == 0 ? __longlong_as_double(0x7ff8000000000000ll) : ord_value(w[base_pad((uint32_t)(a + i - 1))], dt);
    }
};

constexpr size_t kSmallTrainLds = (size_t)(kSampleBlock + kSampleBlock / 16) * 8 + (size_t)kMaxLeaves * (8 + 8 + 4 * 4);

// A whole job in one workgroup, when its sample fits one run of
// kSampleBlock words: gather and count the non-finite words, sort in LDS,
// find each leaf's runs and fit, with the sample and the leaf tables in LDS.
__global__ __launch_bounds__(256) void k_train_small(const ModelJob* jobs, double* models, const LiveCounts* live)
{
    if (live && blockIdx.x >= live->njobs)
        return;
    extern __shared__ __align__(16) unsigned char smem[];
    uint64_t* w = reinterpret_cast<uint64_t*>(smem);
    unsigned long long* s_best = reinterpret_cast<unsigned long long*>(smem + (size_t)base_pad(kSampleBlock) * 8);
    unsigned long long* s_first = s_best + kMaxLeaves;
    int32_t* prv = reinterpret_cast<int32_t*>(s_first + kMaxLeaves);
    int32_t* nxt = prv + kMaxLeaves;                 // reversed index
    uint32_t* kB = reinterpret_cast<uint32_t*>(nxt + kMaxLeaves);
    uint32_t* kd = kB + kMaxLeaves;
    __shared__ uint32_t s_nf[2];
    __shared__ int32_t ws32[17];
    const ModelJob J = jobs[blockIdx.x];
    if (J.m > kSampleBlock)
        return;     // trained from the sample buffers
    const uint32_t n = (uint32_t)J.m;
    const uint32_t L = J.leaves;
    if (threadIdx.x == 0)
        s_nf[0] = s_nf[1] = 0;
    for (uint32_t k = threadIdx.x; k < L; k += 256) {
        s_best[k] = 0;
        s_first[k] = 0;
    }
    uint32_t logN = 4;
    while ((1u << logN) < n)
        ++logN;
    constexpr uint32_t U = kSampleBlock / 256;
    uint64_t raw[U];
#pragma unroll
    for (uint32_t u = 0; u < U; ++u) {
        const uint32_t i = u * 256 + threadIdx.x;
        raw[u] = i < n ? as_global<const uint64_t>(J.src)[sample_index(J.seed, i, J.n)] : 0;
    }
    __syncthreads();
    uint32_t neg = 0, pos = 0;
#pragma unroll
    for (uint32_t u = 0; u < U; ++u) {
        const uint32_t i = u * 256 + threadIdx.x;
        if (i < (1u << logN)) {
            const uint64_t word = i < n ? to_ord(raw[u], J.dtype) : ~0ull;
            w[base_pad(i)] = word;
            if (i < n && J.dtype == kF64) {
                neg += word <= kOrdNegInf;
                pos += word >= kOrdPosInf;
            }
        }
    }
    neg = wave_sum(neg);
    pos = wave_sum(pos);
    if ((threadIdx.x & 63u) == 0) {
        if (neg)
            atomicAdd(&s_nf[0], neg);
        if (pos)
            atomicAdd(&s_nf[1], pos);
    }
    __syncthreads();
    lds_bitonic<256>(w, logN);
    const uint64_t lo = s_nf[0], hi = n - s_nf[1];
    const uint64_t mfin = hi - lo;
    auto val = [&](uint64_t i) { return ord_value(w[base_pad((uint32_t)(lo + i))], J.dtype); };
    if (mfin) {
        const Root R = root_from(val(0), val(mfin - 1), L);
        modes_runs(LdsRunVals{w, lo, J.dtype}, (uint32_t)mfin, lo, lo, R, L, s_best, s_first,
                   [&](double) { return hi; });
    }
    __syncthreads();
    for (uint32_t k = threadIdx.x; k < L; k += 256) {
        const bool ne = s_best[k] != 0;
        prv[k] = ne ? (int32_t)k : -1;
        nxt[L - 1 - k] = ne ? (int32_t)k : 0x7fffffff;
    }
    __syncthreads();
    block_scan_op<int32_t>(prv, L, -1, MaxI32(), ws32);
    const int32_t first_leaf = block_scan_op<int32_t>(nxt, L, 0x7fffffff, MinI32(), ws32);
    // the run of the smallest finite value is leaf 0's first run
    const uint64_t run0 = mfin ? (s_first[0] & 0xffffffffull) : 0;
    fit_model(L, mfin, run0, first_leaf, prv, nxt, kB, kd, models + J.model_off,
              [&](uint32_t k) { return (uint64_t)s_best[k]; }, [&](uint32_t k) { return (uint64_t)s_first[k]; }, val);
}

hipError_t launch_train(const ModelJob* d_jobs, uint32_t njobs, uint32_t total_blocks, uint64_t total,
                        uint64_t max_sample, uint64_t* d_sample, uint64_t* d_tmp, uint64_t* d_best,
                        uint64_t* d_first, uint64_t* d_nf, double* d_models, const LiveCounts* live,
                        hipStream_t st)
{
    if (!njobs)
        return hipSuccess;
    // jobs of at most kSampleBlock sample keys train in one workgroup each;
    // the larger ones (nonzero sampling blocks) from the sample buffers
    k_train_small<<<njobs, 256, kSmallTrainLds, st>>>(d_jobs, d_models, live);
    if (max_sample <= kSampleBlock || !total_blocks || !total)
        return hipGetLastError();
    k_train_runs<<<total_blocks, 256, (size_t)base_pad(kSampleBlock) * 8, st>>>(d_jobs, njobs, d_sample, d_nf,
                                                                                 live);
    uint64_t* src = d_sample;
    uint64_t* dst = d_tmp;
    for (uint64_t w = kSampleBlock; w < max_sample; w *= 2) {
        k_train_merge<<<(uint32_t)((total + 255) / 256), 256, 0, st>>>(d_jobs, njobs, src, dst, w, total, live);
        uint64_t* t = src;
        src = dst;
        dst = t;
    }
    k_train_modes<<<total_blocks, 256, 0, st>>>(d_jobs, njobs, src, d_best, d_first, d_nf, live);
    k_train_fit<<<njobs, 256, 0, st>>>(d_jobs, src, d_best, d_first, d_nf, d_models, live);
    return hipGetLastError();
}

}  // namespace lsort
