// Model training: sample, per-leaf statistics, spline fit (Sec. 6.1).
#include "lsort_device.h"

#pragma clang fp contract(off)

namespace lsort {

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

// Training tables use 0 as their neutral value and the fit kernel returns
// them to 0 after use, so no initialisation pass is needed: per job
// minmax = {~min, max} of the finite sample words, per leaf lcnt = count and
// lmin = ~(smallest word).

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
    constexpr uint32_t U = kSampleBlock / 256;    // independent gathers in flight per lane
    uint64_t raw[U];
#pragma unroll
    for (uint32_t u = 0; u < U; ++u) {
        const uint64_t t = t0 + u * 256 + threadIdx.x;
        raw[u] = t < J.m ? J.src[sample_index(J.seed, t, J.n)] : 0;
    }
#pragma unroll
    for (uint32_t u = 0; u < U; ++u) {
        const uint64_t t = t0 + u * 256 + threadIdx.x;
        if (t < J.m) {
            const uint64_t o = to_ord(raw[u], J.dtype);
            sample[J.sample_off + t] = o;
            if (!nonfinite(raw[u], J.dtype)) {
                lo = o < lo ? o : lo;
                hi = o > hi ? o : hi;
            }
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
            atomicMax((unsigned long long*)&minmax[2 * j], (unsigned long long)~lo);
            atomicMax((unsigned long long*)&minmax[2 * j + 1], (unsigned long long)hi);
        }
    }
}

__device__ __forceinline__ void root_params(const uint64_t* minmax, uint32_t j, uint32_t dt, uint32_t L,
                                            double& xmin, double& xmax, double& rs, bool& any)
{
    uint64_t lo = ~minmax[2 * j], hi = minmax[2 * j + 1];
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
            atomicMax((unsigned long long*)&lmin[J.leaf_off + k], ~mn[k]);
        }
    }
}

// Fit: knots at leaf minima with exact eCDF values, segments to the next knot.
// Prefix counts, previous and next non-empty leaf come from block scans.
__global__ __launch_bounds__(256) void k_train_fit(const ModelJob* jobs, uint64_t* minmax, uint32_t* lcnt,
                                                   uint64_t* lmin, double* models)
{
    __shared__ uint64_t below[kMaxLeaves];
    __shared__ int32_t prv[kMaxLeaves];
    __shared__ int32_t nxt[kMaxLeaves];      // reversed index
    __shared__ uint64_t ws64[5];
    __shared__ int32_t ws32[5];
    const uint32_t j = blockIdx.x;
    const ModelJob J = jobs[j];
    const uint32_t L = J.leaves;
    const uint32_t* cnt = lcnt + J.leaf_off;
    for (uint32_t k = threadIdx.x; k < L; k += blockDim.x) {
        const uint32_t c = cnt[k];
        below[k] = c;
        prv[k] = c ? (int32_t)k : -1;
        nxt[L - 1 - k] = c ? (int32_t)k : 0x7fffffff;
    }
    __syncthreads();
    const uint64_t mfin = block_scan_op<uint64_t>(below, L, 0ull, AddU64(), ws64);
    block_scan_op<int32_t>(prv, L, -1, MaxI32(), ws32);
    block_scan_op<int32_t>(nxt, L, 0x7fffffff, MinI32(), ws32);
    double xmin, xmax, rs;
    bool any;
    root_params(minmax, j, J.dtype, L, xmin, xmax, rs, any);
    double* g = models + J.model_off;
    double* seg = g + 4;                                   // per leaf {X, y, s, yhi}
    uint32_t* prev = reinterpret_cast<uint32_t*>(g + 4 + 4 * (size_t)L);
    if (threadIdx.x == 0) {
        g[0] = mfin ? xmin : 0.0;
        g[1] = mfin ? xmax : 0.0;
        g[2] = mfin ? rs : 0.0;
        g[3] = (double)mfin;
    }
    const double inf = __longlong_as_double(0x7ff0000000000000ll);
    for (uint32_t k = threadIdx.x; k < L; k += blockDim.x) {
        double* o = seg + 4 * (size_t)k;
        if (!mfin) {
            o[0] = inf;
            o[1] = 0.0;
            o[2] = 0.0;
            o[3] = 0.0;
            prev[k] = kNoPrev;
            continue;
        }
        const double yk = (double)below[k] / (double)mfin;
        prev[k] = prv[k] < 0 ? kNoPrev : (uint32_t)prv[k];
        if (!cnt[k]) {
            o[0] = inf;
            o[1] = yk;
            o[2] = 0.0;
            o[3] = yk;
            continue;
        }
        const double Xk = ord_value(~lmin[J.leaf_off + k], J.dtype);
        double Xh = xmax, yh = 1.0;
        const int32_t q = nxt[L - 1 - k];          // first non-empty leaf after k
        if (q != 0x7fffffff) {
            Xh = ord_value(~lmin[J.leaf_off + q], J.dtype);
            yh = (double)below[q] / (double)mfin;
        }
        double sl = (yh - yk) / (Xh - Xk);
        if (!(sl > 0.0) || __builtin_isinf(sl))
            sl = 0.0;
        o[0] = Xk;
        o[1] = yk;
        o[2] = sl;
        o[3] = yh;
    }
    __syncthreads();
    // leave the tables neutral for the next training call
    for (uint32_t k = threadIdx.x; k < L; k += blockDim.x) {
        lcnt[J.leaf_off + k] = 0;
        lmin[J.leaf_off + k] = 0;
    }
    if (threadIdx.x == 0) {
        minmax[2 * j] = 0;
        minmax[2 * j + 1] = 0;
    }
}

hipError_t launch_train(const ModelJob* d_jobs, uint32_t njobs, uint32_t total_blocks, uint64_t* d_sample,
                        uint64_t* d_minmax, uint32_t* d_lcnt, uint64_t* d_lmin, double* d_models,
                        hipStream_t st)
{
    if (!njobs)
        return hipSuccess;
    k_train_sample<<<total_blocks, 256, 0, st>>>(d_jobs, njobs, d_sample, d_minmax);
    k_train_leaves<<<total_blocks, 256, 0, st>>>(d_jobs, njobs, d_sample, d_minmax, d_lcnt, d_lmin);
    k_train_fit<<<njobs, 256, 0, st>>>(d_jobs, d_minmax, d_lcnt, d_lmin, d_models);
    return hipGetLastError();
}

}  // namespace lsort
