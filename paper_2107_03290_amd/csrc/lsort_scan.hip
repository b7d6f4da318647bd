// Exclusive scan of the per-(bucket, chunk) counts of a partition round into
// 64-bit positions: one kernel sums blocks of 4096 counts, a second kernel
// rescans each block after adding the sums of all blocks before it (there
// are at most a few thousand blocks, so each block reduces them itself).
#include "lsort_device.h"

namespace lsort {

constexpr uint32_t kScanBlock = 4096;
constexpr uint32_t kScanThreads = 256;

__global__ __launch_bounds__(kScanThreads) void k_scan_reduce(const uint32_t* in, uint64_t n, uint64_t* sums,
                                                              const LiveCounts* live)
{
    if (live) {
        n = live->entries;
        if ((uint64_t)blockIdx.x * kScanBlock >= n)
            return;
    }
    __shared__ uint64_t ws[kScanThreads / 64];
    const uint64_t base = (uint64_t)blockIdx.x * kScanBlock;
    uint64_t s = 0;
    for (uint32_t i = threadIdx.x; i < kScanBlock; i += kScanThreads) {
        const uint64_t k = base + i;
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

__global__ __launch_bounds__(kScanThreads) void k_scan_down(const uint32_t* in, uint64_t n, const uint64_t* sums,
                                                            uint64_t* out, const LiveCounts* live)
{
    if (live) {
        n = live->entries;
        if ((uint64_t)blockIdx.x * kScanBlock >= n)
            return;
    }
    __shared__ uint64_t ws[kScanThreads / 64 + 1];
    __shared__ uint64_t s_base;
    // prefix of this block: the sums of every earlier block
    uint64_t pre = 0;
    for (uint32_t j = threadIdx.x; j < blockIdx.x; j += kScanThreads)
        pre += sums[j];
    for (uint32_t d = 32; d > 0; d >>= 1)
        pre += __shfl_xor(pre, d, 64);
    if ((threadIdx.x & 63u) == 0)
        ws[threadIdx.x >> 6] = pre;
    __syncthreads();
    if (threadIdx.x == 0)
        s_base = ws[0] + ws[1] + ws[2] + ws[3];
    __syncthreads();
    const uint64_t base = (uint64_t)blockIdx.x * kScanBlock;
    constexpr uint32_t per = kScanBlock / kScanThreads;
    uint32_t v[per];
    uint64_t s = 0;
#pragma unroll
    for (uint32_t i = 0; i < per; ++i) {
        const uint64_t k = base + (uint64_t)threadIdx.x * per + i;
        v[i] = k < n ? in[k] : 0u;
        s += v[i];
    }
    const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
    uint64_t x = s;
    for (uint32_t d = 1; d < 64; d <<= 1) {
        const uint64_t y = __shfl_up(x, d, 64);
        if (lane >= d)
            x += y;
    }
    if (lane == 63)
        ws[wave] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t run = s_base;
        for (uint32_t w = 0; w < kScanThreads / 64; ++w) {
            const uint64_t t = ws[w];
            ws[w] = run;
            run += t;
        }
    }
    __syncthreads();
    uint64_t b = ws[wave] + x - s;
#pragma unroll
    for (uint32_t i = 0; i < per; ++i) {
        const uint64_t k = base + (uint64_t)threadIdx.x * per + i;
        if (k < n)
            out[k] = b;
        b += v[i];
    }
}

size_t scan_tmp_entries(uint64_t n) { return (size_t)((n + kScanBlock - 1) / kScanBlock) + 1; }

hipError_t launch_scan(const uint32_t* d_in, uint64_t* d_out, uint64_t n, uint64_t* d_tmp, const LiveCounts* live,
                       hipStream_t st)
{
    const uint32_t nb = (uint32_t)((n + kScanBlock - 1) / kScanBlock);
    if (!nb)
        return hipSuccess;
    k_scan_reduce<<<nb, kScanThreads, 0, st>>>(d_in, n, d_tmp, live);
    k_scan_down<<<nb, kScanThreads, 0, st>>>(d_in, n, d_tmp, d_out, live);
    return hipGetLastError();
}

}  // namespace lsort
