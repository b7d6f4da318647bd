// Finishing steps: LDS base case, all-equal fills, touch-up check (Alg. 2).
#include "lsort_device.h"

#pragma clang fp contract(off)

namespace lsort {

// ------------------------------------------------------------- base case --

// Sort one group (fewer than 2*thresh <= 8192 keys) in LDS with a bitonic
// network over the next power of two N >= 16, padded with the largest word.
// Each thread keeps 16 elements in registers: the 16 indices that differ only
// in a window of 4 index bits.  Up to four consecutive stages of the network
// touch only bits inside one window, so each LDS round trip runs four stages
// in registers; a phase of the network needs ceil(p/4) round trips.
constexpr uint32_t kBaseThreads = 512;
constexpr uint32_t kBaseMax = kBaseThreads * 16;

__host__ __device__ __forceinline__ uint32_t base_pad(uint32_t i) { return i + (i >> 4); }

// element index of register m of thread t, the 4 register bits at [lo, lo+4)
__device__ __forceinline__ uint32_t base_idx(uint32_t t, uint32_t lo, uint32_t m)
{
    const uint32_t low = t & ((1u << lo) - 1u);
    return low | (m << lo) | ((t >> lo) << (lo + 4));
}

__device__ __forceinline__ void cmpex(uint64_t& a, uint64_t& b, bool up)
{
    const uint64_t lo = a < b ? a : b;
    const uint64_t hi = a < b ? b : a;
    a = up ? lo : hi;
    b = up ? hi : lo;
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

__global__ __launch_bounds__(kBaseThreads) void k_base(const Group* groups)
{
    extern __shared__ __align__(16) unsigned char smem[];
    uint64_t* s = reinterpret_cast<uint64_t*>(smem);
    const Group G = groups[blockIdx.x];
    const uint32_t n = G.n;
    if (n > kBaseMax)            // never produced by the grouping rule; keeps LDS in bounds
        return;
    uint32_t logN = 4;
    while ((1u << logN) < n)
        ++logN;
    const uint32_t N = 1u << logN;
    const uint32_t t = threadIdx.x;
    const bool act = t < (N >> 4);
    for (uint32_t i = t; i < N; i += kBaseThreads)
        s[base_pad(i)] = i < n ? to_ord(G.src[i], G.dtype) : ~0ull;
    __syncthreads();
    uint64_t r[16];
    // phases 1..4: the 16 consecutive elements of each thread
    if (act) {
#pragma unroll
        for (int m = 0; m < 16; ++m)
            r[m] = s[base_pad(16 * t + m)];
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
            s[base_pad(16 * t + m)] = r[m];
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
                    r[m] = s[base_pad(base_idx(t, lo, (uint32_t)m))];
                reg_stages(r, (uint32_t)bit - lo, up);
#pragma unroll
                for (int m = 0; m < 16; ++m)
                    s[base_pad(base_idx(t, lo, (uint32_t)m))] = r[m];
            }
            __syncthreads();
            bit = (int32_t)lo - 1;
        }
    }
    for (uint32_t i = t; i < n; i += kBaseThreads)
        G.dst[i] = from_ord(s[base_pad(i)], G.dtype);
}

hipError_t launch_base(const Group* d_groups, uint32_t ngroups, uint32_t base_cap, hipStream_t st)
{
    if (!ngroups)
        return hipSuccess;
    if (base_cap > kBaseMax)
        return hipErrorInvalidValue;
    k_base<<<ngroups, kBaseThreads, (size_t)base_pad(kBaseMax) * 8, st>>>(d_groups);
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
