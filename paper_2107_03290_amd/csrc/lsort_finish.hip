// Finishing steps (Alg. 2): LDS base case over groups of small buckets,
// fills of all-equal buckets, touch-up check of the seams between ranges.
#include "lsort_device.h"

namespace lsort {

// ------------------------------------------------------------- base case --

// Sort one group (fewer than 2*thresh <= 8192 keys) in LDS with a bitonic
// network over the next power of two N >= 16, padded with the largest word.
// Each thread keeps 16 elements in registers: the 16 indices that differ only
// in a window of 4 index bits.  Up to four consecutive stages of the network
// touch only bits inside one window, so each LDS round trip runs four stages
// in registers; a phase of the network needs ceil(p/4) round trips.  Groups
// come in three size classes so that small groups run in small workgroups:
// up to 1024 keys on 64 lanes, 4096 on 256, 8192 on 512.
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

template <uint32_t NT>
__global__ __launch_bounds__(NT) void k_base(const Group* groups)
{
    extern __shared__ __align__(16) unsigned char smem[];
    uint64_t* s = reinterpret_cast<uint64_t*>(smem);
    const Group G = groups[blockIdx.x];
    const uint32_t n = G.n;
    if (n > NT * 16u)            // never produced by classify; keeps LDS in bounds
        return;
    uint32_t logN = 4;
    while ((1u << logN) < n)
        ++logN;
    const uint32_t N = 1u << logN;
    const uint32_t t = threadIdx.x;
    const bool act = t < (N >> 4);
    for (uint32_t i = t; i < N; i += NT)
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
    for (uint32_t i = t; i < n; i += NT)
        G.dst[i] = from_ord(s[base_pad(i)], G.dtype);
}

hipError_t launch_base(GroupLists groups, const uint32_t* ngroups, hipStream_t st)
{
    if (ngroups[0])
        k_base<64><<<ngroups[0], 64, (size_t)base_pad(kGroupClassCap[0]) * 8, st>>>(groups.g[0]);
    if (ngroups[1])
        k_base<256><<<ngroups[1], 256, (size_t)base_pad(kGroupClassCap[1]) * 8, st>>>(groups.g[1]);
    if (ngroups[2])
        k_base<512><<<ngroups[2], 512, (size_t)base_pad(kGroupClassCap[2]) * 8, st>>>(groups.g[2]);
    return hipGetLastError();
}

// ------------------------------------------------------------------ fill --

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

// -------------------------------------------------------------- touch-up --

// Touch-up check (Alg. 2's final pass): every final range is sorted by
// construction, so only the seam with the preceding range can be out of
// order.  `full` also rechecks every adjacent pair inside the groups.
struct RangeLists {
    const Group* g[kGroupClasses];
    uint32_t ng[kGroupClasses];
    const Fill* fills;
    uint32_t nfill;
};

__global__ __launch_bounds__(256) void k_touchup(RangeLists R, RoundCtl* ctl)
{
    uint32_t i = blockIdx.x * 256 + threadIdx.x;
    const uint64_t* p = nullptr;
    uint64_t start = 0;
    uint32_t dt = 0;
    for (uint32_t c = 0; c < kGroupClasses && !p; ++c) {
        if (i < R.ng[c]) {
            p = R.g[c][i].dst;
            start = R.g[c][i].start;
            dt = R.g[c][i].dtype;
        } else {
            i -= R.ng[c];
        }
    }
    if (!p) {
        if (i >= R.nfill)
            return;
        p = R.fills[i].dst;
        start = R.fills[i].start;
        dt = R.fills[i].dtype;
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

hipError_t launch_touchup(GroupLists groups, const uint32_t* ngroups, const Fill* d_fills, uint32_t nfill, int full,
                          RoundCtl* d_ctl, hipStream_t st)
{
    RangeLists R;
    uint64_t items = nfill;
    for (uint32_t c = 0; c < kGroupClasses; ++c) {
        R.g[c] = groups.g[c];
        R.ng[c] = ngroups[c];
        items += ngroups[c];
    }
    R.fills = d_fills;
    R.nfill = nfill;
    if (items)
        k_touchup<<<(uint32_t)((items + 255) / 256), 256, 0, st>>>(R, d_ctl);
    if (full)
        for (uint32_t c = 0; c < kGroupClasses; ++c)
            if (ngroups[c])
                k_touchup_full<<<ngroups[c], 256, 0, st>>>(groups.g[c], d_ctl);
    return hipGetLastError();
}

}  // namespace lsort
