// Finishing steps (Alg. 2): LDS base case over groups of small buckets,
// fills of all-equal buckets, touch-up check of the seams between ranges.
#include "lsort_device.h"

#include <algorithm>

namespace lsort {

// ------------------------------------------------------------- base case --

// Sort one group (fewer than 2*thresh <= 8192 keys) in LDS with the bitonic
// network of lds_bitonic.  Groups come in three size classes so that small
// groups run in small workgroups: up to 1024 keys on 64 lanes, 4096 on 256,
// 8192 on 512.
template <uint32_t NT>
__global__ __launch_bounds__(NT) void k_base(const Group* groups, uint32_t ngroups, const RoundCtl* gctl,
                                             uint32_t cls)
{
    if (gctl) {
        if (gctl->ntasks != 0 || gctl->overflow)
            return;
        ngroups = gctl->ngroups[cls];
    }
    extern __shared__ __align__(16) unsigned char smem[];
    uint64_t* s = reinterpret_cast<uint64_t*>(smem);
    // one group per workgroup; a grid smaller than the list strides over it
    for (uint32_t g = blockIdx.x; g < ngroups; g += gridDim.x) {
        const Group G = groups[g];
        const gptr<const uint64_t> src = as_global(G.src);
        const gptr<uint64_t> dst = as_global(G.dst);
        const uint32_t n = G.n;
        if (n > NT * 16u)        // never produced by classify; keeps LDS in bounds
            continue;
        uint32_t logN = 4;
        while ((1u << logN) < n)
            ++logN;
        const uint32_t N = 1u << logN;
        for (uint32_t i = threadIdx.x; i < N; i += NT)
            s[base_pad(i)] = i < n ? to_ord(src[i], G.dtype) : ~0ull;
        __syncthreads();
        lds_bitonic<NT>(s, logN);
        for (uint32_t i = threadIdx.x; i < n; i += NT)
            dst[i] = from_ord(s[base_pad(i)], G.dtype);
        __syncthreads();
    }
}

// Workgroups of a graph-mode launch (the list length is only known on the
// device): a few per CU, striding over the list.
constexpr uint32_t kPersistBase[kGroupClasses] = {2048, 1024, 512};
constexpr uint32_t kPersistFill = 2048;
constexpr uint32_t kPersistTouch = 1024;

hipError_t launch_base(const Group* groups, uint32_t ngroups, uint32_t cls, const RoundCtl* gctl, hipStream_t st)
{
    const uint32_t grid = gctl ? std::min(ngroups, kPersistBase[cls]) : ngroups;
    if (!grid)
        return hipSuccess;
    const size_t lds = (size_t)base_pad(kGroupClassCap[cls]) * 8;
    switch (cls) {
    case 0: k_base<64><<<grid, 64, lds, st>>>(groups, ngroups, gctl, 0); break;
    case 1: k_base<256><<<grid, 256, lds, st>>>(groups, ngroups, gctl, 1); break;
    case 2: k_base<512><<<grid, 512, lds, st>>>(groups, ngroups, gctl, 2); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ------------------------------------------------------------------ fill --

__global__ __launch_bounds__(256) void k_fill(const Fill* fills, uint32_t nfill, const RoundCtl* gctl)
{
    if (gctl) {
        if (gctl->ntasks != 0 || gctl->overflow)
            return;
        nfill = gctl->nfill;
    }
    for (uint32_t f = blockIdx.x; f < nfill; f += gridDim.x) {
        const Fill F = fills[f];
        const gptr<uint64_t> dst = as_global(F.dst);
        for (uint32_t i = threadIdx.x; i < F.n; i += 256)
            dst[i] = F.raw;
    }
}

hipError_t launch_fill(const Fill* d_fills, uint32_t nfill, const RoundCtl* gctl, hipStream_t st)
{
    const uint32_t grid = gctl ? std::min(nfill, kPersistFill) : nfill;
    if (grid)
        k_fill<<<grid, 256, 0, st>>>(d_fills, nfill, gctl);
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

__global__ __launch_bounds__(256) void k_touchup(RangeLists R, RoundCtl* ctl, bool graph)
{
    if (graph) {
        if (ctl->ntasks != 0 || ctl->overflow)
            return;
        for (uint32_t c = 0; c < kGroupClasses; ++c)
            R.ng[c] = ctl->ngroups[c];
        R.nfill = ctl->nfill;
    }
    uint64_t items = R.nfill;
    for (uint32_t c = 0; c < kGroupClasses; ++c)
        items += R.ng[c];
    uint32_t bad = 0;
    for (uint64_t it = (uint64_t)blockIdx.x * 256 + threadIdx.x; it < items; it += (uint64_t)gridDim.x * 256) {
        uint64_t i = it;
        const uint64_t* p = nullptr;
        uint64_t start = 0;
        uint32_t dt = 0;
        for (uint32_t c = 0; c < kGroupClasses && !p; ++c) {
            if (i < R.ng[c]) {
                const gptr<const Group> g = as_global(R.g[c]);
                p = g[i].dst;
                start = g[i].start;
                dt = g[i].dtype;
            } else {
                i -= R.ng[c];
            }
        }
        if (!p) {
            const gptr<const Fill> fl = as_global(R.fills);
            p = fl[i].dst;
            start = fl[i].start;
            dt = fl[i].dtype;
        }
        const gptr<const uint64_t> q = as_global(p);
        bad += start > 0 && to_ord(q[-1], dt) > to_ord(q[0], dt);
    }
    if (bad)
        atomicAdd(&ctl->violations, bad);
}

__global__ __launch_bounds__(256) void k_touchup_full(const Group* groups, RoundCtl* ctl)
{
    const Group G = groups[blockIdx.x];
    const gptr<const uint64_t> d = as_global<const uint64_t>(G.dst);
    uint32_t bad = 0;
    for (uint32_t i = threadIdx.x + 1; i < G.n; i += 256)
        bad += to_ord(d[i - 1], G.dtype) > to_ord(d[i], G.dtype);
    if (bad)
        atomicAdd(&ctl->violations, bad);
}

hipError_t launch_touchup(GroupLists groups, const uint32_t* ngroups, const Fill* d_fills, uint32_t nfill, int full,
                          RoundCtl* d_ctl, bool graph, hipStream_t st)
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
    uint64_t grid = (items + 255) / 256;
    if (graph)
        grid = std::min<uint64_t>(grid, kPersistTouch);
    if (grid)
        k_touchup<<<(uint32_t)grid, 256, 0, st>>>(R, d_ctl, graph);
    if (full && !graph)
        for (uint32_t c = 0; c < kGroupClasses; ++c)
            if (ngroups[c])
                k_touchup_full<<<ngroups[c], 256, 0, st>>>(groups.g[c], d_ctl);
    return hipGetLastError();
}

}  // namespace lsort
