// Finishing steps (Alg. 2): LDS base case over groups of small buckets,
// fills of all-equal buckets, touch-up check of the seams between ranges.
#include "lsort_device.h"

#include <algorithm>

namespace lsort {

// ------------------------------------------------------------- base case --

// Sort one group (fewer than 2*thresh <= 8192 keys, the adjacent small
// buckets of a partition) in LDS in linear work, as Alg. 2 finishes a bucket
// with a counting sort on predicted positions followed by a local fix-up:
//   * slots: the group's range [lo, hi] of order words is cut into nslots
//     (the power of two at or above n) equal power-of-two slots, slot(o) =
//     (o - lo) >> sh, a monotone map;
//   * count the keys of each slot (an LDS atomic gives each key its rank in
//     its slot), scan the counts into slot starts, place each key at its
//     slot start plus rank;
//   * fix-up inside a slot: a slot whose keys are all equal is final as
//     placed; in a slot holding different keys, a key's position is the
//     slot start plus the number of its keys that are smaller, or equal and
//     placed before it;
//   * write the group out through LDS in order.
// A group whose range is one value is copied.  A group with a mixed slot of
// more than kBaseSlotMax keys (a fix-up of quadratic cost) is marked and
// sorted afterwards by k_base_slow with the bitonic network of lds_bitonic.
//
// Size classes: up to 1024 keys on 256 lanes, 4096 on 512, 8192 on 1024.
// The grid is a few workgroups per CU; each workgroup strides over the list.
constexpr uint32_t kBaseSlotMax = 64;

// LDS: the group's order words, then per slot (at most CAP / 2 slots) the
// count / start and the mixed flag.
template <uint32_t NT, uint32_t KPT>
__host__ __device__ constexpr size_t base_lds_bytes()
{
    return ((size_t)NT * KPT * 8 + (size_t)(NT * KPT / 2 + 1) * 4 + (size_t)NT * KPT / 2 + 15) & ~(size_t)15;
}

// A group descriptor read with global (not flat) loads, so that it can stay
// in flight while the workgroup waits on LDS.
__device__ __forceinline__ Group group_at(const Group* groups, uint32_t i)
{
    static_assert(sizeof(Group) == 48, "six words");
    const gptr<const uint64_t> w = as_global(reinterpret_cast<const uint64_t*>(groups) + 6ull * i);
    const uint64_t a = w[0], b = w[1], c = w[2], d = w[3], lo = w[4], hi = w[5];
    Group G;
    G.src = reinterpret_cast<const uint64_t*>(a);
    G.dst = reinterpret_cast<uint64_t*>(b);
    G.start = c;
    G.n = (uint32_t)d;
    G.dtype = (uint32_t)(d >> 32);
    G.lo = lo;
    G.hi = hi;
    return G;
}

// Every lane reads the same descriptor: its fields are moved to scalar
// registers where they are used (not where they are loaded, which would wait
// for the load), so that loops over a group's keys branch on the scalar unit.
__device__ __forceinline__ uint32_t uni32(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_readfirstlane((int)v);
}

template <class T>
__device__ __forceinline__ T* uni_ptr(T* p)
{
    const uint64_t v = reinterpret_cast<uint64_t>(p);
    return reinterpret_cast<T*>((uint64_t)uni32((uint32_t)v) | ((uint64_t)uni32((uint32_t)(v >> 32)) << 32));
}

template <uint32_t NT, uint32_t KPT>
__device__ __forceinline__ void base_load(const Group& G, uint64_t (&raw)[KPT])
{
    const gptr<const uint64_t> src = as_global(uni_ptr(G.src));
    const uint32_t gn = uni32(G.n);
    const uint32_t n = gn <= NT * KPT ? gn : 0u;
#pragma unroll
    for (uint32_t k = 0; k < KPT; ++k) {
        const uint32_t i = k * NT + threadIdx.x;
        raw[k] = 0;
        if (k * NT < n && i < n)
            raw[k] = src[i];
    }
}

// A group the slot sort hands over to the bitonic network: the top bit of
// its dtype word in the list marks it until k_base_slow has sorted it.
constexpr uint32_t kSlowMark = 0x80000000u;

__device__ __forceinline__ void mark_slow(const Group* groups, uint32_t g)
{
    uint32_t* w = reinterpret_cast<uint32_t*>(const_cast<Group*>(groups) + g) + 7;   // high half of {n, dtype}
    *as_global(w) = *as_global(w) | kSlowMark;
}

// The groups of one size class that k_base marked: workgroup b looks at
// groups b, b + grid, b + 2 grid, ... (NT descriptors at a time, one per
// lane), so marked groups are spread over the grid, and sorts the marked
// ones with the bitonic network of lds_bitonic (groups of at most 16 NT
// keys).
template <uint32_t NT>
__global__ __launch_bounds__(NT) void k_base_slow(Group* groups, uint32_t ngroups, const RoundCtl* gctl,
                                                  uint32_t cls)
{
    if (gctl) {
        if (gctl->ntasks != 0 || gctl->overflow)
            return;
        ngroups = gctl->ngroups[cls];
    }
    extern __shared__ __align__(16) unsigned char smem[];
    uint64_t* s = reinterpret_cast<uint64_t*>(smem);
    __shared__ uint32_t s_list[NT];
    __shared__ uint32_t s_cnt;
    for (uint64_t j0 = 0; blockIdx.x + j0 * gridDim.x < ngroups; j0 += NT) {
        if (threadIdx.x == 0)
            s_cnt = 0;
        __syncthreads();
        const uint64_t g = blockIdx.x + (j0 + threadIdx.x) * gridDim.x;
        if (g < ngroups && (as_global(&groups[g].dtype)[0] & kSlowMark))
            s_list[atomicAdd(&s_cnt, 1u)] = (uint32_t)g;
        __syncthreads();
        const uint32_t cnt = s_cnt;
        for (uint32_t j = 0; j < cnt; ++j) {
            const uint32_t gi = s_list[j];
            const Group G = groups[gi];
            const uint32_t dt = G.dtype & ~kSlowMark;
            const gptr<const uint64_t> src = as_global(G.src);
            const gptr<uint64_t> dst = as_global(G.dst);
            const uint32_t n = G.n <= 16 * NT ? G.n : 0u;
            uint32_t logN = 4;
            while ((1u << logN) < n)
                ++logN;
            const uint32_t N = 1u << logN;
            for (uint32_t i = threadIdx.x; i < N; i += NT)
                s[base_pad(i)] = i < n ? to_ord(src[i], dt) : ~0ull;
            __syncthreads();
            if (n)
                lds_bitonic<NT>(s, logN);
            for (uint32_t i = threadIdx.x; i < n; i += NT)
                dst[i] = from_ord(s[base_pad(i)], dt);
            if (threadIdx.x == 0)
                groups[gi].dtype = dt;
            __syncthreads();
        }
    }
}

template <uint32_t NT, uint32_t KPT, uint32_t WPE>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(WPE))) void k_base(
    const Group* groups, uint32_t ngroups, const RoundCtl* gctl,
                                             uint32_t cls)
{
    constexpr uint32_t CAP = NT * KPT;
    constexpr uint32_t NW = NT / 64;
    if (gctl) {
        if (gctl->ntasks != 0 || gctl->overflow)
            return;
        ngroups = gctl->ngroups[cls];
    }
    extern __shared__ __align__(16) unsigned char smem[];
    uint64_t* stage = reinterpret_cast<uint64_t*>(smem);                // CAP words
    uint32_t* start = reinterpret_cast<uint32_t*>(stage + CAP);         // CAP / 2 + 1 slot counts / starts
    uint8_t* mixed = reinterpret_cast<uint8_t*>(start + CAP / 2 + 1);   // CAP / 2 slot flags
    __shared__ uint64_t s_lo[NW], s_hi[NW];
    __shared__ uint32_t wsum[NW + 1];
    __shared__ uint32_t s_slow;
    const uint32_t t = threadIdx.x, lane = t & 63u, wave = t >> 6;
    // consecutive groups (adjacent outputs) on one XCD
    uint32_t g = xcd_order(blockIdx.x, gridDim.x);
    Group G{};
    if (g < ngroups)
        G = group_at(groups, g);
    for (; g < ngroups; g += gridDim.x) {
        // the next descriptor is in flight while this group is sorted
        Group Gn{};
        if (g + gridDim.x < ngroups)
            Gn = group_at(groups, g + gridDim.x);
        uint64_t raw[KPT];
        base_load<NT, KPT>(G, raw);
        const gptr<uint64_t> dst = as_global(uni_ptr(G.dst));
        const uint32_t n = uni32(G.n);
        const uint32_t dt = uni32(G.dtype);
        if (n <= CAP) {     // larger groups are never produced by classify; keeps LDS in bounds
            uint64_t o[KPT];
            // the range of the group's order words: given by the partition
            // that formed the group, else reduced here
            uint64_t lo = uni32((uint32_t)G.lo) | ((uint64_t)uni32((uint32_t)(G.lo >> 32)) << 32);
            uint64_t hi = uni32((uint32_t)G.hi) | ((uint64_t)uni32((uint32_t)(G.hi >> 32)) << 32);
            const bool known = lo <= hi;
#pragma unroll
            for (uint32_t k = 0; k < KPT; ++k)
                o[k] = to_ord(raw[k], dt);
            if (!known) {
                lo = ~0ull;
                hi = 0;
#pragma unroll
                for (uint32_t k = 0; k < KPT; ++k) {
                    if (k * NT < n && k * NT + t < n) {
                        lo = o[k] < lo ? o[k] : lo;
                        hi = o[k] > hi ? o[k] : hi;
                    }
                }
#pragma unroll
                for (uint32_t d = 32; d > 0; d >>= 1) {
                    const uint64_t a = __shfl_xor(lo, d, 64), b = __shfl_xor(hi, d, 64);
                    lo = a < lo ? a : lo;
                    hi = b > hi ? b : hi;
                }
                if (lane == 0) {
                    s_lo[wave] = lo;
                    s_hi[wave] = hi;
                }
            }
            // at least two slots, so that the shift below stays under 64
            const uint32_t nslots = pow2_at_least(n < 4 ? 2u : (n + 1) / 2);
            for (uint32_t j = t; j < nslots; j += NT) {
                start[j] = 0;
                mixed[j] = 0;
            }
            if (t == 0)
                s_slow = 0;
            __syncthreads();
            if (!known) {
#pragma unroll
                for (uint32_t w = 0; w < NW; ++w) {
                    lo = s_lo[w] < lo ? s_lo[w] : lo;
                    hi = s_hi[w] > hi ? s_hi[w] : hi;
                }
            }
            if (lo == hi) {     // one value: already in order
#pragma unroll
                for (uint32_t k = 0; k < KPT; ++k) {
                    const uint32_t i = k * NT + t;
                    if (k * NT < n && i < n)
                        dst[i] = from_ord(o[k], dt);
                }
            } else {
                const uint32_t bits = 64u - (uint32_t)__clzll((long long)(hi - lo));
                const uint32_t lg = 31u - __clz(nslots);
                const uint32_t sh = bits > lg ? bits - lg : 0u;
                // slot (low half) and rank in the slot (high half) of each key;
                // both are below 2^13
                uint32_t sr[KPT];
#pragma unroll
                for (uint32_t k = 0; k < KPT; ++k) {
                    sr[k] = 0;
                    if (k * NT < n && k * NT + t < n) {
                        const uint32_t sl = (uint32_t)((o[k] - lo) >> sh);
                        sr[k] = sl | (atomicAdd(&start[sl], 1u) << 16);
                    }
                }
                __syncthreads();
                block_scan_u32(start, nslots, wsum);
                if (t == 0)
                    start[nslots] = n;
#pragma unroll
                for (uint32_t k = 0; k < KPT; ++k)
                    if (k * NT < n && k * NT + t < n)
                        stage[start[sr[k] & 0xffffu] + (sr[k] >> 16)] = o[k];
                __syncthreads();
                // a slot is mixed when one of its keys differs from the key placed first
#pragma unroll
                for (uint32_t k = 0; k < KPT; ++k) {
                    if (k * NT < n && k * NT + t < n) {
                        const uint32_t sl = sr[k] & 0xffffu;
                        const uint32_t s0 = start[sl];
                        if (stage[s0] != o[k]) {
                            mixed[sl] = 1;
                            if (start[sl + 1] - s0 > kBaseSlotMax)
                                s_slow = 1;
                        }
                    }
                }
                __syncthreads();
                if (s_slow) {
                    // left to k_base_slow
                    if (t == 0)
                        mark_slow(groups, g);
                } else {
                    // each key's final index in the group replaces its slot and rank
#pragma unroll
                    for (uint32_t k = 0; k < KPT; ++k) {
                        if (k * NT < n && k * NT + t < n) {
                            const uint32_t sl = sr[k] & 0xffffu;
                            const uint32_t s0 = start[sl];
                            const uint32_t p = s0 + (sr[k] >> 16);
                            const uint32_t mix = mixed[sl];
                            uint32_t q = p;
                            if (mix) {
                                const uint32_t e = start[sl + 1];
                                uint32_t r = 0;
                                // two keys per step: their LDS reads are in flight together
                                uint32_t j = s0;
                                for (; j + 2 <= e; j += 2) {
                                    const uint64_t v0 = stage[j], v1 = stage[j + 1];
                                    r += (v0 < o[k]) | ((v0 == o[k]) & (j < p));
                                    r += (v1 < o[k]) | ((v1 == o[k]) & (j + 1 < p));
                                }
                                if (j < e) {
                                    const uint64_t v = stage[j];
                                    r += (v < o[k]) | ((v == o[k]) & (j < p));
                                }
                                q = s0 + r;
                            }
                            sr[k] = q;
                        }
                    }
                    __syncthreads();
#pragma unroll
                    for (uint32_t k = 0; k < KPT; ++k)
                        if (k * NT < n && k * NT + t < n)
                            stage[sr[k]] = o[k];
                    __syncthreads();
                    for (uint32_t i = t; i < n; i += NT)
                        dst[i] = from_ord(stage[i], dt);
                }
            }
            __syncthreads();
        }
        G = Gn;
    }
}

// Workgroups per launch of each size class: about as many as fit on the
// CUs at once (LDS: 14, 42 and 84 KB per workgroup).
constexpr uint32_t kPersistBase[kGroupClasses] = {2048, 768, 256};
// Workgroups of a graph-mode fill or touch-up launch (the list length is only
// known on the device): a few per CU, striding over the list.
constexpr uint32_t kPersistFill = 2048;
constexpr uint32_t kPersistTouch = 1024;

hipError_t launch_base(const Group* groups, uint32_t ngroups, uint32_t cls, const RoundCtl* gctl, hipStream_t st)
{
    const uint32_t grid = std::min(ngroups, kPersistBase[cls]);
    if (!grid)
        return hipSuccess;
    static_assert(256 * 4 == kGroupClassCap[0] && 512 * 8 == kGroupClassCap[1] && 1024 * 8 == kGroupClassCap[2],
                  "one base-case kernel shape per size class");
    switch (cls) {
    case 0: k_base<256, 4, 8><<<grid, 256, base_lds_bytes<256, 4>(), st>>>(groups, ngroups, gctl, 0); break;
    case 1: k_base<512, 8, 6><<<grid, 512, base_lds_bytes<512, 8>(), st>>>(groups, ngroups, gctl, 1); break;
    case 2: k_base<1024, 8, 4><<<grid, 1024, base_lds_bytes<1024, 8>(), st>>>(groups, ngroups, gctl, 2); break;
    default: return hipErrorInvalidValue;
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    // the marked groups: 64 lanes sort up to 1024 keys, 256 up to 4096, 512 up to 8192
    Group* gm = const_cast<Group*>(groups);
    const size_t lds = (size_t)base_pad(kGroupClassCap[cls]) * 8;
    switch (cls) {
    case 0: k_base_slow<64><<<grid, 64, lds, st>>>(gm, ngroups, gctl, 0); break;
    case 1: k_base_slow<256><<<grid, 256, lds, st>>>(gm, ngroups, gctl, 1); break;
    case 2: k_base_slow<512><<<grid, 512, lds, st>>>(gm, ngroups, gctl, 2); break;
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
