// In-place partition round (Alg. 1 with fragments written back into the
// input, then Defragment), for sorts that cannot afford an n-key scratch
// buffer.  One round over the tasks of a round:
//
//   k_ip_frag     each workgroup streams its chunk of a task range and appends
//                 every key to its bucket's fragment of kIpBlock keys in LDS.
//                 A full fragment is written back into the chunk itself at a
//                 write head that never passes the read position (Alg. 1);
//                 the bucket of every written block, and its index among
//                 the chunk's full blocks of that bucket, are logged.  At the end of
//                 the chunk the partly filled fragments go to a side buffer
//                 and the rest of the chunk is marked empty.  Per (bucket,
//                 chunk) it counts keys and partial keys, and per bucket full
//                 blocks and min/max.
//   (scans, classify, layout as in the out-of-place round)
//   k_ip_plan     bucket b of a task owns the range [S_b, E_b) of the final
//                 layout; its full blocks go to the block-aligned slots
//                 [a_b, a_b + M'_b) inside it (at most one block that does
//                 not fit goes to an overflow block).
//   k_ip_dest     every full block's destination: the blocks of a bucket
//                 fill its slots in chunk order, then in their order inside
//                 a chunk (the counts' scans give where each chunk's run of
//                 them starts), so the permutation is fixed before it runs.
//   k_ip_permute  Defragment as a parallel block permutation: waves claim the
//                 slots of their share one by one (one claim word per slot),
//                 carry each block to its destination, and swap out a block
//                 that nobody has read yet.  A slot's word is touched by at
//                 most its reader and the one block bound for it.
//   k_ip_gather   the partial fragments and overflow blocks fill the rest of
//                 each bucket's range (its head before a_b and its tail after
//                 the placed blocks).
//
// Extra device memory per round: one u16 tag, one u32 index / destination
// and one u32 claim word per block of kIpBlock keys, a side buffer of at most min(chunk, fanout (kIpBlock - 1))
// keys per chunk (a task's fanout is at most its keys / (64 kIpBlock), and
// its chunks hold at least 64 x fanout blocks, so the side buffer is at most
// 1/64 of the keys), one overflow block (at most 1/64 of the keys in all)
// and a small table per bucket.
#include "lsort_device.h"

#include <algorithm>

#pragma clang fp contract(off)

namespace lsort {

constexpr uint32_t kIpThreads = 1024;
constexpr uint32_t kIpKpt = 4;
constexpr uint32_t kIpTile = kIpThreads * kIpKpt;
constexpr uint16_t kIpEmpty = 0xffffu;
constexpr uint32_t kIpSpinLimit = 1u << 22;

// Global slot of slot s of task i: tasks of a round occupy disjoint slot
// ranges floor(cnt_base / B) + i + [0, n / B).
__device__ __forceinline__ uint64_t ip_slot_off(const Task& T, uint32_t ti)
{
    return T.cnt_base / kIpBlock + ti;
}

// Rank of each valid lane's key among the keys of its bucket in this tile
// (an LDS atomic returns it).  Lanes that share a bucket in large groups
// (duplicate-heavy data) are peeled off first and ranked by one atomic per
// group.  Must be called by the whole wave.
__device__ __forceinline__ uint32_t wave_rank(uint32_t* cnt, uint32_t b, bool valid)
{
    bool mine = valid;
    uint32_t rank = 0;
    const uint64_t lt = (1ull << __lane_id()) - 1ull;
    const uint64_t act0 = __ballot(mine);
    if (act0) {
        const int lead0 = __ffsll((unsigned long long)act0) - 1;
        const uint32_t b0 = (uint32_t)__builtin_amdgcn_readlane((int)b, lead0);
        if ((uint32_t)__popcll(__ballot(mine && b == b0)) >= 8u) {
#pragma unroll 1
            for (int it = 0; it < 8; ++it) {
                const uint64_t act = __ballot(mine);
                if (!act)
                    break;
                const int leader = __ffsll((unsigned long long)act) - 1;
                const uint32_t bl = (uint32_t)__builtin_amdgcn_readlane((int)b, leader);
                const uint64_t grp = __ballot(mine && b == bl);
                const uint32_t c = (uint32_t)__popcll(grp);
                uint32_t base = 0;
                if ((int)__lane_id() == leader)
                    base = atomicAdd(&cnt[bl], c);
                base = (uint32_t)__builtin_amdgcn_readlane((int)base, leader);
                if (mine && b == bl) {
                    rank = base + (uint32_t)__popcll(grp & lt);
                    mine = false;
                }
                if (c < 8u)
                    break;
            }
        }
    }
    if (mine)
        rank = atomicAdd(&cnt[b], 1u);
    return rank;
}

// ------------------------------------------------------------- fragments --

struct IpFragLds {
    uint64_t* frag;     // F x kIpBlock keys
    uint32_t* fill;     // keys in each bucket's open fragment
    uint32_t* tcnt;     // keys of each bucket in the current tile
    uint32_t* bbase;    // first new block of each bucket in the tile (relative to the write head)
    uint32_t* nfull;    // new full blocks of each bucket in the tile
    uint32_t* fullc;    // full blocks of each bucket written by this chunk
    unsigned long long* mn;
    unsigned long long* mx;
    void* model;
};

__host__ __device__ inline size_t ip_frag_fixed_bytes(uint32_t f)
{
    return ((size_t)f * kIpBlock * 8 + (size_t)f * 5 * 4 + (size_t)f * 16 + 15) & ~(size_t)15;
}

__device__ __forceinline__ IpFragLds ip_frag_lds(unsigned char* smem, uint32_t f)
{
    IpFragLds L;
    L.frag = reinterpret_cast<uint64_t*>(smem);
    L.mn = reinterpret_cast<unsigned long long*>(L.frag + (size_t)f * kIpBlock);
    L.mx = L.mn + f;
    L.fill = reinterpret_cast<uint32_t*>(L.mx + f);
    L.tcnt = L.fill + f;
    L.bbase = L.tcnt + f;
    L.nfull = L.bbase + f;
    L.fullc = L.nfull + f;
    L.model = smem + ip_frag_fixed_bytes(f);
    return L;
}

template <uint32_t DT, bool MSD>
__device__ void ip_frag_body(const Task& T, const SModel& M, gptr<uint64_t> keys, uint32_t n,
                             gptr<uint16_t> tags, gptr<uint32_t> bidx, gptr<uint64_t> side, const IpFragLds& L,
                             uint32_t* wsum, uint32_t* s_wh, uint32_t flags)
{
    constexpr uint32_t NT = kIpThreads;
    const uint32_t f = T.fanout;
    const double scale = T.scale;
    const int32_t offset = (int32_t)T.offset;
    const uint32_t t = threadIdx.x;
    // the next tile's keys are loaded while this tile is processed: the
    // blocks a tile writes go below the keys read so far, so below the next
    // tile (Alg. 1's invariant), and the prefetched keys are still unread
    uint64_t nxt[kIpKpt];
#pragma unroll
    for (uint32_t u = 0; u < kIpKpt; ++u) {
        const uint32_t i = u * NT + t;
        nxt[u] = i < n ? keys[i] : 0;
    }
    for (uint32_t base = 0; base < n; base += kIpTile) {
        uint64_t raw[kIpKpt];
        uint32_t bk[kIpKpt], rk[kIpKpt];
#pragma unroll
        for (uint32_t u = 0; u < kIpKpt; ++u)
            raw[u] = nxt[u];
        if (base + kIpTile < n) {
#pragma unroll
            for (uint32_t u = 0; u < kIpKpt; ++u) {
                const uint32_t i = base + kIpTile + u * NT + t;
                nxt[u] = i < n ? keys[i] : 0;
            }
        }
#pragma unroll
        for (uint32_t u = 0; u < kIpKpt; ++u) {
            const uint32_t i = base + u * NT + t;
            const bool valid = i < n;
            const uint32_t b = MSD ? msd_bucket<DT>(raw[u], T.shift, f)
                                   : model_bucket<DT>(M, raw[u], scale, offset, f, flags);
            bk[u] = valid ? b : 0u;
            rk[u] = wave_rank(L.tcnt, b, valid);
            if (valid) {
                const unsigned long long o = to_ord(raw[u], DT);
                if (o < L.mn[b])
                    atomicMin(&L.mn[b], o);
                if (o > L.mx[b])
                    atomicMax(&L.mx[b], o);
            }
        }
        __syncthreads();
        // full blocks each bucket completes in this tile, numbered from the
        // write head in bucket order
        for (uint32_t b = t; b < f; b += NT)
            L.nfull[b] = (L.fill[b] + L.tcnt[b]) / kIpBlock;
        __syncthreads();
        const uint32_t newblocks = block_scan_u32(L.nfull, L.bbase, f, wsum);
        const uint32_t wh = *s_wh;
        // the next tile's loads are done by now: wait for them before this
        // tile's stores (vmcnt counts both), not at the loop's back edge
        __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);
        // the open fragment of a bucket that completes a block starts it
        for (uint32_t j = t; j < f * kIpBlock; j += NT) {
            const uint32_t b = j / kIpBlock, p = j % kIpBlock;
            if (L.nfull[b] && p < L.fill[b])
                keys[(uint64_t)(wh + L.bbase[b]) * kIpBlock + p] = L.frag[j];
        }
        for (uint32_t b = t; b < f; b += NT)
            for (uint32_t k = 0; k < L.nfull[b]; ++k) {
                tags[wh + L.bbase[b] + k] = (uint16_t)b;
                bidx[wh + L.bbase[b] + k] = L.fullc[b] + k;
            }
        __syncthreads();
        // keys of completed blocks go to them, the others open a fragment
#pragma unroll
        for (uint32_t u = 0; u < kIpKpt; ++u) {
            if (base + u * NT + t < n) {
                const uint32_t b = bk[u];
                const uint32_t slot = L.fill[b] + rk[u];
                const uint32_t inblocks = L.nfull[b] * kIpBlock;
                if (slot < inblocks)
                    keys[(uint64_t)(wh + L.bbase[b]) * kIpBlock + slot] = raw[u];
                else
                    L.frag[b * kIpBlock + (slot - inblocks)] = raw[u];
            }
        }
        __syncthreads();
        for (uint32_t b = t; b < f; b += NT) {
            L.fill[b] = L.fill[b] + L.tcnt[b] - L.nfull[b] * kIpBlock;
            L.fullc[b] += L.nfull[b];
            L.tcnt[b] = 0;
        }
        if (t == 0)
            *s_wh = wh + newblocks;
        __syncthreads();
    }
    // open fragments to the side buffer, in bucket order; the rest of the
    // chunk's slots are empty
    const uint32_t wh = *s_wh;
    const uint32_t tail = block_scan_u32(L.fill, L.bbase, f, wsum);
    for (uint32_t j = t; j < f * kIpBlock; j += NT) {
        const uint32_t b = j / kIpBlock, p = j % kIpBlock;
        if (p < L.fill[b])
            side[L.bbase[b] + p] = L.frag[j];
    }
    for (uint32_t s = wh + t; s < n / kIpBlock; s += NT)
        tags[s] = kIpEmpty;
    (void)tail;
}

__global__ __launch_bounds__(kIpThreads) void k_ip_frag(const Task* tasks, uint32_t ntasks, uint64_t chunk,
                                                        const double* models, uint32_t* cnt, uint32_t* pcnt,
                                                        uint32_t* fullb, uint64_t* bstat, uint16_t* tags,
                                                        uint32_t* bidx, uint64_t* side, uint32_t flags)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ uint32_t s_task, s_wh;
    __shared__ uint32_t wsum[kIpThreads / 64 + 1];
    if (threadIdx.x == 0) {
        s_task = find_task(tasks, ntasks, blockIdx.x);
        s_wh = 0;
    }
    __syncthreads();
    const uint32_t ti = s_task;
    const Task T = tasks[ti];
    const uint32_t f = T.fanout;
    const IpFragLds L = ip_frag_lds(smem, f);
    for (uint32_t b = threadIdx.x; b < f; b += blockDim.x) {
        L.fill[b] = 0;
        L.tcnt[b] = 0;
        L.fullc[b] = 0;
        L.mn[b] = ~0ull;
        L.mx[b] = 0;
    }
    SModel M{};
    const bool msd = T.kind == kMsd;
    if (!msd)
        load_model(M, models, T.model, T.leaves, L.model);
    __syncthreads();
    const uint32_t lc = blockIdx.x - T.chunk0;
    const uint64_t lo = (uint64_t)lc * chunk;   // a multiple of kIpBlock
    const uint32_t n = (uint32_t)(min(T.n, lo + chunk) - lo);
    const gptr<uint64_t> keys = as_global(T.keys + T.start + lo);
    const gptr<uint16_t> tg = as_global(tags + ip_slot_off(T, ti) + lo / kIpBlock);
    const gptr<uint32_t> bx = as_global(bidx + ip_slot_off(T, ti) + lo / kIpBlock);
    const gptr<uint64_t> sd = as_global(side + T.side_off + (uint64_t)lc * ip_side_keys(chunk, f));
    if (T.dtype == kF64) {
        if (msd) ip_frag_body<kF64, true>(T, M, keys, n, tg, bx, sd, L, wsum, &s_wh, flags);
        else ip_frag_body<kF64, false>(T, M, keys, n, tg, bx, sd, L, wsum, &s_wh, flags);
    } else {
        if (msd) ip_frag_body<kU64, true>(T, M, keys, n, tg, bx, sd, L, wsum, &s_wh, flags);
        else ip_frag_body<kU64, false>(T, M, keys, n, tg, bx, sd, L, wsum, &s_wh, flags);
    }
    __syncthreads();
    for (uint32_t b = threadIdx.x; b < f; b += blockDim.x) {
        const uint64_t e = T.cnt_off + (uint64_t)b * T.nchunks + lc;
        cnt[e] = L.fullc[b] * kIpBlock + L.fill[b];
        pcnt[e] = L.fill[b];
        if (L.fullc[b])
            atomicAdd(&fullb[T.bucket_off + b], L.fullc[b]);
        if (L.fullc[b] || L.fill[b]) {
            atomicMin((unsigned long long*)&bstat[2 * ((uint64_t)T.bucket_off + b)], L.mn[b]);
            atomicMax((unsigned long long*)&bstat[2 * ((uint64_t)T.bucket_off + b) + 1], L.mx[b]);
        }
    }
}

hipError_t launch_ip_frag(const Task* d_tasks, uint32_t ntasks, uint32_t total_chunks, uint64_t chunk,
                          const double* d_models, uint32_t* d_cnt, uint32_t* d_pcnt, uint32_t* d_fullb,
                          uint64_t* d_bstat, uint16_t* d_tags, uint32_t* d_bidx, uint64_t* d_side,
                          uint32_t max_fanout, uint32_t max_leaves, uint32_t flags, hipStream_t st)
{
    if (!total_chunks)
        return hipSuccess;
    if (max_fanout > kIpFanout)
        return hipErrorInvalidValue;
    const size_t smem = ip_frag_fixed_bytes(max_fanout) + model_lds_bytes(max_leaves);
    k_ip_frag<<<total_chunks, kIpThreads, smem, st>>>(d_tasks, ntasks, chunk, d_models, d_cnt, d_pcnt, d_fullb,
                                                      d_bstat, d_tags, d_bidx, d_side, flags);
    return hipGetLastError();
}

size_t ip_frag_lds_bytes(uint32_t fanout, uint32_t leaves)
{
    return ip_frag_fixed_bytes(fanout) + model_lds_bytes(leaves);
}

// ------------------------------------------------------------------ plan --

// The task that owns global bucket gb (tasks are laid out with increasing
// bucket_off).
__device__ __forceinline__ uint32_t find_task_of_bucket(const Task* tasks, uint32_t ntasks, uint64_t gb)
{
    uint32_t lo = 0, hi = ntasks;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (tasks[mid].bucket_off <= gb) lo = mid; else hi = mid;
    }
    return lo;
}

__global__ __launch_bounds__(256) void k_ip_plan(const Task* tasks, uint32_t ntasks, uint64_t nbuckets,
                                                 const uint64_t* pos, const uint32_t* fullb, IpBucket* bk)
{
    const uint64_t gb = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    if (gb >= nbuckets)
        return;
    const uint32_t ti = find_task_of_bucket(tasks, ntasks, gb);
    const Task T = tasks[ti];
    const uint32_t b = (uint32_t)(gb - T.bucket_off);
    const uint64_t S = pos[T.cnt_off + (uint64_t)b * T.nchunks] - T.cnt_base;
    const uint64_t E = b + 1 < T.fanout ? pos[T.cnt_off + (uint64_t)(b + 1) * T.nchunks] - T.cnt_base : T.n;
    // (a bucket that starts in the range's last, partial block has no slot:
    // its area is empty and all its keys are rest keys)
    const uint64_t nslots = T.n / kIpBlock;
    const uint64_t a = (S + kIpBlock - 1) / kIpBlock;
    const uint64_t area = min(a, nslots);
    const uint64_t a_next = b + 1 < T.fanout ? min((E + kIpBlock - 1) / kIpBlock, nslots) : nslots;
    const uint64_t fit = E / kIpBlock > a ? E / kIpBlock - a : 0;
    const uint64_t m = fullb[gb];
    const uint64_t placed = m < fit ? m : fit;
    (void)a_next;
    IpBucket B;
    B.start = S;
    B.end = E;
    B.a = (uint32_t)a;
    B.area = (uint32_t)area;
    B.dend = (uint32_t)(a + placed);
    B.full = (uint32_t)m;
    B.task = ti;
    bk[gb] = B;
}

hipError_t launch_ip_plan(const Task* d_tasks, uint32_t ntasks, uint64_t nbuckets, const uint64_t* d_pos,
                          const uint32_t* d_fullb, IpBucket* d_bk, hipStream_t st)
{
    if (!nbuckets)
        return hipSuccess;
    k_ip_plan<<<(uint32_t)((nbuckets + 255) / 256), 256, 0, st>>>(d_tasks, ntasks, nbuckets, d_pos, d_fullb, d_bk);
    return hipGetLastError();
}

// --------------------------------------------------------------- permute --

// A value every lane of the wave holds (or lane 0's), in a scalar register,
// so that branches on it are uniform.
__device__ __forceinline__ uint64_t ip_uni64(uint64_t v)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(v >> 32));
    return (uint64_t)lo | ((uint64_t)hi << 32);
}

__device__ __forceinline__ uint32_t ip_uni32(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_readfirstlane((int)v);
}

// The key range of a task, as a wave-uniform pointer.
__device__ __forceinline__ uint64_t* uni_keys(const Task& T)
{
    return (uint64_t*)ip_uni64((uint64_t)(T.keys + T.start));
}

// Lane 0: wait (bounded) until the reader that claimed a slot has its block
// in registers (the slot's word holds `rel`); a wait that runs out raises
// the control block's overflow bit 2 (the sort then reports an error)
// instead of hanging.  The only hazard is the reader's load against the
// waiter's later store to the same slot, so plain atomic loads do: no
// acquire (on this GPU an agent-scope acquire invalidates the L2).
__device__ __forceinline__ void ip_wait_released(uint32_t* flag, uint32_t rel, RoundCtl* ctl)
{
    if (threadIdx.x % 64 == 0) {
        uint32_t spins = 0;
        while (__hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != rel) {
            if (++spins >= kIpSpinLimit) {
                atomicOr(&ctl->overflow, 2u);
                break;
            }
            __builtin_amdgcn_s_sleep(2);
        }
    }
}

// Release a slot that was read: once its block is in registers (every load
// of the wave has returned), the word says so.  Nothing written before needs
// to be seen by the waiter, so no fence (an agent-scope release would write
// the L2 back).
__device__ __forceinline__ void ip_release(uint32_t* flag, uint32_t rel)
{
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_waitcnt(0);
    asm volatile("" ::: "memory");
    if (threadIdx.x % 64 == 0)
        __hip_atomic_store(flag, rel, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// The task whose slot range holds global slot g: the last task whose slots
// start at or before it (tasks are laid out with increasing slot offsets;
// one slot between tasks belongs to none).
__device__ __forceinline__ uint32_t find_task_of_slot(const Task* tasks, uint32_t ntasks, uint64_t g)
{
    uint32_t lo = 0, hi = ntasks;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (ip_slot_off(tasks[mid], mid) <= g) lo = mid; else hi = mid;
    }
    return lo;
}

// Destination of every full block, in place of its index: block j of bucket
// b written by chunk c goes to slot a_b + (full blocks of b in chunks before
// c) + j, the full blocks of earlier chunks coming from the scans of the key
// and partial-key counts; past the bucket's placed blocks it is the block
// that does not fit.  Slots without a full block get kIpNoDest.
__global__ __launch_bounds__(256) void k_ip_dest(const Task* tasks, uint32_t ntasks, uint64_t gslots, uint64_t chunk,
                                                 const IpBucket* bk, const uint64_t* pos, const uint64_t* ppos,
                                                 const uint16_t* tags, uint32_t* bidx)
{
    const uint64_t g = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    if (g >= gslots)
        return;
    const uint32_t ti = find_task_of_slot(tasks, ntasks, g);
    const Task& T = tasks[ti];
    const uint64_t s = g - ip_slot_off(T, ti);
    if (s >= T.n / kIpBlock)
        return;                         // the slot between two tasks: never read
    const uint16_t tag = tags[g];
    uint32_t d = kIpNoDest;
    if (tag != kIpEmpty) {
        const uint64_t c = s / (chunk / kIpBlock);
        const uint64_t e0 = T.cnt_off + (uint64_t)tag * T.nchunks, e = e0 + c;
        const uint64_t before = ((pos[e] - pos[e0]) - (ppos[e] - ppos[e0])) / kIpBlock;
        const IpBucket& B = bk[T.bucket_off + tag];
        const uint64_t k = before + bidx[g];
        d = k < (uint64_t)(B.dend - B.a) ? (uint32_t)(B.a + k) : (kIpOvf | tag);
    }
    bidx[g] = d;
}

// Lane 0 swaps a slot's claim word to `cl`; the word it held, in a scalar.
__device__ __forceinline__ uint32_t ip_claim(uint32_t* w, uint32_t cl)
{
    uint32_t old = 0;
    if (threadIdx.x % 64 == 0)
        old = __hip_atomic_exchange(w, cl, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return ip_uni32(old);
}

// Every wave takes an equal share of the round's global slots and claims
// each of them in turn; a slot already claimed this round (as some block's
// destination) is skipped.  The block of a claimed slot is loaded, the slot
// released, and the block carried to its destination: if that slot was
// claimed by its reader, the wave waits for the release (bounded) and
// stores; if it is unclaimed, the wave claims it, swaps its block out and
// carries that one on.  Each destination is the destination of one block
// only, so a slot's word is swapped by at most its reader and that one
// writer: claim words hold 2 epoch (claimed) and 2 epoch + 1 (released);
// words of earlier rounds are smaller.  No word is shared by more than two
// waves, so there is no queue on any address.  The lane l of a wave holds
// key l of the block in hand; all control flow is on wave-uniform values.
__global__ __launch_bounds__(256) void k_ip_permute(const Task* tasks, uint32_t ntasks, uint64_t gslots,
                                                    const uint32_t* dest, uint32_t* word, uint64_t* ovf,
                                                    uint32_t epoch, RoundCtl* ctl)
{
    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t nw = (uint64_t)gridDim.x * (256 / 64);
    const uint64_t w = (uint64_t)blockIdx.x * (256 / 64) + (threadIdx.x >> 6);
    const uint64_t seg_lo = gslots * w / nw, seg_hi = gslots * (w + 1) / nw;
    if (seg_lo >= seg_hi)
        return;
    const uint32_t cl = 2u * epoch, rel = 2u * epoch + 1u;
    const gptr<const uint32_t> gdest = as_global(dest);
    uint32_t ti = ip_uni32(find_task_of_slot(tasks, ntasks, seg_lo));
    for (uint64_t g = seg_lo; g < seg_hi; ++g) {
        while (ti + 1 < ntasks && ip_uni64(ip_slot_off(tasks[ti + 1], ti + 1)) <= g)
            ++ti;
        const uint64_t soff = ip_uni64(ip_slot_off(tasks[ti], ti));
        const uint64_t nslots = ip_uni64(tasks[ti].n / kIpBlock);
        if (g - soff >= nslots)
            continue;                   // the slot between two tasks
        if (ip_claim(word + g, cl) >= cl)
            continue;                   // taken this round as a destination
        const gptr<uint64_t> base = as_global(uni_keys(tasks[ti]));
        const uint64_t bucket_off = ip_uni64(tasks[ti].bucket_off);
        uint32_t d = ip_uni32(gdest[g]);
        uint64_t key = 0;
        if (d != kIpNoDest)
            key = base[(g - soff) * kIpBlock + lane];
        ip_release(word + g, rel);
        bool carrying = d != kIpNoDest && d != (uint32_t)(g - soff);   // (a block already in place stays)
        while (carrying) {
            if (d & kIpOvf) {
                // the bucket's block that does not fit
                ovf[(bucket_off + (d & ~kIpOvf)) * kIpBlock + lane] = key;
                break;
            }
            const uint64_t dg = soff + d;
            const uint32_t old = ip_claim(word + dg, cl);
            if (old >= cl) {
                // its reader has it (or had it): store once it is released
                if (old != rel)
                    ip_wait_released(word + dg, rel, ctl);
                base[(uint64_t)d * kIpBlock + lane] = key;
                break;
            }
            // unclaimed: swap its block out and carry that one
            const uint32_t d2 = ip_uni32(gdest[dg]);
            uint64_t k2 = 0;
            if (d2 != kIpNoDest)
                k2 = base[(uint64_t)d * kIpBlock + lane];
            __builtin_amdgcn_s_waitcnt(0);
            base[(uint64_t)d * kIpBlock + lane] = key;
            key = k2;
            d = d2;
            carrying = d2 != kIpNoDest;
        }
    }
}

hipError_t launch_ip_permute(const Task* d_tasks, uint32_t ntasks, uint64_t gslots, uint64_t chunk,
                             const IpBucket* d_bk, const uint64_t* d_pos, const uint64_t* d_ppos,
                             const uint16_t* d_tags, uint32_t* d_bidx, uint32_t* d_word, uint64_t* d_ovf,
                             uint32_t epoch, RoundCtl* d_ctl, hipStream_t st)
{
    if (!gslots || !ntasks)
        return hipSuccess;
    k_ip_dest<<<(uint32_t)((gslots + 255) / 256), 256, 0, st>>>(d_tasks, ntasks, gslots, chunk, d_bk, d_pos, d_ppos,
                                                               d_tags, d_bidx);
    // about one wave per 32 slots, at most 32 waves per CU (all resident)
    const uint64_t waves = std::min<uint64_t>(std::max<uint64_t>(gslots / 32, 1), 256ull * 32);
    const uint32_t grid = (uint32_t)((waves + 3) / 4);
    k_ip_permute<<<grid, 256, 0, st>>>(d_tasks, ntasks, gslots, d_bidx, d_word, d_ovf, epoch, d_ctl);
    return hipGetLastError();
}

// ---------------------------------------------------------------- gather --

// Position (relative to the task range) of the k-th key of bucket B that is
// not in a placed block: first the head [S, min(a B, E)), then the tail from
// the end of the placed blocks.
__device__ __forceinline__ uint64_t ip_rest_pos(const IpBucket& B, uint64_t k)
{
    const uint64_t ab = (uint64_t)B.a * kIpBlock;
    const uint64_t head = (ab < B.end ? ab : B.end) - B.start;
    return k < head ? B.start + k : (uint64_t)B.dend * kIpBlock + (k - head);
}

// One workgroup per chunk: its open fragments (side buffer, bucket order) go
// to the rest positions of their buckets, after the earlier chunks' ones.
__global__ __launch_bounds__(256) void k_ip_gather(const Task* tasks, uint32_t ntasks, uint64_t chunk,
                                                   const uint32_t* pcnt, const uint64_t* ppos, const IpBucket* bk,
                                                   const uint64_t* side)
{
    __shared__ uint32_t s_task;
    __shared__ uint32_t s_pre[kIpFanout + 1];
    __shared__ uint64_t s_off[kIpFanout];
    __shared__ uint32_t wsum[256 / 64 + 1];
    if (threadIdx.x == 0)
        s_task = find_task(tasks, ntasks, blockIdx.x);
    __syncthreads();
    const Task T = tasks[s_task];
    const uint32_t f = T.fanout;
    const uint32_t lc = blockIdx.x - T.chunk0;
    for (uint32_t b = threadIdx.x; b < f; b += 256) {
        const uint64_t e = T.cnt_off + (uint64_t)b * T.nchunks;
        s_pre[b] = pcnt[e + lc];
        s_off[b] = ppos[e + lc] - ppos[e];     // this chunk's place among the bucket's partial keys
    }
    __syncthreads();
    const uint32_t tail = block_scan_u32(s_pre, f, wsum);
    if (threadIdx.x == 0)
        s_pre[f] = tail;
    __syncthreads();
    const gptr<const uint64_t> sd = as_global(side + T.side_off + (uint64_t)lc * ip_side_keys(chunk, f));
    const gptr<uint64_t> base = as_global(T.keys + T.start);
    for (uint32_t j = threadIdx.x; j < tail; j += 256) {
        uint32_t l = 0, h = f;            // s_pre[l] <= j < s_pre[h]
        while (h - l > 1) {
            const uint32_t mid = (l + h) >> 1;
            if (s_pre[mid] <= j) l = mid; else h = mid;
        }
        const IpBucket B = bk[T.bucket_off + l];
        base[ip_rest_pos(B, s_off[l] + (j - s_pre[l]))] = sd[j];
    }
}

// The overflow block of each bucket (if any) goes after its partial keys.
__global__ __launch_bounds__(64) void k_ip_gather_ovf(const Task* tasks, const IpBucket* bk, const uint64_t* ovf)
{
    const uint64_t gb = blockIdx.x;
    const IpBucket B = bk[gb];
    const uint32_t placed = B.dend - B.a;
    if (B.full <= placed)
        return;     // (at most one block per bucket does not fit)
    const Task& T = tasks[B.task];
    const uint64_t partial = (B.end - B.start) - (uint64_t)B.full * kIpBlock;
    as_global(T.keys + T.start)[ip_rest_pos(B, partial + threadIdx.x)] = ovf[gb * kIpBlock + threadIdx.x];
}

hipError_t launch_ip_gather(const Task* d_tasks, uint32_t ntasks, uint32_t total_chunks, uint64_t chunk,
                            uint64_t nbuckets, const uint32_t* d_pcnt, const uint64_t* d_ppos, const IpBucket* d_bk,
                            const uint64_t* d_side, const uint64_t* d_ovf, hipStream_t st)
{
    if (total_chunks)
        k_ip_gather<<<total_chunks, 256, 0, st>>>(d_tasks, ntasks, chunk, d_pcnt, d_ppos, d_bk, d_side);
    if (nbuckets)
        k_ip_gather_ovf<<<(uint32_t)nbuckets, 64, 0, st>>>(d_tasks, d_bk, d_ovf);
    return hipGetLastError();
}

}  // namespace lsort
