// Partition rounds (Alg. 1 as count-then-place, Alg. 2's recursion):
// histogram, classify, layout of the next round, scatter.
#include "lsort_device.h"

#pragma clang fp contract(off)

namespace lsort {

__global__ void k_round_init(uint64_t* bstat, uint64_t nbuckets, RoundCtl* ctl, bool snapshot)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    // ctl->buckets is not written by this kernel.  Its count is the last
    // layout's, which never exceeds the buffer (zero after an overflow);
    // when the round has no task it is stale and only clears more.
    if (snapshot)
        nbuckets = ctl->buckets;
    if (i == 0) {
        if (snapshot) {
            // a round without tasks runs nothing: its stale layout fields are ignored
            const bool any = ctl->ntasks != 0;
            LiveCounts c;
            c.chunk = ctl->chunk;
            c.nkeys = any ? ctl->nkeys : 0;
            c.entries = any ? ctl->entries : 0;
            c.samples = any ? ctl->samples : 0;
            c.max_sample = any ? ctl->max_sample : 0;
            c.buckets = any ? ctl->buckets : 0;
            c.ntasks = ctl->ntasks;
            c.chunks = any ? ctl->chunks : 0;
            c.njobs = any ? ctl->njobs : 0;
            c.blocks = any ? ctl->blocks : 0;
            c.max_fanout = ctl->max_fanout;
            c.max_leaves = ctl->max_leaves;
            ctl->cur = c;
        }
        ctl->ntasks = 0;
        ctl->classified = 0;
    }
    if (i < nbuckets) {
        bstat[2 * i] = ~0ull;
        bstat[2 * i + 1] = 0;
    }
}

hipError_t launch_round_init(uint64_t* d_bstat, uint64_t nbuckets, RoundCtl* d_ctl, bool snapshot, hipStream_t st)
{
    k_round_init<<<(uint32_t)((nbuckets + 255) / 256 + 1), 256, 0, st>>>(d_bstat, nbuckets, d_ctl, snapshot);
    return hipGetLastError();
}

// ---------------------------------------------------------------- upload --

// The staged counts are read over the bus by every workgroup; the words of
// all lists are then copied grid-stride.
__global__ __launch_bounds__(256) void k_upload(UploadPlan U)
{
    const RoundCtl* c0 = reinterpret_cast<const RoundCtl*>(U.stage);
    uint64_t end[3 + kGroupClasses];
    const uint64_t nctl = sizeof(RoundCtl) / 8;
    end[0] = nctl;
    end[1] = end[0] + (uint64_t)c0->ntasks * (sizeof(Task) / 8);
    end[2] = end[1] + (uint64_t)c0->cur.njobs * (sizeof(ModelJob) / 8);
    for (uint32_t c = 0; c < kGroupClasses; ++c)
        end[3 + c] = end[2 + c] + (uint64_t)c0->ngroups[c] * (sizeof(Group) / 8);
    const uint64_t* w = reinterpret_cast<const uint64_t*>(U.stage);
    for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < end[2 + kGroupClasses];
         i += (uint64_t)gridDim.x * 256) {
        if (i < end[0]) {
            reinterpret_cast<uint64_t*>(U.ctl)[i] = w[i];
        } else if (i < end[1]) {
            reinterpret_cast<uint64_t*>(U.tasks)[i - end[0]] = w[U.off_tasks / 8 + (i - end[0])];
        } else if (i < end[2]) {
            reinterpret_cast<uint64_t*>(U.jobs)[i - end[1]] = w[U.off_jobs / 8 + (i - end[1])];
        } else {
            uint32_t c = 0;
            while (i >= end[3 + c])
                ++c;
            reinterpret_cast<uint64_t*>(U.groups[c])[i - end[2 + c]] = w[U.off_groups[c] / 8 + (i - end[2 + c])];
        }
    }
}

hipError_t launch_upload(const UploadPlan& U, hipStream_t st)
{
    k_upload<<<16, 256, 0, st>>>(U);
    return hipGetLastError();
}

// ------------------------------------------------------------- histogram --

// Bucket sizes per (bucket, chunk) plus per-bucket min/max of the key words
// (Alg. 1 S_B, and the all-equal test of Alg. 2).  A workgroup of 1024 lanes
// streams its chunk; the next 4096 keys are loaded while the current ones are
// classified, so loads stay in flight through the LDS work.
constexpr uint32_t kHistThreads = 1024;
constexpr uint32_t kHistUnroll = 4;
constexpr uint32_t kPeelMin = 8;   // lanes on one bucket before a wave merges them

// Count one key per valid lane.  When many lanes of the wave hit the same
// bucket (duplicate-heavy data), same-address LDS atomics serialise lane by
// lane, so the largest groups are peeled off with two ballots and counted by
// a single atomic.  Must be called by the whole wave.
__device__ __forceinline__ void wave_count(uint32_t* h, uint32_t b, bool valid)
{
    bool mine = valid;
    const uint64_t act0 = __ballot(mine);
    if (act0) {
        const int lead0 = __ffsll((unsigned long long)act0) - 1;
        const uint32_t b0 = (uint32_t)__builtin_amdgcn_readlane((int)b, lead0);
        if ((uint32_t)__popcll(__ballot(mine && b == b0)) >= kPeelMin) {
#pragma unroll 1
            for (int it = 0; it < 8; ++it) {
                const uint64_t act = __ballot(mine);
                if (!act)
                    break;
                const int leader = __ffsll((unsigned long long)act) - 1;
                const uint32_t bl = (uint32_t)__builtin_amdgcn_readlane((int)b, leader);
                const uint64_t grp = __ballot(mine && b == bl);
                const uint32_t c = (uint32_t)__popcll(grp);
                if ((int)__lane_id() == leader)
                    atomicAdd(&h[bl], c);
                if (b == bl)
                    mine = false;
                if (c < kPeelMin)
                    break;
            }
        }
    }
    if (mine)
        atomicAdd(&h[b], 1u);
}

template <uint32_t DT, bool MSD>
__device__ __forceinline__ void hist_body(const Task& T, const SModel& M, gptr<const uint64_t> src, uint32_t cnt,
                                          uint32_t* h, unsigned long long* mn, unsigned long long* mx,
                                          uint32_t flags)
{
    constexpr uint32_t STEP = kHistThreads * kHistUnroll;
    const double scale = T.scale;
    const int32_t offset = (int32_t)T.offset;
    const uint32_t fanout = T.fanout;
    const uint32_t shift = T.shift;
    uint64_t nxt[kHistUnroll];
#pragma unroll
    for (uint32_t u = 0; u < kHistUnroll; ++u) {
        const uint32_t i = u * kHistThreads + threadIdx.x;
        nxt[u] = i < cnt ? src[i] : 0;
    }
    for (uint32_t base = 0; base < cnt; base += STEP) {
        uint64_t raw[kHistUnroll];
#pragma unroll
        for (uint32_t u = 0; u < kHistUnroll; ++u)
            raw[u] = nxt[u];
        if (base + STEP < cnt) {
#pragma unroll
            for (uint32_t u = 0; u < kHistUnroll; ++u) {
                const uint32_t i = base + STEP + u * kHistThreads + threadIdx.x;
                nxt[u] = i < cnt ? src[i] : 0;
            }
        }
#pragma unroll
        for (uint32_t u = 0; u < kHistUnroll; ++u) {
            const uint32_t i = base + u * kHistThreads + threadIdx.x;
            const bool valid = i < cnt;
            const uint32_t b = MSD ? msd_bucket<DT>(raw[u], shift, fanout)
                                   : model_bucket<DT>(M, raw[u], scale, offset, fanout, flags);
            wave_count(h, b, valid);
            if (valid) {
                // Only a new extreme needs an atomic: min only falls and max
                // only rises, so a stale read can cause an extra atomic but
                // never a missed one.
                const unsigned long long o = to_ord(raw[u], DT);
                if (o < mn[b])
                    atomicMin(&mn[b], o);
                if (o > mx[b])
                    atomicMax(&mx[b], o);
            }
        }
    }
}

__global__ __launch_bounds__(kHistThreads) void k_hist(const Task* tasks, uint32_t ntasks, uint64_t chunk,
                                                       const double* models, uint32_t* cnt, uint64_t* bstat,
                                                       uint32_t flags, const LiveCounts* live)
{
    if (live) {
        if (blockIdx.x >= live->chunks)
            return;
        ntasks = live->ntasks;
        chunk = live->chunk;
    }
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
    void* mlds = smem + (((size_t)f * 20 + 15) & ~(size_t)15);
    for (uint32_t b = threadIdx.x; b < f; b += blockDim.x) {
        h[b] = 0;
        mn[b] = ~0ull;
        mx[b] = 0;
    }
    SModel M{};
    const bool msd = T.kind == kMsd;
    if (!msd)
        load_model(M, models, T.model, T.leaves, mlds);
    __syncthreads();
    const uint32_t lc = blockIdx.x - T.chunk0;
    const uint64_t lo = (uint64_t)lc * chunk;
    const uint32_t n = (uint32_t)(min(T.n, lo + chunk) - lo);
    const gptr<const uint64_t> src = as_global<const uint64_t>((T.src ? T.scratch : T.keys) + T.start + lo);
    if (T.dtype == kF64) {
        if (msd) hist_body<kF64, true>(T, M, src, n, h, mn, mx, flags);
        else hist_body<kF64, false>(T, M, src, n, h, mn, mx, flags);
    } else {
        if (msd) hist_body<kU64, true>(T, M, src, n, h, mn, mx, flags);
        else hist_body<kU64, false>(T, M, src, n, h, mn, mx, flags);
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

hipError_t launch_hist(const Task* d_tasks, uint32_t ntasks, uint32_t total_chunks, uint64_t chunk,
                       const double* d_models, uint32_t* d_cnt, uint64_t* d_bstat,
                       uint32_t max_fanout, uint32_t max_leaves, uint32_t flags, const LiveCounts* live,
                       hipStream_t st)
{
    if (!total_chunks)
        return hipSuccess;
    size_t smem = (((size_t)max_fanout * 20 + 15) & ~(size_t)15) + model_lds_bytes(max_leaves);
    k_hist<<<total_chunks, kHistThreads, smem, st>>>(d_tasks, ntasks, chunk, d_models, d_cnt, d_bstat, flags,
                                                     live);
    return hipGetLastError();
}

// -------------------------------------------------------------- classify --

// Classify every bucket of a task: empty, all-equal (filled with its value,
// never moved again), small (sorted in LDS together with its neighbours),
// solo (more than `thresh` but fewer than 2*thresh keys: sorted in LDS as a
// group of its own) or over-full (a task of the next round).  Small buckets
// hold at most `thresh` keys; consecutive small buckets whose starts fall into
// the same window of group_window(thresh) keys form one group, so a group
// holds fewer than 2*thresh keys.  The buckets of a group are already in
// order, so a small window keeps the LDS sorts short (the base case's
// network grows as log^2 of the group).  Everything is decided with
// block-wide scans, no serial walk.
enum : uint8_t { kEmpty = 0, kSmall = 1, kFillB = 2, kBig = 3, kSolo = 4, kLead = 0x80 };

constexpr int32_t kNone = 0x7fffffff;

// ---------------------------------------------------------------- layout --

// Lay out the next round on the device (any block size, multiple of 64 up to
// 1024): chunk size, each task's chunk / bucket / count-matrix offsets, and a
// training job (sample size, leaves, table offsets) for every task that
// needs a local model.  The host only reads the totals back.
constexpr uint32_t kLayoutQ = 10;

__device__ void layout_device(Task* tasks, ModelJob* jobs, const LayoutParams& lp, RoundCtl* ctl,
                              RoundCtl* host_ctl)
{
    __shared__ unsigned long long s_keys, s_maxm;
    __shared__ uint32_t s_maxf, s_maxl, s_maxlev;
    __shared__ uint64_t wsum[kLayoutQ][16];
    __shared__ uint64_t carry[kLayoutQ];
    const uint32_t NT = blockDim.x;
    // after an overflow the lists are incomplete: lay out nothing
    const uint32_t nt = ctl->overflow ? 0u : ctl->ntasks;
    if (threadIdx.x == 0) {
        s_keys = 0;
        s_maxm = 0;
        s_maxf = 2;
        s_maxl = 1;
        s_maxlev = 0;
    }
    if (threadIdx.x < kLayoutQ)
        carry[threadIdx.x] = 0;
    __syncthreads();
    unsigned long long mykeys = 0;
    uint32_t maxf = 2, maxl = 1, maxlev = 0;
    for (uint32_t i = threadIdx.x; i < nt; i += NT) {
        mykeys += tasks[i].n;
        maxf = max(maxf, tasks[i].fanout);
        maxlev = max(maxlev, tasks[i].level);
        if (tasks[i].kind == kGlobal || tasks[i].kind == kGlobalL1)
            maxl = max(maxl, tasks[i].leaves);
    }
    // one LDS atomic per wave: same-address atomics serialise lane by lane
    mykeys = wave_sum(mykeys);
    maxf = wave_max(maxf);
    maxl = wave_max(maxl);
    maxlev = wave_max(maxlev);
    if ((threadIdx.x & 63u) == 0) {
        atomicAdd(&s_keys, mykeys);
        atomicMax(&s_maxf, maxf);
        atomicMax(&s_maxl, maxl);
        atomicMax(&s_maxlev, maxlev);
    }
    __syncthreads();
    const uint64_t nkeys = s_keys;
    // a large round scatters in wide tiles when its fanouts leave room in LDS
    const uint32_t tile =
        lp.tile_wide && nkeys >= lp.wide_keys && s_maxf <= lp.wide_max_fanout &&
                (lp.tile_wide != kTile12 || nkeys < (1ull << 31))
            ? lp.tile_wide : lp.tile;
    // at most lp.target_chunks chunks; a small round gets about one chunk
    // per CU, of one to four tiles
    uint64_t chunk = (nkeys + lp.target_chunks - 1) / lp.target_chunks;
    uint64_t small = (nkeys + kSmallRoundChunks - 1) / kSmallRoundChunks;
    small = small < tile ? tile : (small > 4ull * tile ? 4ull * tile : small);
    chunk = chunk > small ? chunk : small;
    // in-place rounds: chunks of at least kIpChunkBlocks x fanout blocks, so
    // that the open fragments at their ends stay a small fraction of the keys
    if (lp.inplace) {
        const uint64_t least = kIpChunkBlocks * s_maxf * kIpBlock;
        chunk = chunk > least ? chunk : least;
    }
    chunk = (chunk + tile - 1) / tile * tile;
    const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
    uint32_t my_maxl = 1;
    unsigned long long my_maxm = 0;
    for (uint32_t base = 0; base < nt; base += NT) {
        const uint32_t i = base + threadIdx.x;
        const bool valid = i < nt;
        Task T{};
        if (valid)
            T = tasks[i];
        const bool local = valid && T.kind == kLocal;
        uint64_t m = 0;
        uint32_t L = 0;
        if (local) {
            const double want = ceil(lp.rate * (double)T.n);
            m = want < 1.0 ? 1u : (uint64_t)want;
            const uint64_t floor_m = T.n < kLocalMinSample ? T.n : kLocalMinSample;
            m = m > floor_m ? m : floor_m;
            if (lp.cap && m > lp.cap)
                m = lp.cap > floor_m ? lp.cap : floor_m;
            // about 8 sample keys per leaf (the knot of a repeated value
            // needs m/L copies), at most the caller's leaves
            const uint64_t want_l = m / 8 ? m / 8 : 1;
            L = (uint32_t)(want_l < lp.leaves ? want_l : lp.leaves);
            // in-place rounds split many small ranges with small fanouts:
            // their models get 8 leaves per bucket
            if (lp.inplace)
                L = min(L, max(kIpMinLeaves, 8u * T.fanout));
            my_maxl = max(my_maxl, L);
            my_maxm = max(my_maxm, (unsigned long long)m);
        }
        const uint64_t nch = valid ? (T.n + chunk - 1) / chunk : 0;
        // a job whose sample fits one LDS run trains in one workgroup and
        // takes no room in the sample buffers and leaf tables
        const bool sampled = local && m > kSampleBlock;
        uint64_t q[kLayoutQ] = {nch,
                                valid ? T.fanout : 0u,
                                valid ? (uint64_t)T.fanout * nch : 0u,
                                valid ? T.n : 0u,
                                local ? 1u : 0u,
                                sampled ? m : 0u,
                                sampled ? L : 0u,
                                local ? model_doubles(L) : 0u,
                                sampled ? (m + kSampleBlock - 1) / kSampleBlock : 0u,
                                lp.inplace && valid ? nch * ip_side_keys(chunk, T.fanout) : 0u};
        uint64_t x[kLayoutQ];
#pragma unroll
        for (uint32_t j = 0; j < kLayoutQ; ++j) {
            x[j] = q[j];
#pragma unroll
            for (uint32_t d = 1; d < 64; d <<= 1) {
                const uint64_t y = __shfl_up(x[j], d, 64);
                if (lane >= d)
                    x[j] += y;
            }
            if (lane == 63)
                wsum[j][wave] = x[j];
        }
        __syncthreads();
        if (threadIdx.x < kLayoutQ) {
            uint64_t run = carry[threadIdx.x];
            for (uint32_t w = 0; w < NT / 64; ++w) {
                const uint64_t v = wsum[threadIdx.x][w];
                wsum[threadIdx.x][w] = run;
                run += v;
            }
            carry[threadIdx.x] = run;
        }
        __syncthreads();
        uint64_t off[kLayoutQ];
#pragma unroll
        for (uint32_t j = 0; j < kLayoutQ; ++j)
            off[j] = wsum[j][wave] + x[j] - q[j];
        if (valid) {
            T.chunk0 = (uint32_t)off[0];
            T.nchunks = (uint32_t)nch;
            T.bucket_off = off[1];
            T.cnt_off = off[2];
            T.cnt_base = off[3];
            T.side_off = off[9];
            if (local) {
                T.leaves = L;
                T.model = lp.model_base + off[7];
                ModelJob J;
                J.src = (T.src ? T.scratch : T.keys) + T.start;
                J.n = T.n;
                J.m = m;
                J.seed = splitmix64_at(lp.seed ^ (T.start * 0x9e3779b97f4a7c15ull) ^ ((uint64_t)T.seg << 40),
                                       T.level);
                J.sample_off = off[5];
                J.model_off = T.model;
                J.leaf_off = off[6];
                J.leaves = L;
                J.dtype = T.dtype;
                J.block0 = (uint32_t)off[8];
                J.nblocks = sampled ? (uint32_t)((m + kSampleBlock - 1) / kSampleBlock) : 0u;
                jobs[off[4]] = J;
            }
            tasks[i] = T;
        }
        __syncthreads();
    }
    my_maxl = wave_max(my_maxl);
    my_maxm = wave_max(my_maxm);
    if (lane == 0) {
        atomicMax(&s_maxl, my_maxl);
        atomicMax(&s_maxm, my_maxm);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const bool over = ctl->overflow || nkeys > lp.cap_keys || carry[0] > lp.cap_chunks ||
                          carry[1] > lp.cap_buckets || carry[2] > lp.cap_entries || carry[4] > lp.cap_tasks ||
                          carry[5] > lp.cap_samples || carry[6] > lp.cap_leafs || carry[7] > lp.cap_models ||
                          carry[8] > lp.cap_blocks;
        if (over) {
            // no next round: every size it would be launched with is zero
            ctl->overflow = 1;
            ctl->ntasks = 0;
            for (uint32_t j = 0; j < kLayoutQ; ++j)
                carry[j] = 0;
        }
        ctl->chunk = chunk;
        ctl->tile = tile;
        ctl->nkeys = over ? 0 : nkeys;
        ctl->chunks = (uint32_t)carry[0];
        ctl->buckets = carry[1];
        ctl->entries = carry[2];
        ctl->njobs = (uint32_t)carry[4];
        ctl->samples = carry[5];
        ctl->leafs = carry[6];
        ctl->models = carry[7];
        ctl->blocks = (uint32_t)carry[8];
        ctl->side_keys = carry[9];
        ctl->max_fanout = s_maxf;
        ctl->max_leaves = s_maxl;
        ctl->max_level = s_maxlev;
        ctl->max_sample = s_maxm;
        if (nt && !over) {
            ctl->rounds += 1;
            ctl->tasks_total += nt;
        }
        ctl->deepest = max(ctl->deepest, s_maxlev);
        __threadfence();
    }
    __syncthreads();
    // publish to the host without a copy: one word per lane, read from L2
    // (other workgroups added to the counters with atomics)
    constexpr uint32_t kWords = sizeof(RoundCtl) / 8;
    const uint64_t* src = reinterpret_cast<const uint64_t*>(ctl);
    uint64_t* dst = reinterpret_cast<uint64_t*>(host_ctl);
    for (uint32_t i = threadIdx.x; i < kWords; i += NT)
        dst[i] = __hip_atomic_load(src + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __threadfence_system();
    if (lp.host_flag) {
        // every lane's words are out before the flag
        __syncthreads();
        if (threadIdx.x == 0)
            __hip_atomic_store(lp.host_flag, 1ull, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
    }
}

__global__ __launch_bounds__(256) void k_layout(Task* tasks, ModelJob* jobs, LayoutParams lp, RoundCtl* ctl,
                                                RoundCtl* host_ctl)
{
    layout_device(tasks, jobs, lp, ctl, host_ctl);
}

hipError_t launch_layout(Task* d_next, ModelJob* d_jobs, const LayoutParams& lp, RoundCtl* d_ctl, RoundCtl* host_ctl,
                         hipStream_t st)
{
    k_layout<<<1, 256, 0, st>>>(d_next, d_jobs, lp, d_ctl, host_ctl);
    return hipGetLastError();
}

__global__ __launch_bounds__(1024) void k_classify(const Task* tasks, const uint64_t* pos, const uint64_t* bstat,
                                                  uint32_t thresh, uint32_t param_fanout, Task* next,
                                                  GroupLists groups, Fill* fills, uint8_t* skip,
                                                  uint32_t* task_flags, RoundCtl* ctl, ModelJob* jobs,
                                                  LayoutParams lp, RoundCtl* host_ctl, const LiveCounts* live)
{
    uint32_t ntasks = gridDim.x;
    if (live) {
        ntasks = live->ntasks;
        if (blockIdx.x >= ntasks)
            return;
    }
    extern __shared__ __align__(16) unsigned char smem[];
    const Task T = tasks[blockIdx.x];
    const uint32_t f = T.fanout;
    uint64_t* bst = reinterpret_cast<uint64_t*>(smem);   // bucket start (task-relative), f + 1 entries
    int32_t* prv = reinterpret_cast<int32_t*>(bst + f + 1);
    int32_t* nxt = prv + f;                               // next group breaker (reversed index)
    uint32_t* cidx[kGroupClasses];
    cidx[0] = reinterpret_cast<uint32_t*>(nxt + f);
    cidx[1] = cidx[0] + f;
    cidx[2] = reinterpret_cast<uint32_t*>(prv);           // prv is dead once leaders are known
    uint32_t* tidx = cidx[1] + f;
    uint32_t* fidx = tidx + f;
    int32_t* ldr = reinterpret_cast<int32_t*>(fidx + f);   // group leader of each bucket
    uint8_t* kind = reinterpret_cast<uint8_t*>(ldr + f);
    __shared__ uint32_t ws_m[5][17];
    __shared__ int32_t ws_i[17];
    __shared__ uint32_t s_gb[kGroupClasses], s_tb, s_fb, s_noprog, s_nfb, s_over;
    __shared__ unsigned long long s_fkeys, s_gkeys;
    if (threadIdx.x == 0) {
        s_noprog = 0;
        s_nfb = 0;
        s_fkeys = 0;
        s_gkeys = 0;
        bst[f] = T.n;
    }
    const uint32_t fill_min = thresh / 8u > 2u ? thresh / 8u : 2u;
    const uint32_t gw = group_window(thresh);
    for (uint32_t b = threadIdx.x; b < f; b += blockDim.x) {
        const uint64_t s0 = pos[T.cnt_off + (uint64_t)b * T.nchunks] - T.cnt_base;
        const uint64_t s1 = (b + 1 < f) ? pos[T.cnt_off + (uint64_t)(b + 1) * T.nchunks] - T.cnt_base : T.n;
        const uint64_t sz = s1 - s0;
        const uint64_t lo = bstat[2 * ((uint64_t)T.bucket_off + b)];
        const uint64_t hi = bstat[2 * ((uint64_t)T.bucket_off + b) + 1];
        uint8_t k;
        if (sz == 0)
            k = kEmpty;
        else if (lo == hi && sz >= fill_min)
            k = kFillB;
        else if (lo != hi && sz >= 2ull * thresh)
            k = kBig;
        else if (lo != hi && sz > thresh)
            k = kSolo;
        else
            k = kSmall;
        bst[b] = s0;
        kind[b] = k;
        prv[b] = sz ? (int32_t)b : -1;
        skip[(uint64_t)T.bucket_off + b] = (k == kFillB);
    }
    __syncthreads();
    block_scan_op<int32_t>(prv, f, -1, MaxI32(), ws_i);      // prv[b]: last non-empty bucket before b
    unsigned long long my_fkeys = 0, my_gkeys = 0;
    uint32_t my_nfb = 0;
    for (uint32_t b = threadIdx.x; b < f; b += blockDim.x) {
        const uint8_t k = kind[b];
        bool lead = k == kSolo;
        if (k == kSmall) {
            const int32_t p = prv[b];
            lead = p < 0 || kind[p] != kSmall || bst[p] / gw != bst[b] / gw;
        }
        const bool brk = k != kEmpty && (lead || k != kSmall);
        nxt[f - 1 - b] = brk ? (int32_t)b : kNone;
        ldr[b] = brk ? (int32_t)b : -1;
        const uint64_t sz = bst[b + 1] - bst[b];
        tidx[b] = k == kBig ? 1u : 0u;
        fidx[b] = k == kFillB ? (uint32_t)((sz + kFillPiece - 1) / kFillPiece) : 0u;
        if (sz == T.n && (k == kBig || k == kFillB))
            s_noprog = 1;
        if (k == kFillB) {
            my_fkeys += sz;
            ++my_nfb;
        }
        if (k == kSmall || k == kSolo)
            my_gkeys += sz;
    }
    // one LDS atomic per wave
    my_fkeys = wave_sum(my_fkeys);
    my_gkeys = wave_sum(my_gkeys);
    my_nfb = wave_sum(my_nfb);
    if ((threadIdx.x & 63u) == 0) {
        if (my_fkeys)
            atomicAdd(&s_fkeys, my_fkeys);
        if (my_gkeys)
            atomicAdd(&s_gkeys, my_gkeys);
        if (my_nfb)
            atomicAdd(&s_nfb, my_nfb);
    }
    __syncthreads();
    // kind[] must only be rewritten once every thread is done reading it
    for (uint32_t b = threadIdx.x; b < f; b += blockDim.x) {
        const int32_t p = prv[b];
        const uint8_t k = kind[b];
        const bool lead = k == kSolo ||
                          (k == kSmall && (p < 0 || kind[p] != kSmall || bst[p] / gw != bst[b] / gw));
        prv[b] = lead ? 1 : 0;     // temporary: leader flag
    }
    __syncthreads();
    for (uint32_t b = threadIdx.x; b < f; b += blockDim.x)
        if (prv[b])
            kind[b] |= kLead;
    __syncthreads();
    block_scan_op<int32_t>(nxt, f, kNone, MinI32(), ws_i);   // nxt[f-1-b]: first breaker after b
    block_scan_op<int32_t>(ldr, f, -1, MaxI32(), ws_i);      // ldr[b]: last breaker before b
    for (uint32_t b = threadIdx.x; b < f; b += blockDim.x) {
        uint32_t c0 = 0, c1 = 0, c2 = 0;
        if (kind[b] & kLead) {
            const int32_t e = nxt[f - 1 - b];
            const uint64_t gsz = (e == kNone ? T.n : bst[e]) - bst[b];
            c0 = gsz <= kGroupClassCap[0];
            c1 = !c0 && gsz <= kGroupClassCap[1];
            c2 = !c0 && !c1;
        }
        cidx[0][b] = c0;
        cidx[1][b] = c1;
        cidx[2][b] = c2;
    }
    __syncthreads();
    uint32_t* const lists[5] = {cidx[0], cidx[1], cidx[2], tidx, fidx};
    uint32_t tot[5];
    block_scan_u32_multi<5>(lists, f, ws_m, tot);
    const uint32_t ng[kGroupClasses] = {tot[0], tot[1], tot[2]};
    const uint32_t nt = tot[3];
    const uint32_t nf = tot[4];
    if (threadIdx.x == 0) {
        for (uint32_t c = 0; c < kGroupClasses; ++c)
            s_gb[c] = ng[c] ? atomicAdd(&ctl->ngroups[c], ng[c]) : 0;
        s_tb = nt ? atomicAdd(&ctl->ntasks, nt) : 0;
        s_fb = nf ? atomicAdd(&ctl->nfill, nf) : 0;
        if (s_nfb) {
            atomicAdd(&ctl->nfillbuckets, s_nfb);
            atomicAdd((unsigned long long*)&ctl->fillkeys, s_fkeys);
        }
        if (s_gkeys)
            atomicAdd((unsigned long long*)&ctl->group_keys, s_gkeys);
        if (s_noprog)
            atomicAdd((unsigned long long*)&ctl->stall_keys, (unsigned long long)T.n);
        bool over = (uint64_t)s_tb + nt > lp.cap_tasks || (uint64_t)s_fb + nf > lp.cap_fills;
        for (uint32_t c = 0; c < kGroupClasses; ++c)
            over = over || (uint64_t)s_gb[c] + ng[c] > lp.cap_groups[c];
        if (over)
            atomicOr(&ctl->overflow, 1u);
        s_over = over;
        task_flags[blockIdx.x] = s_noprog ? kNoScatter : 0u;
    }
    __syncthreads();
    const bool noprog = s_noprog != 0;
    const bool over = s_over != 0;
    // where the keys of this round's buckets live after the scatter
    const uint64_t* moved = (noprog ? (T.src ? T.scratch : T.keys) : (T.src ? T.keys : T.scratch)) + T.start;
    for (uint32_t b = over ? f : threadIdx.x; b < f; b += blockDim.x) {
        const uint8_t kl = kind[b];
        const uint8_t k = kl & ~kLead;
        const uint64_t sz = bst[b + 1] - bst[b];
        if (kl & kLead) {
            const int32_t e = nxt[f - 1 - b];
            Group G;
            G.src = moved + bst[b];
            G.dst = T.keys + T.start + bst[b];
            G.start = T.start + bst[b];
            G.n = (uint32_t)((e == kNone ? T.n : bst[e]) - bst[b]);
            G.dtype = T.dtype;
            // the group's range: its first bucket's min and max here, the
            // group's other buckets fold theirs in below
            G.lo = bstat[2 * ((uint64_t)T.bucket_off + b)];
            G.hi = bstat[2 * ((uint64_t)T.bucket_off + b) + 1];
            const uint32_t c = G.n <= kGroupClassCap[0] ? 0u : (G.n <= kGroupClassCap[1] ? 1u : 2u);
            groups.g[c][s_gb[c] + cidx[c][b]] = G;
        } else if (k == kBig) {
            Task C = T;
            C.start = T.start + bst[b];
            C.n = sz;
            C.src = noprog ? T.src : 1u - T.src;
            C.level = T.level + 1;
            C.chunk0 = C.nchunks = C.bucket_off = 0;
            C.cnt_off = C.cnt_base = 0;
            const uint64_t lo = bstat[2 * ((uint64_t)T.bucket_off + b)];
            const uint64_t hi = bstat[2 * ((uint64_t)T.bucket_off + b) + 1];
            const bool stalled = noprog || (T.kind == kLocal && sz > T.n - T.n / 8u);
            const uint32_t fc0 = child_fanout(sz, thresh, param_fanout);
            const uint32_t fc = lp.inplace ? ip_fanout(sz, fc0) : fc0;
            if (T.kind == kGlobal) {
                // Alg. 2 level 1: the array's model again, f1 sub-buckets of bucket b
                C.kind = kGlobalL1;
                C.fanout = fc;
                C.scale = (double)f * (double)fc;
                C.offset = (int64_t)b * (int64_t)fc;
            } else if (T.kind == kLocal && stalled) {
                // no model progress: split on the highest differing bit
                const uint32_t d = 63u - (uint32_t)__clzll((long long)(lo ^ hi));
                const uint32_t lf = 31u - __clz(fc);
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
                C.fanout = fc;
                C.scale = (double)fc;
                C.offset = 0;
            }
            next[s_tb + tidx[b]] = C;
        }
    }
    // The other buckets of each group fold their min and max into the
    // group's range, after the groups written above have reached memory
    // (vmcnt counts this thread's stores; the barrier covers every thread's).
    if (!over) {
        __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);
        __syncthreads();
        for (uint32_t b = threadIdx.x; b < f; b += blockDim.x) {
            if (kind[b] != kSmall)      // leaders carry kLead; other kinds form no group
                continue;
            const int32_t L = ldr[b];
            if (L < 0)                  // a member always follows its leader
                continue;
            const int32_t e = nxt[f - 1 - L];
            const uint64_t gsz = (e == kNone ? T.n : bst[e]) - bst[L];
            const uint32_t c = gsz <= kGroupClassCap[0] ? 0u : (gsz <= kGroupClassCap[1] ? 1u : 2u);
            Group* G = &groups.g[c][s_gb[c] + cidx[c][L]];
            atomicMin(reinterpret_cast<unsigned long long*>(&G->lo),
                      (unsigned long long)bstat[2 * ((uint64_t)T.bucket_off + b)]);
            atomicMax(reinterpret_cast<unsigned long long*>(&G->hi),
                      (unsigned long long)bstat[2 * ((uint64_t)T.bucket_off + b) + 1]);
        }
    }
    // Fill pieces, spread over the workgroup (one all-equal bucket of a
    // skewed input can hold hundreds of pieces): piece q belongs to the last
    // bucket whose first piece fidx[b] is at most q.
    for (uint32_t q = over ? nf : threadIdx.x; q < nf; q += blockDim.x) {
        uint32_t lo = 0, hi = f;           // fidx[lo] <= q; the answer is below hi
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (fidx[mid] <= q)
                lo = mid;
            else
                hi = mid;
        }
        const uint32_t b = lo;
        const uint64_t sz = bst[b + 1] - bst[b];
        const uint64_t off = (uint64_t)(q - fidx[b]) * kFillPiece;
        Fill F;
        F.dst = T.keys + T.start + bst[b] + off;
        F.raw = from_ord(bstat[2 * ((uint64_t)T.bucket_off + b)], T.dtype);
        F.start = T.start + bst[b] + off;
        F.n = (uint32_t)min((uint64_t)kFillPiece, sz - off);
        F.dtype = T.dtype;
        fills[s_fb + q] = F;
    }
    // The last workgroup to finish lays out the next round.
    __shared__ uint32_t s_last;
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0)
        s_last = atomicAdd(&ctl->classified, 1u) == ntasks - 1;
    __syncthreads();
    if (s_last) {
        __threadfence();
        layout_device(next, jobs, lp, ctl, host_ctl);
    }
}

hipError_t launch_classify(const Task* d_tasks, uint32_t ntasks, const uint64_t* d_pos, const uint64_t* d_bstat,
                           uint32_t thresh, uint32_t param_fanout, Task* d_next, GroupLists groups, Fill* d_fills,
                           uint8_t* d_skip, uint32_t* d_task_flags, RoundCtl* d_ctl, uint32_t max_fanout,
                           ModelJob* d_jobs, const LayoutParams& lp, RoundCtl* host_ctl, const LiveCounts* live,
                           hipStream_t st)
{
    if (!ntasks)
        return hipSuccess;
    size_t smem = (size_t)(max_fanout + 1) * 8 + (size_t)max_fanout * (4 + 4 + 4 + 4 + 4 + 4 + 4 + 1) + 64;
    // a round with a few wide tasks (level 0) gets wide workgroups
    const uint32_t threads = (ntasks <= 64 && max_fanout >= 1024) ? 1024u : 256u;
    k_classify<<<ntasks, threads, smem, st>>>(d_tasks, d_pos, d_bstat, thresh, param_fanout, d_next, groups,
                                          d_fills, d_skip, d_task_flags, d_ctl, d_jobs, lp, host_ctl, live);
    return hipGetLastError();
}

// --------------------------------------------------------------- scatter --

constexpr uint32_t kScatterThreads = 1024;

// Scatter: stage one tile in LDS ordered by bucket, then write each bucket's
// run at its cursor so consecutive lanes write consecutive addresses.  Each
// key's bucket is computed again from the model (as in the histogram, with
// the same arithmetic, so the same bucket): nothing is stored between the
// two passes.  The next tile's keys are loaded while the current one is
// ranked and written.
//
// LDS: the staged tile (8 B keys), then per bucket the cursor and the tile's
// write base (8 B each; 4 B in the 12,288-key tile, whose rounds hold fewer
// than 2^31 keys, so task-relative positions fit), the tile count and tile
// start (4 B each), then the staged bucket numbers (2 B per key), then the
// model.  A cursor's top bit marks a bucket that is not moved.
template <typename CT = uint64_t>
struct ScatterLdsT {
    uint64_t* stage;
    CT* cur;
    CT* wbase;
    uint32_t* tcnt;
    uint32_t* tstart;
    uint16_t* sb;
    void* model;
    // spill-bucket rounds (k_scatter_ls1): per bucket {slot offset, first
    // position past its capacity, spill offset}, all relative to a key's
    // position in the task's count-ordered layout
    uint64_t* ls1;
};
using ScatterLds = ScatterLdsT<uint64_t>;

template <typename CT = uint64_t>
__device__ __forceinline__ ScatterLdsT<CT> scatter_lds(unsigned char* smem, uint32_t tile, uint32_t f)
{
    ScatterLdsT<CT> L;
    L.stage = reinterpret_cast<uint64_t*>(smem);
    L.cur = reinterpret_cast<CT*>(L.stage + tile);
    L.wbase = L.cur + f;
    L.tcnt = reinterpret_cast<uint32_t*>(L.wbase + f);
    L.tstart = L.tcnt + f;
    L.sb = reinterpret_cast<uint16_t*>(L.tstart + f);
    L.model = smem + (sizeof(CT) == 8 ? scatter_lds_bytes(tile, f) : scatter_lds_bytes32(tile, f));
    return L;
}

// One tile takes five barriers: after ranking; two inside the scan of the
// tile counts; after the scan (which also moves the cursors on and clears the
// counts, so the write loop needs only the write base); after staging.  The
// write loop needs none behind it: the next tile's ranking touches only the
// counts and the cursors' skip bits, and everything the write loop reads is
// rewritten only after the next tile's first barrier.
template <uint32_t KPT, uint32_t DT, bool MSD, bool LS1 = false, typename CT = uint64_t>
__device__ __forceinline__ void scatter_body(const Task& T, const SModel& M, gptr<const uint64_t> src,
                                             gptr<uint64_t> dst, uint32_t n, const ScatterLdsT<CT>& L,
                                             uint32_t* wsum, uint32_t flags, gptr<uint64_t> spill = {})
{
    constexpr uint32_t NT = kScatterThreads;
    constexpr uint32_t TILE = KPT * NT;
    const uint32_t f = T.fanout;
    const double scale = T.scale;
    const int32_t offset = (int32_t)T.offset;
    const uint32_t shift = T.shift;
    // buckets of this thread in the tile scan
    const uint32_t per = (f + NT - 1) / NT;
    const uint32_t blo = min(f, threadIdx.x * per), bhi = min(f, blo + per);
    const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
    uint64_t nxt[KPT];
#pragma unroll
    for (uint32_t u = 0; u < KPT; ++u) {
        const uint32_t i = u * NT + threadIdx.x;
        nxt[u] = i < n ? src[i] : 0;
    }
    for (uint32_t base = 0; base < n; base += TILE) {
        uint64_t raw[KPT];
        uint32_t bk[KPT];
        uint32_t rk[KPT];
#pragma unroll
        for (uint32_t u = 0; u < KPT; ++u)
            raw[u] = nxt[u];
        if (base + TILE < n) {
#pragma unroll
            for (uint32_t u = 0; u < KPT; ++u) {
                const uint32_t i = base + TILE + u * NT + threadIdx.x;
                nxt[u] = i < n ? src[i] : 0;
            }
        }
        // bucket of each key, and its rank among the tile's keys of that bucket
#pragma unroll
        for (uint32_t u = 0; u < KPT; ++u) {
            const uint32_t i = base + u * NT + threadIdx.x;
            bk[u] = ~0u;
            rk[u] = 0;
            if (i < n) {
                const uint32_t b = MSD ? msd_bucket<DT>(raw[u], shift, f)
                                       : model_bucket<DT>(M, raw[u], scale, offset, f, flags);
                if (!(L.cur[b] & (CT(1) << (sizeof(CT) * 8 - 1)))) {
                    bk[u] = b;
                    rk[u] = atomicAdd(&L.tcnt[b], 1u);
                }
            }
        }
        __syncthreads();
        // exclusive scan of the tile counts; write base = cursor - tile start
        uint32_t s = 0;
        for (uint32_t b = blo; b < bhi; ++b)
            s += L.tcnt[b];
        uint32_t x = s;
#pragma unroll
        for (uint32_t d = 1; d < 64; d <<= 1) {
            const uint32_t y = __shfl_up(x, d, 64);
            if (lane >= d)
                x += y;
        }
        if (lane == 63)
            wsum[wave] = x;
        __syncthreads();
        wave_totals_scan<uint32_t>(wsum, NT / 64, 0u, AddU32());
        __syncthreads();
        uint32_t run = wsum[wave] + x - s;
        for (uint32_t b = blo; b < bhi; ++b) {
            const uint32_t c = L.tcnt[b];
            L.tstart[b] = run;
            L.wbase[b] = L.cur[b] - run;   // modulo 2^64; a bucket with no key here is never read
            L.cur[b] += c;
            L.tcnt[b] = 0;
            run += c;
        }
        const uint32_t ntile = wsum[NT / 64];
        __syncthreads();
#pragma unroll
        for (uint32_t u = 0; u < KPT; ++u) {
            if (bk[u] != ~0u) {
                const uint32_t p = L.tstart[bk[u]] + rk[u];
                L.stage[p] = raw[u];
                L.sb[p] = (uint16_t)bk[u];
            }
        }
        __syncthreads();
        if (!LS1) {
            for (uint32_t p = threadIdx.x; p < ntile; p += NT)
                dst[L.wbase[L.sb[p]] + p] = L.stage[p];
        } else {
            // a key whose rank in its bucket is below the capacity takes its
            // slot in the bucket; the rest go to the spill area as order words
            for (uint32_t p = threadIdx.x; p < ntile; p += NT) {
                const uint32_t b = L.sb[p];
                const uint64_t g = L.wbase[b] + p;
                if (g < L.ls1[3 * b + 1])
                    dst[g + L.ls1[3 * b]] = L.stage[p];
                else
                    spill[g + L.ls1[3 * b + 2]] = to_ord(L.stage[p], DT);
            }
        }
    }
}

template <uint32_t KPT>
__global__ __launch_bounds__(kScatterThreads) void k_scatter(const Task* tasks, uint32_t ntasks, uint64_t chunk,
                                                             const double* models, const uint64_t* pos,
                                                             const uint8_t* skip, const uint32_t* task_flags,
                                                             uint32_t flags, const LiveCounts* live)
{
    if (live) {
        if (blockIdx.x >= live->chunks)
            return;
        ntasks = live->ntasks;
        chunk = live->chunk;
    }
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr uint32_t TILE = KPT * kScatterThreads;
    using CT = typename std::conditional<KPT == 12, uint32_t, uint64_t>::type;
    constexpr CT kSkip = CT(1) << (sizeof(CT) * 8 - 1);
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
    const ScatterLdsT<CT> L = scatter_lds<CT>(smem, TILE, f);
    const uint32_t lc = blockIdx.x - T.chunk0;
    for (uint32_t b = threadIdx.x; b < f; b += blockDim.x) {
        const CT c = (CT)(pos[T.cnt_off + (uint64_t)b * T.nchunks + lc] - T.cnt_base);
        L.cur[b] = skip[(uint64_t)T.bucket_off + b] ? (CT)(c | kSkip) : c;
        L.tcnt[b] = 0;
    }
    SModel M{};
    const bool msd = T.kind == kMsd;
    if (!msd)
        load_model(M, models, T.model, T.leaves, L.model);
    __syncthreads();
    const uint64_t lo = (uint64_t)lc * chunk;
    const uint32_t n = (uint32_t)(min(T.n, lo + chunk) - lo);
    const gptr<const uint64_t> src = as_global<const uint64_t>((T.src ? T.scratch : T.keys) + T.start + lo);
    const gptr<uint64_t> dst = as_global((T.src ? T.keys : T.scratch) + T.start);
    if (T.dtype == kF64) {
        if (msd) scatter_body<KPT, kF64, true, false, CT>(T, M, src, dst, n, L, wsum, flags);
        else scatter_body<KPT, kF64, false, false, CT>(T, M, src, dst, n, L, wsum, flags);
    } else {
        if (msd) scatter_body<KPT, kU64, true, false, CT>(T, M, src, dst, n, L, wsum, flags);
        else scatter_body<KPT, kU64, false, false, CT>(T, M, src, dst, n, L, wsum, flags);
    }
}

// Partition of LearnedSort 1.0 (Sec. 2, Fig. 1) for the spill-bucket
// ablation: one task, every bucket b holds at most `cap` keys in the slots
// [b cap, (b + 1) cap) of dst; the keys of a bucket past its capacity go to
// the spill area (order words), entry (b, chunk) of them at spoff[entry].
// Ranks inside a bucket follow the count-ordered layout of pos (chunk by
// chunk), so which keys spill is fixed by the scan; their order in the spill
// area does not matter (it is sorted).
template <uint32_t KPT>
__global__ __launch_bounds__(kScatterThreads) void k_scatter_ls1(const Task* tasks, uint64_t chunk,
                                                                 const double* models, const uint64_t* pos,
                                                                 const uint64_t* spoff, uint64_t cap,
                                                                 uint64_t* dst, uint64_t* spill, uint32_t flags)
{
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr uint32_t TILE = KPT * kScatterThreads;
    __shared__ uint32_t wsum[kScatterThreads / 64 + 1];
    const Task T = tasks[0];
    const uint32_t f = T.fanout;
    ScatterLds L = scatter_lds(smem, TILE, f);
    L.ls1 = reinterpret_cast<uint64_t*>(reinterpret_cast<unsigned char*>(L.model) +
                                        ls1_model_lds_bytes(T.leaves));
    const uint32_t lc = blockIdx.x;
    for (uint32_t b = threadIdx.x; b < f; b += blockDim.x) {
        const uint64_t e = (uint64_t)b * T.nchunks;
        const uint64_t start = pos[e], c = pos[e + lc];
        const uint64_t lim = start + cap;
        L.cur[b] = c;
        L.tcnt[b] = 0;
        L.ls1[3 * b] = (uint64_t)b * cap - start;                 // modulo 2^64
        L.ls1[3 * b + 1] = lim;
        L.ls1[3 * b + 2] = spoff[e + lc] - (c > lim ? c : lim);   // modulo 2^64
    }
    SModel M{};
    load_model(M, models, T.model, T.leaves, L.model);
    __syncthreads();
    const uint64_t lo = (uint64_t)lc * chunk;
    const uint32_t n = (uint32_t)(min(T.n, lo + chunk) - lo);
    const gptr<const uint64_t> src = as_global<const uint64_t>(T.keys + lo);
    if (T.dtype == kF64)
        scatter_body<KPT, kF64, false, true>(T, M, src, as_global(dst), n, L, wsum, flags, as_global(spill));
    else
        scatter_body<KPT, kU64, false, true>(T, M, src, as_global(dst), n, L, wsum, flags, as_global(spill));
}

hipError_t launch_scatter_ls1(const Task* d_task, uint32_t nchunks, uint64_t chunk, const double* d_models,
                              const uint64_t* d_pos, const uint64_t* d_spoff, uint64_t cap, uint64_t* d_dst,
                              uint64_t* d_spill, uint32_t fanout, uint32_t leaves, hipStream_t st)
{
    if (!nchunks)
        return hipSuccess;
    const size_t smem = ls1_scatter_lds_bytes(fanout, leaves);
    k_scatter_ls1<kLs1Tile / kScatterThreads><<<nchunks, kScatterThreads, smem, st>>>(
        d_task, chunk, d_models, d_pos, d_spoff, cap, d_dst, d_spill, 0u);
    return hipGetLastError();
}

// Round 0 of device-described segments, in one workgroup: segments are taken
// 1024 at a time; each lane classifies its segment (nothing, a base-case
// group, or a task with a global model), and block scans of the nine list
// counters give every item its place, in segment order (the same lists the
// host builds for host-described arrays).
constexpr uint32_t kSegQ = 9;   // groups x3, tasks, samples, blocks, leafs, models, group keys

__global__ __launch_bounds__(1024) void k_seg_prepare(SegPrepare A)
{
    __shared__ uint64_t wsum[kSegQ][1024 / 64];
    __shared__ uint64_t carry[kSegQ];
    __shared__ uint64_t s_maxm;
    __shared__ uint32_t s_err;
    const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
    if (threadIdx.x < kSegQ)
        carry[threadIdx.x] = 0;
    if (threadIdx.x == 0) {
        s_maxm = 0;
        s_err = A.nseg && A.off[0] != 0 ? 1u : 0u;
    }
    __syncthreads();
    uint64_t my_maxm = 0;
    uint32_t my_err = 0;
    for (uint64_t base = 0; base < A.nseg; base += 1024) {
        const uint64_t i = base + threadIdx.x;
        const bool valid = i < A.nseg;
        uint64_t lo = 0, n = 0;
        uint32_t dt = A.dtype;
        if (valid) {
            lo = A.off[i];
            const uint64_t hi = A.off[i + 1];
            if (hi < lo)
                my_err = 1;
            else
                n = hi - lo;
            if (A.dtypes)
                dt = A.dtypes[i];
        }
        const bool small = n > 1 && n <= 2ull * A.base;
        const bool task = n > 2ull * A.base;
        const uint32_t cls = small ? group_class((uint32_t)n) : 0u;
        const uint64_t m = task ? sample_size(n, A.rate, A.cap) : 0;
        const bool sampled = task && m > kSampleBlock;
        uint64_t q[kSegQ] = {small && cls == 0 ? 1u : 0u,
                             small && cls == 1 ? 1u : 0u,
                             small && cls == 2 ? 1u : 0u,
                             task ? 1u : 0u,
                             sampled ? m : 0u,
                             sampled ? (m + kSampleBlock - 1) / kSampleBlock : 0u,
                             sampled ? A.leaves : 0u,
                             task ? model_doubles(A.leaves) : 0u,
                             small ? n : 0u};
        uint64_t x[kSegQ];
#pragma unroll
        for (uint32_t j = 0; j < kSegQ; ++j) {
            x[j] = q[j];
#pragma unroll
            for (uint32_t d = 1; d < 64; d <<= 1) {
                const uint64_t y = __shfl_up(x[j], d, 64);
                if (lane >= d)
                    x[j] += y;
            }
            if (lane == 63)
                wsum[j][wave] = x[j];
        }
        __syncthreads();
        if (threadIdx.x < kSegQ) {
            uint64_t run = carry[threadIdx.x];
            for (uint32_t w = 0; w < 1024 / 64; ++w) {
                const uint64_t t = wsum[threadIdx.x][w];
                wsum[threadIdx.x][w] = run;
                run += t;
            }
            carry[threadIdx.x] = run;
        }
        __syncthreads();
        uint64_t off[kSegQ];
#pragma unroll
        for (uint32_t j = 0; j < kSegQ; ++j)
            off[j] = wsum[j][wave] + x[j] - q[j];
        uint64_t* keys = A.keys + lo;
        if (small) {
            Group g;
            g.src = keys;
            g.dst = keys;
            g.start = 0;
            g.n = (uint32_t)n;
            g.dtype = dt;
            g.lo = ~0ull;   // range not known: the base case finds it
            g.hi = 0;
            A.groups[cls][off[cls]] = g;
        }
        if (task) {
            Task t{};
            t.keys = keys;
            t.scratch = A.inplace ? keys : A.scratch + lo;
            t.n = n;
            t.dtype = dt;
            t.seg = (uint32_t)i;
            t.kind = kGlobal;
            t.fanout = child_fanout(n, A.base, A.fanout);
            if (A.inplace)
                t.fanout = ip_fanout(n, t.fanout);
            t.scale = (double)t.fanout;
            t.leaves = A.leaves;
            t.model = off[7];
            A.tasks[off[3]] = t;
            ModelJob J;
            J.src = keys;
            J.n = n;
            J.m = m;
            J.seed = A.seed;
            J.sample_off = off[4];
            J.model_off = off[7];
            J.leaf_off = off[6];
            J.leaves = A.leaves;
            J.dtype = dt;
            J.block0 = (uint32_t)off[5];
            J.nblocks = sampled ? (uint32_t)((m + kSampleBlock - 1) / kSampleBlock) : 0u;
            A.jobs[off[3]] = J;
            my_maxm = max(my_maxm, (unsigned long long)m);
        }
        __syncthreads();
    }
    my_maxm = wave_max(my_maxm);
    if (lane == 0)
        atomicMax((unsigned long long*)&s_maxm, (unsigned long long)my_maxm);
    if (my_err)
        atomicOr(&s_err, 1u);
    __syncthreads();
    if (threadIdx.x == 0) {
        RoundCtl c{};
        c.ntasks = (uint32_t)carry[3];
        for (uint32_t k = 0; k < kGroupClasses; ++k)
            c.ngroups[k] = (uint32_t)carry[k];
        c.cur.njobs = (uint32_t)carry[3];
        c.cur.blocks = (uint32_t)carry[5];
        c.cur.samples = carry[4];
        c.cur.max_sample = s_maxm;
        *A.ctl = c;
        A.summary[0] = carry[8];
        A.summary[1] = carry[6];
        A.summary[2] = carry[7];
        A.summary[3] = s_err;
    }
}

hipError_t launch_seg_prepare(const SegPrepare& A, hipStream_t st)
{
    k_seg_prepare<<<1, 1024, 0, st>>>(A);
    return hipGetLastError();
}

hipError_t launch_scatter(const Task* d_tasks, uint32_t ntasks, uint32_t total_chunks, uint64_t chunk,
                          const double* d_models, const uint64_t* d_pos, const uint8_t* d_skip,
                          const uint32_t* d_task_flags, uint32_t tile, uint32_t max_fanout, uint32_t max_leaves,
                          uint32_t flags, const LiveCounts* live, hipStream_t st)
{
    if (!total_chunks)
        return hipSuccess;
    const size_t smem = scatter_lds_bytes(tile, max_fanout) + model_lds_bytes(max_leaves);
    switch (tile) {
    case 1024:
        k_scatter<1><<<total_chunks, kScatterThreads, smem, st>>>(d_tasks, ntasks, chunk, d_models, d_pos, d_skip,
                                                                  d_task_flags, flags, live);
        break;
    case 2048:
        k_scatter<2><<<total_chunks, kScatterThreads, smem, st>>>(d_tasks, ntasks, chunk, d_models, d_pos, d_skip,
                                                                  d_task_flags, flags, live);
        break;
    case 4096:
        k_scatter<4><<<total_chunks, kScatterThreads, smem, st>>>(d_tasks, ntasks, chunk, d_models, d_pos, d_skip,
                                                                  d_task_flags, flags, live);
        break;
    case kTile12:
        k_scatter<12><<<total_chunks, kScatterThreads,
                        scatter_lds_bytes32(tile, max_fanout) + model_lds_bytes(max_leaves), st>>>(
            d_tasks, ntasks, chunk, d_models, d_pos, d_skip, d_task_flags, flags, live);
        break;
    case 8192:
        k_scatter<8><<<total_chunks, kScatterThreads, smem, st>>>(d_tasks, ntasks, chunk, d_models, d_pos, d_skip,
                                                                  d_task_flags, flags, live);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace lsort
