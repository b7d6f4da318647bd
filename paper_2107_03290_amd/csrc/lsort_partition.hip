// Partition rounds: histogram, scan, classify, scatter (Alg. 1 / Alg. 2).
#include "lsort_device.h"

#pragma clang fp contract(off)

namespace lsort {

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
// (Alg. 1 S_B, and the all-equal test of Alg. 2).  A workgroup of 1024 lanes
// streams its chunk; the next 4096 keys are loaded while the current ones are
// classified, so loads stay in flight through the LDS work.
constexpr uint32_t kHistThreads = 1024;
constexpr uint32_t kHistUnroll = 4;

template <uint32_t DT, bool MSD>
__device__ __forceinline__ void hist_body(const Task& T, const SModel& M, const uint64_t* src, uint32_t cnt,
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
            if (i < cnt) {
                const uint32_t b = MSD ? msd_bucket<DT>(raw[u], shift, fanout)
                                       : model_bucket<DT>(M, raw[u], scale, offset, fanout, flags);
                atomicAdd(&h[b], 1u);
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
    const uint64_t* src = (T.src ? T.scratch : T.keys) + T.start + lo;
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
                       const double* d_models, uint32_t* d_cnt, uint64_t* d_bstat, uint32_t max_fanout,
                       uint32_t max_leaves, uint32_t flags, hipStream_t st)
{
    size_t smem = (((size_t)max_fanout * 20 + 15) & ~(size_t)15) + model_lds_bytes(max_leaves);
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
// never moved again), small (sorted in LDS together with its neighbours) or
// over-full (a task of the next round).  Small buckets hold at most `thresh`
// keys; consecutive small buckets whose starts fall into the same window of
// `thresh` keys form one group, so a group holds fewer than 2*thresh keys.
// Everything is decided with block-wide scans, no serial walk.
enum : uint8_t { kEmpty = 0, kSmall = 1, kFillB = 2, kBig = 3 };

constexpr int32_t kNone = 0x7fffffff;

__global__ __launch_bounds__(256) void k_classify(const Task* tasks, const uint64_t* pos, const uint64_t* bstat,
                                                  uint32_t thresh, uint32_t param_fanout, Task* next,
                                                  Group* groups, Fill* fills, uint8_t* skip,
                                                  uint32_t* task_flags, RoundCtl* ctl)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const Task T = tasks[blockIdx.x];
    const uint32_t f = T.fanout;
    uint64_t* bst = reinterpret_cast<uint64_t*>(smem);   // bucket start (task-relative)
    uint64_t* bsz = bst + f;                              // bucket size
    int32_t* prv = reinterpret_cast<int32_t*>(bsz + f);   // previous non-empty bucket
    int32_t* nxt = prv + f;                               // next group breaker (reversed index)
    uint32_t* gidx = reinterpret_cast<uint32_t*>(nxt + f);
    uint32_t* tidx = gidx + f;
    uint32_t* fidx = tidx + f;
    uint8_t* kind = reinterpret_cast<uint8_t*>(fidx + f);
    __shared__ uint32_t ws_u[5];
    __shared__ int32_t ws_i[5];
    __shared__ uint32_t s_gb, s_tb, s_fb, s_noprog, s_nfb;
    __shared__ unsigned long long s_fkeys, s_gkeys;
    if (threadIdx.x == 0) {
        s_noprog = 0;
        s_nfb = 0;
        s_fkeys = 0;
        s_gkeys = 0;
    }
    const uint32_t fill_min = thresh / 8u > 2u ? thresh / 8u : 2u;
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
        else if (lo != hi && sz > thresh)
            k = kBig;
        else
            k = kSmall;
        bst[b] = s0;
        bsz[b] = sz;
        kind[b] = k;
        prv[b] = sz ? (int32_t)b : -1;
        skip[(uint64_t)T.bucket_off + b] = (k == kFillB);
    }
    __syncthreads();
    block_scan_op<int32_t>(prv, f, -1, MaxI32(), ws_i);      // prv[b]: last non-empty bucket before b
    for (uint32_t b = threadIdx.x; b < f; b += blockDim.x) {
        const uint8_t k = kind[b];
        bool lead = false;
        if (k == kSmall) {
            const int32_t p = prv[b];
            lead = p < 0 || kind[p] != kSmall || bst[p] / thresh != bst[b] / thresh;
        }
        const bool brk = k != kEmpty && (lead || k != kSmall);
        gidx[b] = lead ? 1u : 0u;
        tidx[b] = k == kBig ? 1u : 0u;
        fidx[b] = k == kFillB ? (uint32_t)((bsz[b] + kFillPiece - 1) / kFillPiece) : 0u;
        nxt[f - 1 - b] = brk ? (int32_t)b : kNone;
        if (bsz[b] == T.n && (k == kBig || k == kFillB))
            s_noprog = 1;
        if (k == kFillB) {
            atomicAdd(&s_fkeys, (unsigned long long)bsz[b]);
            atomicAdd(&s_nfb, 1u);
        }
        if (k == kSmall)
            atomicAdd(&s_gkeys, (unsigned long long)bsz[b]);
    }
    __syncthreads();
    block_scan_op<int32_t>(nxt, f, kNone, MinI32(), ws_i);   // nxt[f-1-b]: first breaker after b
    const uint32_t ng = block_scan_u32(gidx, f, ws_u);
    const uint32_t nt = block_scan_u32(tidx, f, ws_u);
    const uint32_t nf = block_scan_u32(fidx, f, ws_u);
    if (threadIdx.x == 0) {
        s_gb = ng ? atomicAdd(&ctl->ngroups, ng) : 0;
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
        task_flags[blockIdx.x] = s_noprog ? kNoScatter : 0u;
    }
    __syncthreads();
    const bool noprog = s_noprog != 0;
    // where the keys of this round's buckets live after the scatter
    const uint64_t* moved = (noprog ? (T.src ? T.scratch : T.keys) : (T.src ? T.keys : T.scratch)) + T.start;
    const uint32_t lf = 31u - __clz(param_fanout);
    for (uint32_t b = threadIdx.x; b < f; b += blockDim.x) {
        const uint8_t k = kind[b];
        if (k == kSmall) {
            const int32_t p = prv[b];
            const bool lead = p < 0 || kind[p] != kSmall || bst[p] / thresh != bst[b] / thresh;
            if (!lead)
                continue;
            const int32_t e = nxt[f - 1 - b];
            const uint64_t end = e == kNone ? T.n : bst[e];
            Group G;
            G.src = moved + bst[b];
            G.dst = T.keys + T.start + bst[b];
            G.start = T.start + bst[b];
            G.n = (uint32_t)(end - bst[b]);
            G.dtype = T.dtype;
            groups[s_gb + gidx[b]] = G;
        } else if (k == kFillB) {
            const uint64_t raw = from_ord(bstat[2 * ((uint64_t)T.bucket_off + b)], T.dtype);
            const uint64_t sz = bsz[b];
            const uint32_t np = (uint32_t)((sz + kFillPiece - 1) / kFillPiece);
            for (uint32_t q = 0; q < np; ++q) {
                Fill F;
                const uint64_t off = (uint64_t)q * kFillPiece;
                F.dst = T.keys + T.start + bst[b] + off;
                F.raw = raw;
                F.start = T.start + bst[b] + off;
                F.n = (uint32_t)min((uint64_t)kFillPiece, sz - off);
                F.dtype = T.dtype;
                fills[s_fb + fidx[b] + q] = F;
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
                C.kind = kGlobalL1;             // Alg. 2: level 1 reuses the array's model
                C.scale = (double)f * (double)f;
                C.offset = (int64_t)b * (int64_t)f;
            } else if (T.kind == kLocal && stalled) {
                // no model progress: split on the highest differing bit
                const uint32_t d = 63u - (uint32_t)__clzll((long long)(lo ^ hi));
                uint32_t bits = lf < d + 1 ? lf : d + 1;
                bits = bits ? bits : 1;
                C.kind = kMsd;
                C.fanout = 1u << bits;
                C.shift = d + 1 - bits;
                C.scale = 0.0;
                C.offset = 0;
                atomicAdd(&ctl->fallbacks, 1u);
            } else {
                C.kind = kLocal;                // model trained on the range before the next round
                C.fanout = param_fanout;
                C.scale = (double)param_fanout;
                C.offset = 0;
            }
            next[s_tb + tidx[b]] = C;
        }
    }
}

hipError_t launch_classify(const Task* d_tasks, uint32_t ntasks, const uint64_t* d_pos, const uint64_t* d_bstat,
                           uint32_t thresh, uint32_t param_fanout, Task* d_next, Group* d_groups, Fill* d_fills,
                           uint8_t* d_skip, uint32_t* d_task_flags, RoundCtl* d_ctl, uint32_t max_fanout,
                           hipStream_t st)
{
    size_t smem = (size_t)max_fanout * (8 + 8 + 4 + 4 + 4 + 4 + 4 + 1) + 16;
    k_classify<<<ntasks, 256, smem, st>>>(d_tasks, d_pos, d_bstat, thresh, param_fanout, d_next, d_groups,
                                          d_fills, d_skip, d_task_flags, d_ctl);
    return hipGetLastError();
}

constexpr uint32_t kScatterThreads = 1024;

// Scatter: stage one tile in LDS ordered by bucket, then write each bucket's
// run at its cursor so consecutive lanes write consecutive addresses.  The
// next tile's keys are loaded while the current one is ranked and written.
template <uint32_t KPT, uint32_t DT, bool MSD>
__device__ __forceinline__ void scatter_body(const Task& T, const SModel& M, const uint64_t* src, uint64_t* dst,
                                             uint32_t n, unsigned char* smem, uint32_t* wsum, uint32_t flags)
{
    constexpr uint32_t TILE = KPT * kScatterThreads;
    const uint32_t f = T.fanout;
    uint64_t* stage = reinterpret_cast<uint64_t*>(smem);
    uint64_t* cur = stage + TILE;
    uint32_t* tcnt = reinterpret_cast<uint32_t*>(cur + f);
    uint32_t* tstart = tcnt + f;
    uint16_t* sb = reinterpret_cast<uint16_t*>(tstart + f);
    const double scale = T.scale;
    const int32_t offset = (int32_t)T.offset;
    const uint32_t shift = T.shift;
    uint64_t nxt[KPT];
#pragma unroll
    for (uint32_t u = 0; u < KPT; ++u) {
        const uint32_t i = u * kScatterThreads + threadIdx.x;
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
                const uint32_t i = base + TILE + u * kScatterThreads + threadIdx.x;
                nxt[u] = i < n ? src[i] : 0;
            }
        }
#pragma unroll
        for (uint32_t u = 0; u < KPT; ++u) {
            const uint32_t i = base + u * kScatterThreads + threadIdx.x;
            bk[u] = ~0u;
            rk[u] = 0;
            if (i < n) {
                const uint32_t b = MSD ? msd_bucket<DT>(raw[u], shift, f)
                                       : model_bucket<DT>(M, raw[u], scale, offset, f, flags);
                if (!(cur[b] & kSkipBit)) {
                    bk[u] = b;
                    rk[u] = atomicAdd(&tcnt[b], 1u);
                }
            }
        }
        __syncthreads();
        for (uint32_t b = threadIdx.x; b < f; b += kScatterThreads)
            tstart[b] = tcnt[b];
        __syncthreads();
        const uint32_t ntile = block_scan_u32(tstart, f, wsum);
#pragma unroll
        for (uint32_t u = 0; u < KPT; ++u) {
            if (bk[u] != ~0u) {
                const uint32_t p = tstart[bk[u]] + rk[u];
                stage[p] = raw[u];
                sb[p] = (uint16_t)bk[u];
            }
        }
        __syncthreads();
        for (uint32_t p = threadIdx.x; p < ntile; p += kScatterThreads) {
            const uint32_t b = sb[p];
            dst[cur[b] + (p - tstart[b])] = stage[p];
        }
        __syncthreads();
        for (uint32_t b = threadIdx.x; b < f; b += kScatterThreads) {
            cur[b] += tcnt[b];
            tcnt[b] = 0;
        }
        __syncthreads();
    }
}

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
    uint64_t* cur = reinterpret_cast<uint64_t*>(smem) + TILE;
    uint32_t* tcnt = reinterpret_cast<uint32_t*>(cur + f);
    void* mlds = smem + (((size_t)TILE * 10 + (size_t)f * 16 + 15) & ~(size_t)15);
    const uint32_t lc = blockIdx.x - T.chunk0;
    for (uint32_t b = threadIdx.x; b < f; b += blockDim.x) {
        const uint64_t c = pos[T.cnt_off + (uint64_t)b * T.nchunks + lc] - T.cnt_base;
        cur[b] = skip[(uint64_t)T.bucket_off + b] ? (c | kSkipBit) : c;
        tcnt[b] = 0;
    }
    SModel M{};
    const bool msd = T.kind == kMsd;
    if (!msd)
        load_model(M, models, T.model, T.leaves, mlds);
    __syncthreads();
    const uint64_t lo = (uint64_t)lc * chunk;
    const uint32_t n = (uint32_t)(min(T.n, lo + chunk) - lo);
    const uint64_t* src = (T.src ? T.scratch : T.keys) + T.start + lo;
    uint64_t* dst = (T.src ? T.keys : T.scratch) + T.start;
    if (T.dtype == kF64) {
        if (msd) scatter_body<KPT, kF64, true>(T, M, src, dst, n, smem, wsum, flags);
        else scatter_body<KPT, kF64, false>(T, M, src, dst, n, smem, wsum, flags);
    } else {
        if (msd) scatter_body<KPT, kU64, true>(T, M, src, dst, n, smem, wsum, flags);
        else scatter_body<KPT, kU64, false>(T, M, src, dst, n, smem, wsum, flags);
    }
}

hipError_t launch_scatter(const Task* d_tasks, uint32_t ntasks, uint32_t total_chunks, uint64_t chunk,
                          const double* d_models, const uint64_t* d_pos, const uint8_t* d_skip,
                          const uint32_t* d_task_flags, uint32_t tile, uint32_t max_fanout, uint32_t max_leaves,
                          uint32_t flags, hipStream_t st)
{
    size_t smem = (((size_t)tile * 10 + (size_t)max_fanout * 16 + 15) & ~(size_t)15) + model_lds_bytes(max_leaves);
    switch (tile) {
    case 1024:
        k_scatter<1><<<total_chunks, kScatterThreads, smem, st>>>(d_tasks, ntasks, chunk, d_models, d_pos, d_skip,
                                                                  d_task_flags, flags);
        break;
    case 2048:
        k_scatter<2><<<total_chunks, kScatterThreads, smem, st>>>(d_tasks, ntasks, chunk, d_models, d_pos, d_skip,
                                                                  d_task_flags, flags);
        break;
    case 4096:
        k_scatter<4><<<total_chunks, kScatterThreads, smem, st>>>(d_tasks, ntasks, chunk, d_models, d_pos, d_skip,
                                                                  d_task_flags, flags);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace lsort
