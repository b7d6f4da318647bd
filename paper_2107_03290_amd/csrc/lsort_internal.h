// Internal structures shared by the HIP kernels and the host pipeline.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lsort {

constexpr uint32_t kF64 = 1;
constexpr uint32_t kU64 = 2;

constexpr uint32_t kMaxFanout = 4096;
constexpr uint32_t kMaxLeaves = 1024;
constexpr uint32_t kMaxBase = 8192;        // largest group the LDS base case sorts
constexpr uint32_t kNoPrev = 0xffffu;      // "no knot below": F = 0
constexpr uint64_t kFillPiece = 1u << 16;  // keys per fill work item
constexpr uint32_t kTargetChunks = 2048;   // chunks per partition round (8 per CU)
constexpr uint32_t kSmallRoundChunks = 256; // chunks of a small round (one per CU)
constexpr uint32_t kLocalMinSample = 1024; // smallest sample of a local model
constexpr uint32_t kSampleBlock = 4096;    // sample keys per training block (one LDS-sorted run)
constexpr uint32_t kGroupClasses = 3;      // base-case size classes: <= 1024, 4096, 8192 keys
constexpr uint32_t kGroupClassCap[kGroupClasses] = {1024, 4096, 8192};
// Static device array of the no-allocation sort, per device.
constexpr size_t kNoAllocBytes = (size_t)128 << 20;

// How a task maps a key to a bucket.
enum TaskKind : uint32_t {
    kGlobal = 0,     // level 0: floor(F * f), F the array's model
    kGlobalL1 = 1,   // level 1 under parent i: floor(F * f * f1) - i*f1 (same model)
    kLocal = 2,      // deeper: floor(F_local * f), model trained on the range
    kMsd = 3,        // no model progress: digit of the order-preserving word
};

// A key range that still has to be partitioned.
struct Task {
    uint64_t* keys;       // the array's final buffer (caller's)
    uint64_t* scratch;    // the array's scratch buffer (same length)
    uint64_t start;       // first key of the range, relative to the array
    uint64_t n;           // keys in the range
    uint64_t model;       // offset (in doubles) of the model in the model pool
    double scale;         // kGlobal / kLocal: f; kGlobalL1: f * f1
    int64_t offset;       // kGlobalL1: i * f1
    uint32_t fanout;
    uint32_t kind;        // TaskKind
    uint32_t dtype;       // kF64 / kU64
    uint32_t src;         // 0: keys live in `keys`, 1: in `scratch`
    uint32_t leaves;      // leaves of the model
    uint32_t shift;       // kMsd: bucket = (ord >> shift) & (fanout - 1)
    uint32_t level;
    uint32_t chunk0;      // first chunk of this task in the round
    uint32_t nchunks;
    uint64_t bucket_off;  // first bucket of this task in the round's bucket table
    uint64_t cnt_off;     // first entry of this task in the round's count matrix
    uint64_t cnt_base;    // sum of the sizes of the round's earlier tasks
    uint32_t seg;
    uint32_t pad;
    uint64_t side_off;    // in-place rounds: first key of this task's part of the side buffer
};

// A run of adjacent small buckets sorted by one workgroup in LDS.
struct Group {
    const uint64_t* src;
    uint64_t* dst;
    uint64_t start;       // of dst, relative to its array (0: no seam to check)
    uint32_t n;
    uint32_t dtype;
    // smallest and largest order word of the group's keys when known (the
    // partition's per-bucket min and max); lo > hi: not known
    uint64_t lo;
    uint64_t hi;
};

// The three size-class lists of groups (device pointers, passed by value).
struct GroupLists {
    Group* g[kGroupClasses];
};

// Part of an all-equal bucket: written with its single value, never sorted.
struct Fill {
    uint64_t* dst;
    uint64_t raw;
    uint64_t start;       // relative to the array
    uint32_t n;
    uint32_t dtype;
};

// One model to train: sample m keys of src[0..n) and fit L leaves.
struct ModelJob {
    const uint64_t* src;
    uint64_t n;
    uint64_t m;
    uint64_t seed;
    uint64_t sample_off;  // into the sample buffer
    uint64_t model_off;   // into the model pool (doubles)
    uint64_t leaf_off;    // into the leaf-statistics tables
    uint32_t leaves;
    uint32_t dtype;
    uint32_t block0;      // first sampling block of this job
    uint32_t nblocks;
};

// Parameters the device-side round layout needs.
struct LayoutParams {
    uint32_t fanout;      // the caller's fanout
    uint32_t leaves;
    uint32_t tile;        // keys per scatter tile
    uint32_t tile_wide;   // tile of rounds of at least wide_keys keys (0: always `tile`)
    uint64_t wide_keys;
    uint32_t wide_max_fanout;   // largest task fanout whose wide-tile scatter fits in LDS
    uint32_t target_chunks;     // chunks a large round is cut into (kTargetChunks; in-place rounds fewer)
    uint32_t inplace;           // in-place rounds (LS_FLAG_INPLACE)
    uint32_t pad;
    double rate;
    uint64_t cap;
    uint64_t seed;
    uint64_t model_base;  // local models start after the arrays' global models
    // Capacities (entries) of the buffers a round writes: the lists classify
    // appends to, and the next round's tables.  A round that would exceed
    // one raises RoundCtl::overflow and ends the sort; the host sizes the
    // buffers from bounds, so this only guards memory.
    uint64_t cap_tasks, cap_fills, cap_groups[kGroupClasses];
    uint64_t cap_keys, cap_chunks, cap_buckets, cap_entries, cap_samples, cap_blocks, cap_leafs, cap_models;
    // Mapped host word set to 1 once the control block is published (null:
    // none).  The host then reads the next round's sizes and queues its
    // launches while the rest of the round (the scatter) still runs.
    uint64_t* host_flag;
};

// In-place partition (LS_FLAG_INPLACE): keys per block and the largest
// fanout (the LDS holds one open fragment of a block per bucket).
constexpr uint32_t kIpBlock = 64;
constexpr uint32_t kIpFanout = 128;
// Fewest leaves of a local model in an in-place round (which otherwise gets
// 8 leaves per bucket).
constexpr uint32_t kIpMinLeaves = 16;

// Chunks of an in-place round hold at least kIpChunkBlocks x fanout blocks,
// and a task of n keys has a fanout of at most n / (kIpChunkBlocks kIpBlock):
// the open fragments a chunk leaves (fewer than fanout x kIpBlock keys) and
// the overflow blocks (at most one per bucket) each stay under 1/64 of the
// keys.
constexpr uint64_t kIpChunkBlocks = 64;

// Fanout of a task of n keys in an in-place round: at most the out-of-place
// choice fc, and at most n / (kIpChunkBlocks kIpBlock) (at least 2).  A power
// of two when fc is one.
__host__ __device__ inline uint32_t ip_fanout(uint64_t n, uint32_t fc)
{
    const uint64_t lim = n / (kIpChunkBlocks * kIpBlock);
    uint32_t f = 2;
    while ((uint64_t)f * 2 <= lim && f * 2 <= fc)
        f *= 2;
    return f < fc ? f : fc;
}

// Keys of the side buffer one chunk of an in-place task may fill.
__host__ __device__ inline uint64_t ip_side_keys(uint64_t chunk, uint32_t fanout)
{
    const uint64_t most = (uint64_t)fanout * (kIpBlock - 1);
    return chunk < most ? chunk : most;
}

// A bucket of an in-place round: its range [start, end) in the task's final
// layout; its full blocks go to the slots [a, dend) (one more that does not
// fit goes to an overflow block).
struct IpBucket {
    uint64_t start, end;
    uint32_t a, area, dend, full, task, pad;
};

// Destination of a block slot in the permutation: a slot of the task, or
// kIpOvf | b for bucket b's block that does not fit, or kIpNoDest for a slot
// that holds no full block.
constexpr uint32_t kIpOvf = 0x80000000u;
constexpr uint32_t kIpNoDest = 0xffffffffu;

// Sizes of the running round, copied from the control block when the round
// starts.  In graph mode the kernels are launched with upper-bound grids and
// read their real sizes here (blocks beyond them exit at once).
struct LiveCounts {
    uint64_t chunk, nkeys, entries, samples, max_sample, buckets;
    uint32_t ntasks, chunks, njobs, blocks, max_fanout, max_leaves;
};

// Counters the classify and layout kernels fill in; read by the host after
// each round (one small copy) to size the next round's launches.
struct RoundCtl {
    // written by classify (cumulative over rounds unless noted)
    uint32_t ntasks;                  // next-round tasks (reset every round)
    uint32_t nfill;                   // fill items
    uint32_t ngroups[kGroupClasses];  // base-case groups per size class
    uint32_t nfillbuckets;
    uint64_t fillkeys;
    uint64_t group_keys;              // keys in base-case groups
    uint64_t stall_keys;              // keys of tasks that made no progress (not scattered)
    uint32_t fallbacks;
    uint32_t violations;              // out-of-order seams found by the touch-up
    uint32_t overflow;                // a list or table would have exceeded its buffer
    // written by the layout kernel for the next round
    uint64_t chunk;                   // keys per chunk
    uint64_t nkeys;                   // keys in the round's tasks
    uint64_t entries;                 // count-matrix entries
    uint64_t samples, leafs, models;  // training-table sizes
    uint64_t max_sample;              // largest sample of one job
    uint64_t buckets;
    uint32_t chunks, njobs, blocks;
    uint32_t max_fanout, max_leaves, max_level;
    uint32_t classified;              // classify workgroups finished (reset every round)
    // written by the layout kernel, cumulative over the sort
    uint32_t rounds;                  // rounds laid out with at least one task
    uint32_t deepest;                 // largest task level laid out
    uint32_t tile;                    // scatter tile of the next round (written by the layout)
    uint32_t pad;
    uint64_t tasks_total;             // tasks over all rounds
    uint64_t side_keys;               // in-place rounds: side-buffer keys of the next round
    LiveCounts cur;                   // graph mode: the running round's sizes
};

static_assert(sizeof(RoundCtl) % 8 == 0 && sizeof(Task) % 8 == 0 && sizeof(ModelJob) % 8 == 0 &&
                  sizeof(Group) % 8 == 0,
              "the control block is published, and the round-0 lists uploaded, as 8-byte words");

// Device model layout (doubles): header [xmin, xmax, rs, m'], then for the
// L leaf knots and the start knot (index L): {X, ylo, s, yhi} each; then the
// L + 1 mid-ranks ym, the L + 1 values y and y1 (kept for export only), and L
// previous-knot indices (u32, kNoPrev for none).
constexpr uint32_t kModelSeg = 4;
__host__ __device__ inline size_t model_ym_off(uint32_t L) { return kModelSeg + 4 * ((size_t)L + 1); }
__host__ __device__ inline size_t model_y_off(uint32_t L) { return model_ym_off(L) + L + 1; }
__host__ __device__ inline size_t model_y1_off(uint32_t L) { return model_y_off(L) + L + 1; }
__host__ __device__ inline size_t model_prev_off(uint32_t L) { return model_y1_off(L) + L + 1; }
// (rounded up to an even count, so consecutive models keep their knot
// records 16-byte aligned)
__host__ __device__ inline size_t model_doubles(uint32_t L) { return (model_prev_off(L) + (L + 1) / 2 + 1) & ~(size_t)1; }

// LDS bytes of a model in a partition kernel: L + 1 segments and mid-ranks,
// L indices.
__host__ __device__ inline size_t model_lds_bytes(uint32_t L)
{
    return (size_t)(L + 1) * 40 + (size_t)L * 2 + 32;
}

// Spill-bucket partition (LearnedSort 1.0 ablation): its scatter tile, and
// its LDS (the scatter's, the model rounded up to 16 bytes, three words per
// bucket).
constexpr uint32_t kLs1Tile = 4096;
__host__ __device__ inline size_t ls1_model_lds_bytes(uint32_t L) { return (model_lds_bytes(L) + 15) & ~(size_t)15; }
size_t ls1_scatter_lds_bytes(uint32_t fanout, uint32_t leaves);

// Keys of a round from which the default tile is doubled: a larger tile
// makes longer runs per bucket in the scatter's writes, and a round this
// large still has thousands of chunks.
constexpr uint64_t kWideTileKeys = 1ull << 25;

// LDS bytes of the scatter without its model: the staged tile (8 B keys + 2 B
// bucket numbers) and, per bucket, the cursor and the tile's write base (8 B
// each), tile count and tile start (4 B each).
__host__ __device__ inline size_t scatter_lds_bytes(uint32_t tile, uint32_t fanout)
{
    return ((size_t)tile * 10 + (size_t)fanout * 24 + 15) & ~(size_t)15;
}

// The 12,288-key tile: 32-bit cursors (task-relative; taken only by rounds
// of fewer than 2^31 keys) leave room for it when the model has at most 512
// leaves, and its runs per bucket are half as long again as the 8192-key
// tile's.
constexpr uint32_t kTile12 = 12288;
__host__ __device__ inline size_t scatter_lds_bytes32(uint32_t tile, uint32_t fanout)
{
    return ((size_t)tile * 10 + (size_t)fanout * 16 + 15) & ~(size_t)15;
}

// Keys per window within which consecutive small buckets are sorted as one
// base-case group.
constexpr uint32_t kGroupWindow = 512;
__host__ __device__ inline uint32_t group_window(uint32_t thresh)
{
    return thresh < kGroupWindow ? thresh : kGroupWindow;
}

__host__ __device__ inline uint32_t pow2_at_least(uint64_t x)
{
    uint32_t p = 1;
    while (p < x && p < (1u << 30))
        p <<= 1;
    return p;
}

// Fanout of a range of n keys: many more buckets than needed to bring it
// under the base threshold (duplicate-heavy ranges need narrow buckets for
// their repeated keys to end up alone), at least 64, capped by the caller's
// fanout.  Bounds a round's bucket count by 256 * keys / thresh.
__host__ __device__ inline uint32_t child_fanout(uint64_t n, uint32_t thresh, uint32_t cap)
{
    uint32_t f = pow2_at_least((64u * n + thresh - 1) / thresh);
    f = f < 64u ? 64u : f;
    return f > cap ? cap : f;
}

// Sample size of a global model over n keys (rate, at least 1, at most cap
// when cap is nonzero).
__host__ __device__ inline uint64_t sample_size(uint64_t n, double rate, uint64_t cap)
{
    const double want = ceil(rate * (double)n);
    uint64_t m = want < 1.0 ? 1u : (uint64_t)want;
    if (cap && m > cap)
        m = cap;
    return m;
}

// Base-case size class of a group of n keys.
__host__ __device__ inline uint32_t group_class(uint32_t n)
{
    return n <= kGroupClassCap[0] ? 0u : (n <= kGroupClassCap[1] ? 1u : 2u);
}

// Round 0 of a batch of segments described on the device (offsets and dtypes
// in device memory): the kernel writes what the host-side preparation writes
// for host-described arrays (groups of small segments, one global-model task
// and its training job per large segment, the round-0 control block) and a
// summary for the host.
struct SegPrepare {
    uint64_t* keys;
    uint64_t* scratch;            // null in place
    const uint64_t* off;          // nseg + 1 offsets
    const uint8_t* dtypes;        // null: every segment has `dtype`
    uint64_t nseg;
    uint32_t dtype, base, fanout, leaves, inplace, pad;
    double rate;
    uint64_t cap, seed;
    Task* tasks;
    ModelJob* jobs;
    Group* groups[kGroupClasses];
    RoundCtl* ctl;
    uint64_t* summary;            // kSegSummary words
};
// summary: [0] keys in base-case groups, [1] leaf-table entries of sampled
// jobs, [2] model-pool doubles, [3] nonzero when the offsets are invalid
// (offsets[0] != 0 or decreasing)
constexpr uint32_t kSegSummary = 4;
hipError_t launch_seg_prepare(const SegPrepare& A, hipStream_t st);

// Round-0 lists staged in pinned, device-mapped host memory: the control
// block at offset 0, then the tasks, the global training jobs and the groups
// of each size class at the given offsets.  The counts are the staged control
// block's (ntasks, cur.njobs, ngroups).
struct UploadPlan {
    const unsigned char* stage;   // device address of the staging area
    RoundCtl* ctl;
    Task* tasks;
    ModelJob* jobs;
    Group* groups[kGroupClasses];
    uint64_t off_tasks, off_jobs, off_groups[kGroupClasses];
};

// Kernel launchers.
// Copy the staged round-0 lists to the device (one launch, any counts).
hipError_t launch_upload(const UploadPlan& U, hipStream_t st);
// Train njobs models: gather each job's sample, sort it (runs of
// kSampleBlock in LDS, then merge passes between d_sample and d_tmp), find
// each leaf's most repeated value and fit.  d_best / d_first: per-leaf
// tables, d_nf: two counts per job; all start and end at zero.
// total: sample words of all jobs.  live (graph mode, may be null): njobs,
// total_blocks and total are upper bounds and the real counts are read from
// live (njobs, blocks, samples); max_sample, a bound on one job's sample,
// fixes the merge passes (extra passes copy whole runs).
hipError_t launch_train(const ModelJob* d_jobs, uint32_t njobs, uint32_t total_blocks, uint64_t total,
                        uint64_t max_sample, uint64_t* d_sample, uint64_t* d_tmp, uint64_t* d_best,
                        uint64_t* d_first, uint64_t* d_nf, double* d_models, const LiveCounts* live,
                        hipStream_t st);
// snapshot (graph mode): copy the next-round sizes into ctl->cur first and
// clear ctl->buckets entries (nbuckets is then the grid's upper bound).
hipError_t launch_round_init(uint64_t* d_bstat, uint64_t nbuckets, RoundCtl* d_ctl, bool snapshot, hipStream_t st);
hipError_t launch_hist(const Task* d_tasks, uint32_t ntasks, uint32_t total_chunks, uint64_t chunk,
                       const double* d_models, uint32_t* d_cnt, uint64_t* d_bstat,
                       uint32_t max_fanout, uint32_t max_leaves, uint32_t flags, const LiveCounts* live,
                       hipStream_t st);
hipError_t launch_scan(const uint32_t* d_in, uint64_t* d_out, uint64_t n, uint64_t* d_tmp, const LiveCounts* live,
                       hipStream_t st);
size_t scan_tmp_entries(uint64_t n);
// Classify every bucket of the round's tasks; the last workgroup to finish
// then lays out the next round (see launch_layout) and copies the control
// block to host_ctl (device-visible pinned host memory).
hipError_t launch_classify(const Task* d_tasks, uint32_t ntasks, const uint64_t* d_pos,
                           const uint64_t* d_bstat, uint32_t thresh, uint32_t param_fanout,
                           Task* d_next, GroupLists groups, Fill* d_fills, uint8_t* d_skip,
                           uint32_t* d_task_flags, RoundCtl* d_ctl, uint32_t max_fanout,
                           ModelJob* d_jobs, const LayoutParams& lp, RoundCtl* host_ctl, const LiveCounts* live,
                           hipStream_t st);
// Lay out the ctl->ntasks tasks of d_next: chunk size and offsets, and a
// training job for each task that needs a local model; totals go to ctl and
// to host_ctl.
hipError_t launch_layout(Task* d_next, ModelJob* d_jobs, const LayoutParams& lp, RoundCtl* d_ctl,
                         RoundCtl* host_ctl, hipStream_t st);
// Spill-bucket ablation (LearnedSort 1.0): the fixed-capacity partition of
// one task (d_task, a global-model task over the whole array), its spill
// counts per (bucket, chunk) entry, the bucket table, the packing of the
// sorted buckets into order words, the conversion back, and the library sort
// and merge of the spill area (a null temp asks for the temp size).
hipError_t launch_scatter_ls1(const Task* d_task, uint32_t nchunks, uint64_t chunk, const double* d_models,
                              const uint64_t* d_pos, const uint64_t* d_spoff, uint64_t cap, uint64_t* d_dst,
                              uint64_t* d_spill, uint32_t fanout, uint32_t leaves, hipStream_t st);
hipError_t launch_ls1_spill_counts(const uint64_t* d_pos, const uint32_t* d_cnt, uint64_t entries,
                                   uint32_t nchunks, uint64_t cap, uint32_t* d_spilled, hipStream_t st);
hipError_t launch_ls1_buckets(const uint64_t* d_pos, const uint64_t* d_spoff, const uint32_t* d_spilled,
                              uint32_t fanout, uint32_t nchunks, uint64_t n, uint64_t* d_out, hipStream_t st);
hipError_t launch_ls1_compact(const uint64_t* d_slots, const uint64_t* d_fill, uint64_t cap, uint32_t fanout,
                              uint32_t dtype, uint64_t* d_out, hipStream_t st);
hipError_t launch_from_ord(const uint64_t* d_ord, uint64_t n, uint32_t dtype, uint64_t* d_out, hipStream_t st);
hipError_t ls1_radix_sort(void* d_temp, size_t* temp_bytes, const uint64_t* d_in, uint64_t* d_out, uint64_t n,
                          hipStream_t st);
hipError_t ls1_merge(void* d_temp, size_t* temp_bytes, const uint64_t* d_a, uint64_t na, const uint64_t* d_b,
                     uint64_t nb, uint64_t* d_out, hipStream_t st);
// The scatter evaluates each key's bucket again from the task's model (the
// same arithmetic as the histogram).
hipError_t launch_scatter(const Task* d_tasks, uint32_t ntasks, uint32_t total_chunks, uint64_t chunk,
                          const double* d_models, const uint64_t* d_pos, const uint8_t* d_skip,
                          const uint32_t* d_task_flags, uint32_t tile, uint32_t max_fanout, uint32_t max_leaves,
                          uint32_t flags, const LiveCounts* live, hipStream_t st);
// In-place round (LS_FLAG_INPLACE): fragments written back into the chunks
// (cnt: keys, pcnt: partial keys per (bucket, chunk); fullb: full blocks per
// bucket, cleared by the caller; tags: the bucket of every block slot; bidx:
// the block's index among its bucket's full blocks of its chunk; side:
// ip_side_keys(chunk, fanout) keys per chunk of a task from its side_off),
// the plan of each bucket's slots, the block permutation (pos, ppos: the
// scans of cnt and pcnt; bidx becomes each slot's destination; word: one
// claim word per slot, in which `epoch` (never 0, larger every round) marks
// this round) and the gather of the rest.
hipError_t launch_ip_frag(const Task* d_tasks, uint32_t ntasks, uint32_t total_chunks, uint64_t chunk,
                          const double* d_models, uint32_t* d_cnt, uint32_t* d_pcnt, uint32_t* d_fullb,
                          uint64_t* d_bstat, uint16_t* d_tags, uint32_t* d_bidx, uint64_t* d_side,
                          uint32_t max_fanout, uint32_t max_leaves, uint32_t flags, hipStream_t st);
size_t ip_frag_lds_bytes(uint32_t fanout, uint32_t leaves);
hipError_t launch_ip_plan(const Task* d_tasks, uint32_t ntasks, uint64_t nbuckets, const uint64_t* d_pos,
                          const uint32_t* d_fullb, IpBucket* d_bk, hipStream_t st);
hipError_t launch_ip_permute(const Task* d_tasks, uint32_t ntasks, uint64_t gslots, uint64_t chunk,
                             const IpBucket* d_bk, const uint64_t* d_pos, const uint64_t* d_ppos,
                             const uint16_t* d_tags, uint32_t* d_bidx, uint32_t* d_word, uint64_t* d_ovf,
                             uint32_t epoch, RoundCtl* d_ctl, hipStream_t st);
hipError_t launch_ip_gather(const Task* d_tasks, uint32_t ntasks, uint32_t total_chunks, uint64_t chunk,
                            uint64_t nbuckets, const uint32_t* d_pcnt, const uint64_t* d_ppos, const IpBucket* d_bk,
                            const uint64_t* d_side, const uint64_t* d_ovf, hipStream_t st);
// Finishing kernels.  gctl (graph mode, may be null): ngroups / nfill are
// upper bounds, the real counts are read from gctl, and nothing is done
// while gctl->ntasks says partition rounds are still pending or after an
// overflow.
// In graph mode the grids are capped and the workgroups stride over the lists.
// One size class (cls) of base-case groups.
hipError_t launch_base(const Group* groups, uint32_t ngroups, uint32_t cls, const RoundCtl* gctl, hipStream_t st);
hipError_t launch_fill(const Fill* d_fills, uint32_t nfill, const RoundCtl* gctl, hipStream_t st);
// No-allocation sort: device address and size of this device's static
// array (looked up once per device; the device must be current).
hipError_t noalloc_setup(int device, void** out, size_t* bytes);
// Clear bytes / 8 words at p with a kernel on st.
hipError_t launch_zero(void* p, size_t bytes, hipStream_t st);
hipError_t launch_touchup(GroupLists groups, const uint32_t* ngroups, const Fill* d_fills, uint32_t nfill,
                          int full, RoundCtl* d_ctl, bool graph, hipStream_t st);

}  // namespace lsort
