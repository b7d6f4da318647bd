// Host side of the LearnedSort 2.0 pipeline and the C ABI (include/lsort.h).
//
// One sort (or one batch of arrays) runs as:
//   train   global models on a 1% sample of each large array (Sec. 6.1),
//   rounds  histogram -> scan -> classify -> layout -> scatter over every
//           task of the round (Alg. 1 as a count-then-place partition; the
//           next round's task list is built and laid out on the device, the
//           host reads back one control block per round),
//   finish  LDS base case over the groups of small buckets, fills of the
//           all-equal buckets, touch-up seam check (Alg. 2).
#include "lsort.h"
#include "lsort_internal.h"

#include <algorithm>
#include <array>
#include <cmath>
#include <condition_variable>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

using namespace lsort;

namespace {

constexpr uint32_t kDefaultFanout = 1024;
constexpr uint32_t kDefaultLeaves = 1024;
constexpr uint32_t kDefaultTile = 4096;
constexpr uint32_t kDefaultBase = 4096;
constexpr uint64_t kDefaultSeed = 0x2107032900000001ull;
constexpr uint64_t kDefaultSampleCap = 1ull << 18;   // the 1% rate holds up to 26.2M keys

struct DevBuf {
    void* p = nullptr;
    size_t cap = 0;
};

struct PinBuf {
    void* p = nullptr;
    void* dev = nullptr;   // its device address (mapped)
    size_t cap = 0;
};

struct Params {
    uint32_t fanout, leaves, tile, base, flags;
    uint32_t tile_wide = 0;         // automatic tile: large rounds use this one (0: never)
    uint32_t wide_max_fanout = 0;   // largest task fanout whose wide-tile scatter fits in LDS
    double rate;
    uint64_t cap, seed;
};

struct Array {
    uint64_t* keys;
    uint64_t* scratch;
    uint64_t n;
    uint32_t dtype;
};


// A captured replay of one batch size class (keys, arrays), valid while no
// buffer it uses has been reallocated (gen).
struct GraphEntry {
    uint64_t keys, arrays, gen;
    Params P;
    uint32_t rounds;      // partition rounds in the replay
    hipGraphExec_t exec;
    void* list_final;     // the task list the replay's last layout writes
};

// Partition rounds the last batch of a size class needed (the next replay
// of the class holds that many).
struct RoundsHint {
    uint64_t keys, arrays;
    Params P;
    uint32_t rounds;
};


}  // namespace

struct ls_ctx {
    int device = 0;
    std::string err;
    DevBuf scratch, tune, models, sample, sample2, tbest, tfirst, tnf, gjobs, ljobs, tasks, next, cnt, pos, scantmp,
        bstat,
        skip, tflags, fills, ctl;
    // in-place rounds (LS_FLAG_INPLACE): partial counts and their scan, the
    // bucket plans, full blocks per bucket, overflow blocks, block tags and
    // read flags, the side buffer of open fragments
    DevBuf pcnt, ppos, ipb, fullb, ovf, tags, done, sidebuf, bidx;
    uint32_t ip_epoch = 0;
    DevBuf groups[kGroupClasses];
    PinBuf pin_jobs;
    PinBuf estage;                   // round-0 lists of a host-driven sort (read by the upload kernel)
    RoundCtl* h_ctl = nullptr;       // pinned, device-mapped: kernels publish the control block here
    RoundCtl* d_h_ctl = nullptr;     // its device address
    uint64_t* h_flag = nullptr;      // pinned, device-mapped: set once a layout has published h_ctl
    uint64_t* d_h_flag = nullptr;
    uint64_t stats[8] = {0};
    uint32_t dev_status = 0;
    size_t lds_limit = 65536;
    // LS_FLAG_PROFILE: event pairs around each kernel class
    double prof_ms[8] = {0}, prof_launch[8] = {0}, prof_bytes[8] = {0};
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used = 0;
    // graph mode
    uint64_t gen = 0;                    // bumped whenever a buffer is reallocated
    PinBuf gstage;                       // staging of the replays' uploads
    hipStream_t cap_stream = nullptr;    // capture only; replays run on the caller's stream
    // the end of the context's last queued sort on the caller's stream:
    // sync, trim and destroy wait for this context's work, not the device's
    hipEvent_t ev_done = nullptr;
    bool done_pending = false;
    std::vector<GraphEntry> graphs;
    std::vector<RoundsHint> hints;
    // no-allocation sorts (ls_sort_noalloc): this device's static array, and
    // whether the running sort works out of it (buffers never grow then)
    void* na_base = nullptr;
    size_t na_bytes = 0;
    bool no_alloc = false;
};

namespace {

// Graph captures are kept apart from every other HIP call the library makes
// in the process (other contexts, other threads): a capture waits until no
// library call is in progress, and library calls wait while a capture is in
// progress or waiting.  A thread that captures inside a library call steps
// out of it for the capture.
struct CaptureGate {
    std::mutex m;
    std::condition_variable cv;
    int active = 0, waiting = 0;
    bool capturing = false;
};

CaptureGate& capture_gate()
{
    static CaptureGate g;
    return g;
}

thread_local int t_gate_depth = 0;

struct GateUse {
    GateUse()
    {
        if (t_gate_depth++ != 0)
            return;
        CaptureGate& G = capture_gate();
        std::unique_lock<std::mutex> lk(G.m);
        G.cv.wait(lk, [&] { return !G.capturing && G.waiting == 0; });
        ++G.active;
    }
    ~GateUse()
    {
        if (--t_gate_depth != 0)
            return;
        CaptureGate& G = capture_gate();
        {
            std::lock_guard<std::mutex> lk(G.m);
            --G.active;
        }
        G.cv.notify_all();
    }
};

struct GateCapture {
    bool inside;
    GateCapture()
    {
        CaptureGate& G = capture_gate();
        std::unique_lock<std::mutex> lk(G.m);
        inside = t_gate_depth > 0;
        if (inside)
            --G.active;
        ++G.waiting;
        G.cv.notify_all();
        G.cv.wait(lk, [&] { return !G.capturing && G.active == 0; });
        --G.waiting;
        G.capturing = true;
    }
    ~GateCapture()
    {
        CaptureGate& G = capture_gate();
        std::unique_lock<std::mutex> lk(G.m);
        G.capturing = false;
        G.cv.notify_all();
        if (inside) {
            G.cv.wait(lk, [&] { return !G.capturing && G.waiting == 0; });
            ++G.active;
        }
    }
};

ls_status fail(ls_ctx* C, ls_status s, const std::string& msg)
{
    if (C)
        C->err = msg;
    return s;
}

#define HIPCHECK(C, expr)                                                                      \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess)                                                                  \
            return fail((C), LS_ERR_HIP, std::string(#expr ": ") + hipGetErrorString(e_));     \
    } while (0)

#define TRY(expr)                       \
    do {                                \
        ls_status s_ = (expr);          \
        if (s_ != LS_OK)                \
            return s_;                  \
    } while (0)

// Grow a device buffer; queued work may still use the old one, so wait first.
ls_status ensure(ls_ctx* C, DevBuf& b, size_t bytes, hipStream_t st, size_t keep = 0)
{
    if (bytes <= b.cap && b.p)
        return LS_OK;
    if (C->no_alloc)
        return fail(C, LS_ERR_NOMEM, "no-allocation sort: a buffer needs " + std::to_string(bytes) +
                                         " bytes, more than its share of the static array");
    size_t nb = std::max(bytes, b.cap + b.cap / 2);
    nb = std::max<size_t>(nb, 256);
    void* np = nullptr;
    if (hipMalloc(&np, nb) != hipSuccess) {
        (void)hipGetLastError();
        return fail(C, LS_ERR_NOMEM, "device allocation of " + std::to_string(nb) + " bytes failed");
    }
    HIPCHECK(C, hipStreamSynchronize(st));
    if (keep && b.p)
        HIPCHECK(C, hipMemcpy(np, b.p, std::min(keep, b.cap), hipMemcpyDeviceToDevice));
    if (b.p)
        HIPCHECK(C, hipFree(b.p));
    b.p = np;
    b.cap = nb;
    ++C->gen;
    return LS_OK;
}

// Pinned staging for asynchronous uploads.
ls_status ensure_pinned(ls_ctx* C, PinBuf& b, size_t bytes, hipStream_t st)
{
    if (bytes <= b.cap && b.p)
        return LS_OK;
    if (C->no_alloc)
        return fail(C, LS_ERR_NOMEM, "no-allocation sort: the round-0 lists need more pinned staging than the "
                                     "context holds");
    HIPCHECK(C, hipStreamSynchronize(st));
    if (b.p)
        HIPCHECK(C, hipHostFree(b.p));
    b.p = b.dev = nullptr;
    size_t nb = std::max<size_t>({bytes, b.cap * 2, 4096});
    if (hipHostMalloc(&b.p, nb, hipHostMallocMapped) != hipSuccess ||
        hipHostGetDevicePointer(&b.dev, b.p, 0) != hipSuccess) {
        (void)hipGetLastError();
        if (b.p)
            (void)hipHostFree(b.p);
        b.p = b.dev = nullptr;
        b.cap = 0;
        return fail(C, LS_ERR_NOMEM, "pinned host allocation failed");
    }
    b.cap = nb;
    ++C->gen;
    return LS_OK;
}

template <typename T>
ls_status upload(ls_ctx* C, PinBuf& pin, DevBuf& dst, const std::vector<T>& v, hipStream_t st)
{
    if (v.empty())
        return LS_OK;
    const size_t bytes = v.size() * sizeof(T);
    TRY(ensure_pinned(C, pin, bytes, st));
    std::memcpy(pin.p, v.data(), bytes);
    HIPCHECK(C, hipMemcpyAsync(dst.p, pin.p, bytes, hipMemcpyHostToDevice, st));
    return LS_OK;
}

// Event pairs around the launches of the kernel classes being timed; read
// back at the end of the sort, after its final stream sync.
struct Prof {
    ls_ctx* C;
    hipStream_t st;
    bool on;
    struct Rec {
        int k;
        hipEvent_t a, b;
        double bytes;
    };
    std::vector<Rec> recs;
    int only = -1;        // time only this class (LS_FLAG_PROFILE_ONLY), -1: all
    bool open = false;    // the last begin() recorded an event
    hipEvent_t ev()
    {
        if (C->ev_used == C->ev_pool.size()) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess)
                return nullptr;
            C->ev_pool.push_back(e);
        }
        return C->ev_pool[C->ev_used++];
    }
    void begin(int k)
    {
        open = false;
        if (!on || (only >= 0 && k != only))
            return;
        Rec r{k, ev(), ev(), 0.0};
        if (r.a && r.b && hipEventRecord(r.a, st) == hipSuccess) {
            recs.push_back(r);
            open = true;
        }
    }
    void end(double bytes)
    {
        if (!open)
            return;
        open = false;
        recs.back().bytes = bytes;
        (void)hipEventRecord(recs.back().b, st);
    }
    // after the final stream sync of the sort (every event is complete)
    void collect()
    {
        for (auto& r : recs) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
                C->prof_ms[r.k] += ms;
                C->prof_launch[r.k] += 1;
                C->prof_bytes[r.k] += r.bytes;
            }
        }
        recs.clear();
        C->ev_used = 0;
    }
};

ls_status resolve(ls_ctx* C, const ls_params* p, Params& P)
{
    P.fanout = kDefaultFanout;
    P.leaves = kDefaultLeaves;
    P.tile = kDefaultTile;
    P.tile_wide = p ? 0 : 2 * kDefaultTile;
    P.base = kDefaultBase;
    P.flags = 0;
    P.rate = 0.01;
    P.cap = kDefaultSampleCap;
    P.seed = kDefaultSeed;
    if (p) {
        if (p->struct_size != sizeof(ls_params))
            return fail(C, LS_ERR_INVALID, "ls_params.struct_size mismatch");
        if (p->fanout) P.fanout = p->fanout;
        if (p->leaves) P.leaves = p->leaves;
        if (p->tile) P.tile = p->tile;
        else P.tile_wide = 2 * kDefaultTile;
        if (p->base_threshold) P.base = p->base_threshold;
        P.flags = p->flags;
        if (((P.flags >> 8) & 0xfu) > 8u)
            return fail(C, LS_ERR_INVALID, "LS_FLAG_PROFILE_ONLY takes a kernel class 0..7");
        if (p->sample_rate != 0.0) P.rate = p->sample_rate;
        P.cap = p->sample_cap;
        if (p->seed) P.seed = p->seed;
    }
    if (P.fanout < 2 || P.fanout > kMaxFanout)
        return fail(C, LS_ERR_INVALID, "fanout must be in [2, 4096]");
    if (P.flags & LS_FLAG_INPLACE)   // one open fragment per bucket in LDS
        P.fanout = std::min(P.fanout, kIpFanout);
    if (P.leaves < 1 || P.leaves > kMaxLeaves)
        return fail(C, LS_ERR_INVALID, "leaves must be in [1, 1024]");
    if (P.tile != 1024 && P.tile != 2048 && P.tile != 4096 && P.tile != 8192)
        return fail(C, LS_ERR_INVALID, "tile must be 0 (automatic), 1024, 2048, 4096 or 8192");
    if (P.base < 2 || 2 * P.base > kMaxBase)
        return fail(C, LS_ERR_INVALID, "base_threshold must be in [2, 4096]");
    if (!(P.rate > 0.0) || P.rate > 1.0)
        return fail(C, LS_ERR_INVALID, "sample_rate must be in (0, 1]");
    // the scatter holds the staged tile, per-bucket tables and the model
    const size_t model_lds = model_lds_bytes(P.leaves);
    auto scatter_lds = [&](uint32_t tile) { return scatter_lds_bytes(tile, P.fanout) + model_lds + 128; };
    // the largest tile up to the given (or automatic) one that fits
    while (P.tile > 1024 && scatter_lds(P.tile) > C->lds_limit)
        P.tile /= 2;
    size_t hist_lds = (((size_t)P.fanout * 20 + 15) & ~(size_t)15) + model_lds + 64;
    if (scatter_lds(P.tile) > C->lds_limit || hist_lds > C->lds_limit ||
        ((P.flags & LS_FLAG_INPLACE) && ip_frag_lds_bytes(P.fanout, P.leaves) + 128 > C->lds_limit))
        return fail(C, LS_ERR_UNSUPPORTED, "tile/fanout/leaves exceed the LDS of one workgroup");
    // automatic tile: the wide tile is taken only by rounds whose fanouts fit
    P.wide_max_fanout = 0;
    if (P.tile_wide) {
        // the 12,288-key tile (32-bit cursors) where the model leaves room for it
        const size_t fixed12 = scatter_lds_bytes32(kTile12, 0) + model_lds + 128 + 16;
        const size_t f12 = C->lds_limit > fixed12 ? (C->lds_limit - fixed12) / 16 : 0;
        if (f12 >= P.fanout) {
            P.tile_wide = kTile12;
            P.wide_max_fanout = (uint32_t)std::min<size_t>(f12, kMaxFanout);
            return LS_OK;
        }
    }
    if (P.tile_wide) {
        const size_t fixed = scatter_lds_bytes(P.tile_wide, 0) + model_lds + 128 + 16;
        P.wide_max_fanout = C->lds_limit > fixed ? (uint32_t)std::min<size_t>((C->lds_limit - fixed) / 24, kMaxFanout)
                                                 : 0u;
        if (P.wide_max_fanout < 2)
            P.tile_wide = 0;
    }
    return LS_OK;
}

// Global models of the large arrays, built on the host.
struct Trainer {
    std::vector<ModelJob> jobs;
    uint64_t samples = 0, leaves = 0, models = 0, max_sample = 0;
    uint32_t blocks = 0;

    uint64_t add(const uint64_t* src, uint64_t n, uint64_t m, uint64_t seed, uint32_t L, uint32_t dtype)
    {
        ModelJob J;
        J.src = src;
        J.n = n;
        J.m = m;
        J.seed = seed;
        J.sample_off = samples;
        J.model_off = models;
        J.leaf_off = leaves;
        J.leaves = L;
        J.dtype = dtype;
        J.block0 = blocks;
        // (a job whose sample fits one LDS run takes no room in the sample
        // buffers and leaf tables: it trains in one workgroup)
        const bool sampled = m > kSampleBlock;
        J.nblocks = sampled ? (uint32_t)((m + kSampleBlock - 1) / kSampleBlock) : 0u;
        max_sample = std::max(max_sample, m);
        samples += sampled ? m : 0;
        leaves += sampled ? L : 0;
        models += model_doubles(L);
        blocks += J.nblocks;
        jobs.push_back(J);
        return J.model_off;
    }
};

// Train njobs models described by d_jobs (device) into the pool at model_base.
ls_status train(ls_ctx* C, const DevBuf& jobs, uint32_t njobs, uint32_t blocks, uint64_t samples, uint64_t leafs,
                uint64_t max_sample, uint64_t model_base, uint64_t models, hipStream_t st, Prof* prof)
{
    if (!njobs)
        return LS_OK;
    TRY(ensure(C, C->models, (model_base + models) * sizeof(double), st, model_base * sizeof(double)));
    // jobs whose sample fits one LDS run need no global buffers
    if (max_sample > kSampleBlock) {
        TRY(ensure(C, C->sample, samples * 8, st));
        TRY(ensure(C, C->sample2, samples * 8, st));
        // the per-leaf and per-job tables start at zero and the fit kernel
        // leaves them at zero; only freshly allocated memory needs clearing
        DevBuf* tabs[3] = {&C->tbest, &C->tfirst, &C->tnf};
        const size_t need[3] = {leafs * 8, leafs * 8, (size_t)njobs * 16};
        for (int i = 0; i < 3; ++i) {
            const void* before = tabs[i]->p;
            TRY(ensure(C, *tabs[i], need[i], st));
            if (tabs[i]->p != before)
                HIPCHECK(C, hipMemsetAsync(tabs[i]->p, 0, tabs[i]->cap, st));
        }
    }
    if (prof)
        prof->begin(0);
    HIPCHECK(C, launch_train((const ModelJob*)jobs.p, njobs, blocks, samples, max_sample, (uint64_t*)C->sample.p,
                             (uint64_t*)C->sample2.p, (uint64_t*)C->tbest.p, (uint64_t*)C->tfirst.p,
                             (uint64_t*)C->tnf.p, (double*)C->models.p, nullptr, st));
    if (prof)
        prof->end((double)samples * 16.0);
    return LS_OK;
}

ls_status read_ctl(ls_ctx* C, hipStream_t st)
{
    HIPCHECK(C, hipMemcpyAsync(C->h_ctl, C->ctl.p, sizeof(RoundCtl), hipMemcpyDeviceToHost, st));
    HIPCHECK(C, hipStreamSynchronize(st));
    return LS_OK;
}

// The layout (alone, or at the end of classify) writes the control block
// into mapped host memory and then sets a flag there.
//
// Clear the publish flag before launching a layout that sets it.
void arm_publish(ls_ctx* C)
{
    __atomic_store_n(C->h_flag, 0ull, __ATOMIC_RELEASE);
}

// Wait until the layout has published the control block (its flag is set),
// not for the whole stream: the round's scatter may still run while the host
// reads the next round's sizes and queues its launches behind it.  If the
// stream drains (or fails) without the flag, the wait ends with an error.
ls_status wait_published(ls_ctx* C, hipStream_t st)
{
    for (uint32_t spin = 1;; ++spin) {
        if (__atomic_load_n(C->h_flag, __ATOMIC_ACQUIRE))
            return LS_OK;
        if (spin % 4096 == 0) {
            const hipError_t e = hipStreamQuery(st);
            if (e == hipSuccess) {
                if (__atomic_load_n(C->h_flag, __ATOMIC_ACQUIRE))
                    return LS_OK;
                return fail(C, LS_ERR_HIP, "the control block was not published");
            }
            if (e != hipErrorNotReady) {
                (void)hipGetLastError();
                return fail(C, LS_ERR_HIP, std::string("stream failed: ") + hipGetErrorString(e));
            }
        }
        __builtin_ia32_pause();
    }
}

// Round-0 work of a batch: small arrays go straight to the base case, large
// ones get a global model (level 0 of Alg. 2), or an MSD split of the key
// bits in the repair pass.
struct Batch {
    std::vector<Group> groups0[kGroupClasses];
    std::vector<Task> tasks;
    Trainer tr;
    uint64_t total = 0, group0_keys = 0;
};

void prepare(std::vector<Array>& arrays, void* scratch, const Params& P, bool msd_only, Batch& B)
{
    const uint32_t lf = 31u - (uint32_t)__builtin_clz(P.fanout);
    // in-place rounds keep every key in the caller's buffer
    const bool inplace = (P.flags & LS_FLAG_INPLACE) != 0;
    uint64_t off = 0;
    for (uint32_t i = 0; i < arrays.size(); ++i) {
        Array& a = arrays[i];
        a.scratch = inplace ? a.keys : (uint64_t*)scratch + off;
        off += a.n;
        if (a.n <= 1)
            continue;
        if (a.n <= 2ull * P.base) {
            B.groups0[group_class((uint32_t)a.n)].push_back(Group{a.keys, a.keys, 0, (uint32_t)a.n, a.dtype, ~0ull, 0});
            B.group0_keys += a.n;
            continue;
        }
        Task t{};
        t.keys = a.keys;
        t.scratch = a.scratch;
        t.n = a.n;
        t.dtype = a.dtype;
        t.seg = i;
        if (msd_only) {
            t.kind = kMsd;
            t.fanout = inplace ? ip_fanout(a.n, 1u << lf) : 1u << lf;
            t.shift = 64 - lf;
        } else {
            t.kind = kGlobal;
            t.fanout = child_fanout(a.n, P.base, P.fanout);
            if (inplace)
                t.fanout = ip_fanout(a.n, t.fanout);
            t.scale = (double)t.fanout;
            t.leaves = P.leaves;
            t.model = B.tr.add(a.keys, a.n, sample_size(a.n, P.rate, P.cap), P.seed, P.leaves, a.dtype);
        }
        B.tasks.push_back(t);
    }
    B.total = off;
}

// Where the round-0 lists of a batch sit in a staging area (control block
// first), for the given capacities.
struct StageLayout {
    size_t off_tasks, off_jobs, off_groups[kGroupClasses], bytes;
};

StageLayout stage_layout(uint64_t tasks, uint64_t jobs, const uint64_t* groups)
{
    StageLayout L;
    size_t off = (sizeof(RoundCtl) + 255) & ~(size_t)255;
    L.off_tasks = off;
    off += tasks * sizeof(Task);
    L.off_jobs = off;
    off += jobs * sizeof(ModelJob);
    for (uint32_t c = 0; c < kGroupClasses; ++c) {
        L.off_groups[c] = off;
        off += groups[c] * sizeof(Group);
    }
    L.bytes = off;
    return L;
}

// Write a batch's round-0 lists and initial control block into a staging
// area laid out by L.
void fill_stage(unsigned char* sp, const StageLayout& L, const Batch& B)
{
    RoundCtl* c0 = reinterpret_cast<RoundCtl*>(sp);
    std::memset(c0, 0, sizeof(RoundCtl));
    c0->ntasks = (uint32_t)B.tasks.size();
    for (uint32_t c = 0; c < kGroupClasses; ++c) {
        c0->ngroups[c] = (uint32_t)B.groups0[c].size();
        if (!B.groups0[c].empty())
            std::memcpy(sp + L.off_groups[c], B.groups0[c].data(), B.groups0[c].size() * sizeof(Group));
    }
    // the global training reads its sizes here
    c0->cur.njobs = (uint32_t)B.tr.jobs.size();
    c0->cur.blocks = B.tr.blocks;
    c0->cur.samples = B.tr.samples;
    c0->cur.max_sample = B.tr.max_sample;
    if (!B.tasks.empty())
        std::memcpy(sp + L.off_tasks, B.tasks.data(), B.tasks.size() * sizeof(Task));
    if (!B.tr.jobs.empty())
        std::memcpy(sp + L.off_jobs, B.tr.jobs.data(), B.tr.jobs.size() * sizeof(ModelJob));
}

UploadPlan upload_plan(ls_ctx* C, const PinBuf& stage, const StageLayout& L)
{
    UploadPlan U;
    U.stage = (const unsigned char*)stage.dev;
    U.ctl = (RoundCtl*)C->ctl.p;
    U.tasks = (Task*)C->next.p;
    U.jobs = (ModelJob*)C->gjobs.p;
    U.off_tasks = L.off_tasks;
    U.off_jobs = L.off_jobs;
    for (uint32_t c = 0; c < kGroupClasses; ++c) {
        U.groups[c] = (Group*)C->groups[c].p;
        U.off_groups[c] = L.off_groups[c];
    }
    return U;
}

constexpr uint64_t kUnbounded = ~0ull;

LayoutParams layout_params(const Params& P, uint64_t model_base)
{
    LayoutParams lp;
    std::memset(&lp, 0, sizeof lp);
    lp.fanout = P.fanout;
    lp.leaves = P.leaves;
    lp.tile = P.tile;
    lp.tile_wide = P.tile_wide;
    lp.wide_keys = kWideTileKeys;
    lp.wide_max_fanout = P.wide_max_fanout;
    // in-place rounds: one chunk per CU, so that the open fragments left at
    // the chunks' ends (side buffer) stay a small fraction of the keys
    lp.target_chunks = (P.flags & LS_FLAG_INPLACE) ? kSmallRoundChunks : kTargetChunks;
    lp.inplace = (P.flags & LS_FLAG_INPLACE) ? 1u : 0u;
    lp.rate = P.rate;
    lp.cap = P.cap;
    lp.seed = P.seed;
    lp.model_base = model_base;
    lp.cap_tasks = lp.cap_fills = kUnbounded;
    for (uint32_t c = 0; c < kGroupClasses; ++c)
        lp.cap_groups[c] = kUnbounded;
    lp.cap_keys = lp.cap_chunks = lp.cap_buckets = lp.cap_entries = kUnbounded;
    lp.cap_samples = lp.cap_blocks = lp.cap_leafs = lp.cap_models = kUnbounded;
    return lp;
}

ls_status check_overflow(ls_ctx* C)
{
    if (C->h_ctl->overflow & 2u)
        return fail(C, LS_ERR_HIP, "in-place block permutation: a block slot was not released in time");
    if (C->h_ctl->overflow)
        return fail(C, LS_ERR_HIP, "a partition round exceeded its buffers (internal size bound)");
    return LS_OK;
}

// Partition rounds, driven from the host: each round's launches are sized
// from the control block the previous layout published.
ls_status rounds_eager(ls_ctx* C, hipStream_t st, const Params& P, LayoutParams lp, uint32_t flags, Prof& prof)
{
    // each layout sets the flag once the control block is published; the
    // profile's events are read at the end of the sort, when all are done
    lp.host_flag = C->d_h_flag;
    while (C->h_ctl->ntasks) {
        const RoundCtl R = *C->h_ctl;
        const uint32_t nt = R.ntasks;
        std::swap(C->tasks, C->next);
        TRY(ensure(C, C->cnt, R.entries * 4, st));
        TRY(ensure(C, C->pos, R.entries * 8, st));
        TRY(ensure(C, C->scantmp, scan_tmp_entries(R.entries) * 8, st));
        TRY(ensure(C, C->bstat, (uint64_t)R.buckets * 16, st));
        TRY(ensure(C, C->skip, R.buckets, st));
        TRY(ensure(C, C->tflags, (size_t)nt * 4, st));
        const bool inplace = (P.flags & LS_FLAG_INPLACE) != 0;
        const uint64_t gslots = R.nkeys / kIpBlock + nt + 1;   // block slots of the round's tasks
        if (inplace) {
            TRY(ensure(C, C->pcnt, R.entries * 4, st));
            TRY(ensure(C, C->ppos, R.entries * 8, st));
            TRY(ensure(C, C->ipb, R.buckets * sizeof(IpBucket), st));
            TRY(ensure(C, C->fullb, (R.buckets + 1) / 2 * 8, st));
            TRY(ensure(C, C->ovf, R.buckets * kIpBlock * 8, st));
            TRY(ensure(C, C->tags, gslots * 2, st));
            TRY(ensure(C, C->bidx, gslots * 4, st));
            TRY(ensure(C, C->sidebuf, std::max<size_t>(R.side_keys, 1) * 8, st));
            // read flags hold the epoch of the round that released the slot
            // (never 0, the value of a cleared flag)
            const void* before = C->done.p;
            TRY(ensure(C, C->done, (gslots + 1) / 2 * 8, st));
            if (C->done.p != before)
                HIPCHECK(C, launch_zero(C->done.p, C->done.cap / 8 * 8, st));
        }
        // Output lists, sized by what classify can emit: a next-round task
        // is a bucket of at least 2T keys; a fill bucket holds at least
        // max(T/8, 2) keys (plus one piece per kFillPiece keys); a group of
        // class c > 0 holds more than the previous class cap; a group of
        // class 0 is a solo bucket (more than T keys) or starts where a run
        // of small buckets is broken by the task start, a W-key window
        // boundary (W = group_window(T) <= T) or a big / fill / solo bucket,
        // so there are at most 3 n/W + n/fill_min + 2 of them per task.
        const uint64_t max_tasks = std::min<uint64_t>(R.buckets, R.nkeys / (2ull * P.base)) + 1;
        const uint64_t fill_min = std::max<uint64_t>(P.base / 8, 2);
        const uint64_t max_fills = std::min<uint64_t>(R.buckets, R.nkeys / fill_min) + R.nkeys / kFillPiece + 1;
        const uint64_t g0 = 3 * (R.nkeys / group_window(P.base)) + R.nkeys / fill_min + 2 * (uint64_t)nt + 2;
        const uint64_t max_groups[kGroupClasses] = {std::min<uint64_t>(R.buckets, g0) + 1,
                                                    R.nkeys / (kGroupClassCap[0] + 1) + 1,
                                                    R.nkeys / (kGroupClassCap[1] + 1) + 1};
        TRY(ensure(C, C->next, max_tasks * sizeof(Task), st));
        GroupLists gl;
        // (a no-allocation sort keeps the lists it was given, sized for the
        // whole sort; classify's capacity check guards them)
        for (uint32_t c = 0; c < kGroupClasses; ++c) {
            if (!C->no_alloc)
                TRY(ensure(C, C->groups[c], ((size_t)R.ngroups[c] + max_groups[c]) * sizeof(Group), st,
                           (size_t)R.ngroups[c] * sizeof(Group)));
            gl.g[c] = (Group*)C->groups[c].p;
            lp.cap_groups[c] = C->groups[c].cap / sizeof(Group);
        }
        if (!C->no_alloc)
            TRY(ensure(C, C->fills, ((size_t)R.nfill + max_fills) * sizeof(Fill), st,
                       (size_t)R.nfill * sizeof(Fill)));
        lp.cap_fills = C->fills.cap / sizeof(Fill);
        // local models of this round's tasks (jobs written by the last layout)
        TRY(train(C, C->ljobs, R.njobs, R.blocks, R.samples, R.leafs, R.max_sample, lp.model_base, R.models, st,
                  &prof));
        TRY(ensure(C, C->ljobs, max_tasks * sizeof(ModelJob), st));
        lp.cap_tasks = std::min(C->next.cap / sizeof(Task), C->ljobs.cap / sizeof(ModelJob));
        HIPCHECK(C, launch_round_init((uint64_t*)C->bstat.p, R.buckets, (RoundCtl*)C->ctl.p, false, st));
        prof.begin(1);
        if (inplace) {
            // fragments written back into each chunk (Alg. 1): every key read
            // and written once
            HIPCHECK(C, launch_zero(C->fullb.p, (R.buckets + 1) / 2 * 8, st));
            HIPCHECK(C, launch_ip_frag((const Task*)C->tasks.p, nt, R.chunks, R.chunk, (const double*)C->models.p,
                                       (uint32_t*)C->cnt.p, (uint32_t*)C->pcnt.p, (uint32_t*)C->fullb.p,
                                       (uint64_t*)C->bstat.p, (uint16_t*)C->tags.p, (uint32_t*)C->bidx.p,
                                       (uint64_t*)C->sidebuf.p,
                                       R.max_fanout, R.max_leaves, flags, st));
            prof.end((double)R.nkeys * 16.0);
        } else {
            HIPCHECK(C, launch_hist((const Task*)C->tasks.p, nt, R.chunks, R.chunk, (const double*)C->models.p,
                                    (uint32_t*)C->cnt.p, (uint64_t*)C->bstat.p, R.max_fanout, R.max_leaves, flags,
                                    nullptr, st));
            // the method reads each key once
            prof.end((double)R.nkeys * 8.0);
        }
        prof.begin(2);
        HIPCHECK(C, launch_scan((const uint32_t*)C->cnt.p, (uint64_t*)C->pos.p, R.entries, (uint64_t*)C->scantmp.p,
                                nullptr, st));
        if (inplace)
            HIPCHECK(C, launch_scan((const uint32_t*)C->pcnt.p, (uint64_t*)C->ppos.p, R.entries,
                                    (uint64_t*)C->scantmp.p, nullptr, st));
        prof.end((double)R.entries * (inplace ? 32.0 : 16.0));
        prof.begin(3);
        arm_publish(C);
        HIPCHECK(C, launch_classify((const Task*)C->tasks.p, nt, (const uint64_t*)C->pos.p,
                                    (const uint64_t*)C->bstat.p, P.base, P.fanout, (Task*)C->next.p, gl,
                                    (Fill*)C->fills.p, (uint8_t*)C->skip.p, (uint32_t*)C->tflags.p,
                                    (RoundCtl*)C->ctl.p, R.max_fanout, (ModelJob*)C->ljobs.p, lp, C->d_h_ctl,
                                    nullptr, st));
        prof.end((double)R.buckets * 32.0);
        const size_t scatter_rec = prof.recs.size();
        prof.begin(4);
        if (inplace) {
            // Defragment: blocks to their buckets' slots, then the open
            // fragments and overflow blocks to the rest of each bucket
            HIPCHECK(C, launch_ip_plan((const Task*)C->tasks.p, nt, R.buckets, (const uint64_t*)C->pos.p,
                                       (const uint32_t*)C->fullb.p, (IpBucket*)C->ipb.p, st));
            // claim words hold 2 epoch and 2 epoch + 1 of their round; once
            // the epoch would pass 2^31 they are cleared and it starts over
            if (++C->ip_epoch >= (1u << 31)) {
                HIPCHECK(C, launch_zero(C->done.p, C->done.cap / 8 * 8, st));
                C->ip_epoch = 1;
            }
            HIPCHECK(C, launch_ip_permute((const Task*)C->tasks.p, nt, gslots, R.chunk, (const IpBucket*)C->ipb.p,
                                          (const uint64_t*)C->pos.p, (const uint64_t*)C->ppos.p,
                                          (const uint16_t*)C->tags.p, (uint32_t*)C->bidx.p, (uint32_t*)C->done.p,
                                          (uint64_t*)C->ovf.p, C->ip_epoch, (RoundCtl*)C->ctl.p, st));
            HIPCHECK(C, launch_ip_gather((const Task*)C->tasks.p, nt, R.chunks, R.chunk, R.buckets,
                                         (const uint32_t*)C->pcnt.p,
                                         (const uint64_t*)C->ppos.p, (const IpBucket*)C->ipb.p,
                                         (const uint64_t*)C->sidebuf.p, (const uint64_t*)C->ovf.p, st));
            // every key read and written once more (blocks and the rest)
            prof.end((double)R.nkeys * 16.0);
        } else {
            HIPCHECK(C, launch_scatter((const Task*)C->tasks.p, nt, R.chunks, R.chunk, (const double*)C->models.p,
                                       (const uint64_t*)C->pos.p, (const uint8_t*)C->skip.p,
                                       (const uint32_t*)C->tflags.p, R.tile, R.max_fanout, R.max_leaves, flags,
                                       nullptr, st));
            prof.end(0.0);
        }
        TRY(wait_published(C, st));
        if (!inplace && prof.recs.size() > scatter_rec) {
            // scatter: reads every key of a task that progressed and writes
            // those not in all-equal buckets
            const double moved = (double)(R.nkeys - (C->h_ctl->stall_keys - R.stall_keys));
            const double kept = moved - (double)(C->h_ctl->fillkeys - R.fillkeys);
            prof.recs.back().bytes = 8.0 * moved + 8.0 * kept;
        }
        TRY(check_overflow(C));
    }
    return LS_OK;
}

// The base case over the three size classes and the fills, one after
// another on the sort's stream.  (Running classes 1 and 2 on side streams
// forked from it and joined back was slower on every workload measured: the
// cross-stream waits cost more than the overlap gained.)
ls_status launch_finish_lists(ls_ctx* C, const GroupLists& gl, const uint32_t* ngroups, const Fill* fills,
                              uint32_t nfill, const RoundCtl* gctl, hipStream_t st)
{
    for (uint32_t c = 0; c < kGroupClasses; ++c)
        HIPCHECK(C, launch_base(gl.g[c], ngroups[c], c, gctl, st));
    HIPCHECK(C, launch_fill(fills, nfill, gctl, st));
    return LS_OK;
}

// Finish: LDS base case, all-equal fills, touch-up; reads the final control
// block back.
ls_status finish_eager(ls_ctx* C, hipStream_t st, const Params& P, Prof& prof, uint64_t group0_keys)
{
    const RoundCtl F = *C->h_ctl;
    GroupLists gl;
    for (uint32_t c = 0; c < kGroupClasses; ++c)
        gl.g[c] = (Group*)C->groups[c].p;
    const double gkeys = (double)F.group_keys + (double)group0_keys;
    if (prof.on) {
        // timed one kernel class at a time
        prof.begin(5);
        for (uint32_t c = 0; c < kGroupClasses; ++c)
            HIPCHECK(C, launch_base(gl.g[c], F.ngroups[c], c, nullptr, st));
        prof.end(16.0 * gkeys);
        prof.begin(6);
        HIPCHECK(C, launch_fill((const Fill*)C->fills.p, F.nfill, nullptr, st));
        prof.end(8.0 * (double)F.fillkeys);
    } else {
        TRY(launch_finish_lists(C, gl, F.ngroups, (const Fill*)C->fills.p, F.nfill, nullptr, st));
    }
    prof.begin(7);
    HIPCHECK(C, launch_touchup(gl, F.ngroups, (const Fill*)C->fills.p, F.nfill,
                               (P.flags & LS_FLAG_DEBUG_TOUCHUP) ? 1 : 0, (RoundCtl*)C->ctl.p, false, st));
    const uint64_t ngroups = (uint64_t)F.ngroups[0] + F.ngroups[1] + F.ngroups[2];
    prof.end(16.0 * (double)(ngroups + F.nfill));
    TRY(read_ctl(C, st));
    prof.collect();
    return LS_OK;
}

ls_status run_pipeline(ls_ctx* C, std::vector<Array>& arrays, hipStream_t st, const Params& P, bool msd_only);

// Statistics of the finished sort, and the touch-up repair when a seam was
// out of order.
ls_status conclude(ls_ctx* C, std::vector<Array>& arrays, hipStream_t st, const Params& P, bool msd_only)
{
    TRY(check_overflow(C));
    const RoundCtl fin = *C->h_ctl;
    C->stats[0] = fin.rounds;
    C->stats[1] = fin.tasks_total;
    C->stats[2] = (uint64_t)fin.ngroups[0] + fin.ngroups[1] + fin.ngroups[2];
    C->stats[3] = fin.nfillbuckets;
    C->stats[4] = fin.fillkeys;
    C->stats[5] = fin.fallbacks;
    C->stats[6] = fin.violations;
    C->stats[7] = fin.deepest;
    if (fin.fallbacks)
        C->dev_status |= LS_DEV_FALLBACK;
    if (fin.deepest > 1)
        C->dev_status |= LS_DEV_DEEP;
    if (fin.violations) {
        if (msd_only)
            return fail(C, LS_ERR_HIP, "touch-up found out-of-order seams after the repair pass");
        // Touch-up repair: the model put keys out of order (only possible
        // with the test hook); re-partition on the key bits alone.
        uint64_t saved[8];
        std::memcpy(saved, C->stats, sizeof saved);
        TRY(run_pipeline(C, arrays, st, P, true));
        std::memcpy(C->stats, saved, sizeof saved);
        C->dev_status |= LS_DEV_SEAM_REPAIRED;
    }
    return LS_OK;
}

// ------------------------------------------------------------ graph mode --
//
// A batch of at most kGraphMaxKeys keys can run as one replay of a HIP graph
// captured for its size class (keys and arrays rounded up to powers of two):
// uploads of the round-0 lists, global training, layout, R partition rounds
// and the finish.  R is the number of rounds the class's last batch needed
// (at most kGraphMaxRounds; one graph per R).  Every buffer is sized from
// bounds on what kGraphMaxRounds rounds of the class can produce, the kernels
// are launched with grids for those bounds and read their real sizes from
// the control block, and rounds past the last task run nothing.  A batch
// that needs more rounds continues on the host-driven path from the state
// the replay left.

constexpr uint64_t kGraphMinKeys = 1ull << 16;
constexpr uint64_t kGraphMaxKeys = 1ull << 22;
constexpr uint64_t kGraphMinArrays = 64;
constexpr uint64_t kGraphMaxArrays = 1ull << 16;
constexpr uint32_t kGraphMaxRounds = 4;
constexpr uint32_t kGraphFirstRounds = 2;   // hint for a class's first batch

uint64_t pow2_ge(uint64_t x)
{
    uint64_t p = 1;
    while (p < x)
        p <<= 1;
    return p;
}

// Upper bounds for a batch of at most `keys` keys in at most `arrays` arrays.
struct Caps {
    uint64_t keys, arrays;
    // round 0
    uint64_t tasks0, gsamples, gblocks, gleafs, gmodels, gmax_sample;
    // one partition round
    uint64_t tasks, chunks, buckets, entries, samples, blocks, leafs, models, max_sample;
    // over the whole replay
    uint64_t groups[kGroupClasses], fills;
    StageLayout stage;   // round-0 lists: tasks0 tasks and jobs, `arrays` groups per class
};

Caps graph_caps(uint64_t keys, uint64_t arrays, const Params& P)
{
    Caps K{};
    const uint64_t N = keys, T = P.base;
    K.keys = N;
    K.arrays = arrays;
    const uint64_t rate_n = (uint64_t)std::ceil(P.rate * (double)N);
    // round 0: one task and one global model per array of more than 2T keys
    K.tasks0 = std::min<uint64_t>(arrays, N / (2 * T + 1)) + 1;
    K.gsamples = std::min<uint64_t>(N, rate_n + K.tasks0);
    K.gblocks = K.gsamples / kSampleBlock + K.tasks0 + 1;
    K.gleafs = K.tasks0 * P.leaves;
    K.gmodels = K.tasks0 * model_doubles(P.leaves);
    K.gmax_sample = std::max<uint64_t>(1, P.cap ? std::min<uint64_t>(rate_n, P.cap) : rate_n);
    // a round: tasks are arrays or buckets of at least 2T keys; a task of n
    // keys has at most 66 + 128 n / T buckets (child_fanout) in at most
    // n / chunk + 1 chunks, with chunk >= keys / kTargetChunks; a local
    // sample takes ceil(rate n) or up to kLocalMinSample keys, and about one
    // leaf per 8 sample keys
    K.tasks = std::max<uint64_t>(K.tasks0, N / (2 * T) + 1);
    K.chunks = kTargetChunks + K.tasks;
    K.buckets = std::min<uint64_t>((uint64_t)P.fanout * K.tasks, 66 * K.tasks + 128 * N / T + 128);
    K.entries = (uint64_t)P.fanout * kTargetChunks + K.buckets;
    K.samples = std::min<uint64_t>(N, rate_n + (kLocalMinSample + 1) * K.tasks);
    K.blocks = K.samples / kSampleBlock + K.tasks + 1;
    K.leafs = std::min<uint64_t>((uint64_t)P.leaves * K.tasks, K.samples / 8 + K.tasks);
    K.models = 8 * K.leafs + 16 * K.tasks;
    K.max_sample = std::min<uint64_t>(N, std::max<uint64_t>(K.gmax_sample, kLocalMinSample));
    // lists: the per-round bounds of rounds_eager, over every round, plus
    // the small arrays of round 0
    const uint64_t fill_min = std::max<uint64_t>(P.base / 8, 2);
    const uint64_t g0 =
        std::min<uint64_t>(K.buckets, 3 * (N / group_window(P.base)) + N / fill_min + 2 * K.tasks + 2) + 1;
    K.groups[0] = arrays + kGraphMaxRounds * g0;
    K.groups[1] = arrays + kGraphMaxRounds * (N / (kGroupClassCap[0] + 1) + 1);
    K.groups[2] = arrays + kGraphMaxRounds * (N / (kGroupClassCap[1] + 1) + 1);
    K.fills = kGraphMaxRounds * (std::min<uint64_t>(K.buckets, N / fill_min) + N / kFillPiece + 1);
    const uint64_t ga[kGroupClasses] = {arrays, arrays, arrays};
    K.stage = stage_layout(K.tasks0, K.tasks0, ga);
    return K;
}

bool same_params(const Params& a, const Params& b)
{
    return a.fanout == b.fanout && a.leaves == b.leaves && a.tile == b.tile && a.base == b.base &&
           a.flags == b.flags && a.rate == b.rate && a.cap == b.cap && a.seed == b.seed;
}

// Size every buffer the replay touches for the class.
ls_status size_for_graph(ls_ctx* C, const Caps& K, hipStream_t st)
{
    TRY(ensure(C, C->scratch, K.keys * 8, st));
    TRY(ensure(C, C->ctl, sizeof(RoundCtl), st));
    TRY(ensure(C, C->next, K.tasks * sizeof(Task), st));
    TRY(ensure(C, C->tasks, K.tasks * sizeof(Task), st));
    TRY(ensure(C, C->gjobs, K.tasks0 * sizeof(ModelJob), st));
    TRY(ensure(C, C->ljobs, K.tasks * sizeof(ModelJob), st));
    TRY(ensure(C, C->models, (K.gmodels + K.models) * sizeof(double), st));
    TRY(ensure(C, C->sample, std::max(K.gsamples, K.samples) * 8, st));
    TRY(ensure(C, C->sample2, std::max(K.gsamples, K.samples) * 8, st));
    DevBuf* tabs[3] = {&C->tbest, &C->tfirst, &C->tnf};
    const size_t need[3] = {std::max(K.gleafs, K.leafs) * 8, std::max(K.gleafs, K.leafs) * 8,
                            std::max(K.tasks0, K.tasks) * 16};
    for (int i = 0; i < 3; ++i) {
        const void* before = tabs[i]->p;
        TRY(ensure(C, *tabs[i], need[i], st));
        if (tabs[i]->p != before)
            HIPCHECK(C, hipMemsetAsync(tabs[i]->p, 0, tabs[i]->cap, st));
    }
    TRY(ensure(C, C->cnt, K.entries * 4, st));
    TRY(ensure(C, C->pos, K.entries * 8, st));
    TRY(ensure(C, C->scantmp, scan_tmp_entries(K.entries) * 8, st));
    TRY(ensure(C, C->bstat, K.buckets * 16, st));
    TRY(ensure(C, C->skip, K.buckets, st));
    TRY(ensure(C, C->tflags, K.tasks * 4, st));
    for (uint32_t c = 0; c < kGroupClasses; ++c)
        TRY(ensure(C, C->groups[c], K.groups[c] * sizeof(Group), st));
    TRY(ensure(C, C->fills, K.fills * sizeof(Fill), st));
    TRY(ensure_pinned(C, C->gstage, K.stage.bytes, st));
    return LS_OK;
}

LayoutParams graph_layout_params(ls_ctx* C, const Caps& K, const Params& P)
{
    LayoutParams lp = layout_params(P, K.gmodels);
    lp.tile_wide = 0;   // the captured scatter launch has one tile
    lp.cap_tasks = K.tasks;
    lp.cap_fills = C->fills.cap / sizeof(Fill);
    for (uint32_t c = 0; c < kGroupClasses; ++c)
        lp.cap_groups[c] = C->groups[c].cap / sizeof(Group);
    lp.cap_keys = K.keys;
    lp.cap_chunks = K.chunks;
    lp.cap_buckets = K.buckets;
    lp.cap_entries = K.entries;
    lp.cap_samples = K.samples;
    lp.cap_blocks = K.blocks;
    lp.cap_leafs = K.leafs;
    lp.cap_models = K.models;
    return lp;
}

// The launches of one replay, recorded on the capture stream.
ls_status record_graph(ls_ctx* C, const Caps& K, const Params& P, uint32_t rounds, hipStream_t cs)
{
    RoundCtl* ctl = (RoundCtl*)C->ctl.p;
    const LiveCounts* live = &ctl->cur;
    HIPCHECK(C, launch_upload(upload_plan(C, C->gstage, K.stage), cs));
    uint64_t* sample = (uint64_t*)C->sample.p;
    uint64_t* sample2 = (uint64_t*)C->sample2.p;
    uint64_t* tbest = (uint64_t*)C->tbest.p;
    uint64_t* tfirst = (uint64_t*)C->tfirst.p;
    uint64_t* tnf = (uint64_t*)C->tnf.p;
    double* models = (double*)C->models.p;
    // global models: the host put their counts in ctl->cur
    HIPCHECK(C, launch_train((const ModelJob*)C->gjobs.p, (uint32_t)K.tasks0, (uint32_t)K.gblocks, K.gsamples,
                             K.gmax_sample, sample, sample2, tbest, tfirst, tnf, models, live, cs));
    const LayoutParams lp = graph_layout_params(C, K, P);
    HIPCHECK(C, launch_layout((Task*)C->next.p, (ModelJob*)C->ljobs.p, lp, ctl, C->d_h_ctl, cs));
    Task* lists[2] = {(Task*)C->next.p, (Task*)C->tasks.p};
    GroupLists gl;
    for (uint32_t c = 0; c < kGroupClasses; ++c)
        gl.g[c] = (Group*)C->groups[c].p;
    const uint32_t flags = P.flags & LS_FLAG_NONMONOTONE;
    for (uint32_t r = 0; r < rounds; ++r) {
        Task* in = lists[r & 1];
        Task* out = lists[(r + 1) & 1];
        const uint32_t nt = (uint32_t)(r == 0 ? K.tasks0 : K.tasks);
        HIPCHECK(C, launch_round_init((uint64_t*)C->bstat.p, K.buckets, ctl, true, cs));
        // local models: the tasks of the first two rounds use the arrays'
        // global models (levels 0 and 1 of Alg. 2), later ones their own
        if (r >= 2)
            HIPCHECK(C, launch_train((const ModelJob*)C->ljobs.p, (uint32_t)K.tasks, (uint32_t)K.blocks,
                                     K.samples, K.max_sample, sample, sample2, tbest, tfirst, tnf, models, live,
                                     cs));
        HIPCHECK(C, launch_hist(in, nt, (uint32_t)K.chunks, 0, models, (uint32_t*)C->cnt.p, (uint64_t*)C->bstat.p,
                                P.fanout, P.leaves, flags, live, cs));
        HIPCHECK(C, launch_scan((const uint32_t*)C->cnt.p, (uint64_t*)C->pos.p, K.entries, (uint64_t*)C->scantmp.p,
                                live, cs));
        HIPCHECK(C, launch_classify(in, nt, (const uint64_t*)C->pos.p, (const uint64_t*)C->bstat.p, P.base,
                                    P.fanout, out, gl, (Fill*)C->fills.p, (uint8_t*)C->skip.p,
                                    (uint32_t*)C->tflags.p, ctl, P.fanout, (ModelJob*)C->ljobs.p, lp, C->d_h_ctl,
                                    live, cs));
        HIPCHECK(C, launch_scatter(in, nt, (uint32_t)K.chunks, 0, models, (const uint64_t*)C->pos.p,
                                   (const uint8_t*)C->skip.p, (const uint32_t*)C->tflags.p, P.tile, P.fanout, P.leaves,
                                   flags, live, cs));
    }
    uint32_t gmax[kGroupClasses];
    for (uint32_t c = 0; c < kGroupClasses; ++c)
        gmax[c] = (uint32_t)std::min<uint64_t>(lp.cap_groups[c], 0xffffffffu);
    const uint32_t fmax = (uint32_t)std::min<uint64_t>(lp.cap_fills, 0xffffffffu);
    TRY(launch_finish_lists(C, gl, gmax, (const Fill*)C->fills.p, fmax, ctl, cs));
    HIPCHECK(C, launch_touchup(gl, gmax, (const Fill*)C->fills.p, fmax, 0, ctl, true, cs));
    HIPCHECK(C, hipMemcpyAsync(C->h_ctl, ctl, sizeof(RoundCtl), hipMemcpyDeviceToHost, cs));
    return LS_OK;
}

ls_status capture_graph(ls_ctx* C, const Caps& K, const Params& P, uint32_t rounds, hipGraphExec_t* out)
{
    if (!C->cap_stream)
        HIPCHECK(C, hipStreamCreateWithFlags(&C->cap_stream, hipStreamNonBlocking));
    hipStream_t cs = C->cap_stream;
    GateCapture gate;
    HIPCHECK(C, hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed));
    ls_status rc = record_graph(C, K, P, rounds, cs);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(cs, &g);
    if (rc == LS_OK && e != hipSuccess)
        rc = fail(C, LS_ERR_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    if (rc == LS_OK) {
        const hipError_t ei = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
        if (ei != hipSuccess)
            rc = fail(C, LS_ERR_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(ei));
    }
    if (g)
        (void)hipGraphDestroy(g);
    return rc;
}

void drop_graphs(ls_ctx* C, bool all)
{
    for (size_t i = 0; i < C->graphs.size();) {
        if (all || C->graphs[i].gen != C->gen) {
            (void)hipGraphExecDestroy(C->graphs[i].exec);
            C->graphs[i] = C->graphs.back();
            C->graphs.pop_back();
        } else {
            ++i;
        }
    }
}

bool graph_eligible(uint64_t total, size_t narrays, const Params& P)
{
    return (P.flags & LS_FLAG_GRAPH) && !(P.flags & (LS_FLAG_PROFILE | LS_FLAG_DEBUG_TOUCHUP | LS_FLAG_INPLACE)) &&
           total > 0 &&
           total <= kGraphMaxKeys && narrays <= kGraphMaxArrays;
}

// One batch as a replay of its class's graph (captured on first use).
ls_status run_graph(ls_ctx* C, std::vector<Array>& arrays, hipStream_t st, const Params& P, Batch& B)
{
    const uint64_t ckeys = std::max(pow2_ge(B.total), kGraphMinKeys);
    const uint64_t carrays = std::max(pow2_ge(arrays.size()), kGraphMinArrays);
    const Caps K = graph_caps(ckeys, carrays, P);
    if (B.tasks.size() > K.tasks0 || B.tr.samples > K.gsamples || B.tr.blocks > K.gblocks ||
        B.tr.max_sample > K.gmax_sample || B.tr.leaves > K.gleafs || B.tr.models > K.gmodels)
        return fail(C, LS_ERR_HIP, "batch exceeds the bounds of its graph class");
    // rounds in the replay: none without a round-0 task, else as many as
    // the class's last batch needed
    RoundsHint* H = nullptr;
    for (auto& h : C->hints)
        if (h.keys == ckeys && h.arrays == carrays && same_params(h.P, P))
            H = &h;
    const uint32_t rounds = B.tasks.empty() ? 0u : (H ? H->rounds : kGraphFirstRounds);
    GraphEntry* G = nullptr;
    for (auto& e : C->graphs)
        if (e.keys == ckeys && e.arrays == carrays && e.rounds == rounds && e.gen == C->gen && same_params(e.P, P))
            G = &e;
    if (!G) {
        TRY(size_for_graph(C, K, st));
        drop_graphs(C, false);
        void* lists[2] = {C->next.p, C->tasks.p};
        GraphEntry e{ckeys, carrays, C->gen, P, rounds, nullptr, lists[rounds & 1]};
        TRY(capture_graph(C, K, P, rounds, &e.exec));
        C->graphs.push_back(e);
        G = &C->graphs.back();
    }
    // the replay's upload kernel reads the staging area
    fill_stage((unsigned char*)C->gstage.p, K.stage, B);
    HIPCHECK(C, hipGraphLaunch(G->exec, st));
    HIPCHECK(C, hipStreamSynchronize(st));
    TRY(check_overflow(C));
    // Host-driven rounds swap the two task lists without reallocating them,
    // so since the capture they may have traded places: the continuation
    // expects the replay's last next-round list in C->next.
    if (C->next.p != G->list_final) {
        if (C->tasks.p != G->list_final)
            return fail(C, LS_ERR_HIP, "graph task lists out of step with the context");
        std::swap(C->tasks, C->next);
    }
    if (C->h_ctl->ntasks) {
        // more rounds than the replay holds: continue from its state
        Prof prof{C, st, false, {}};
        TRY(rounds_eager(C, st, P, layout_params(P, K.gmodels), P.flags & LS_FLAG_NONMONOTONE, prof));
        TRY(finish_eager(C, st, P, prof, B.group0_keys));
    }
    if (!B.tasks.empty()) {
        const uint32_t need = std::min(std::max<uint32_t>(C->h_ctl->rounds, 1), kGraphMaxRounds);
        if (H)
            H->rounds = need;
        else
            C->hints.push_back(RoundsHint{ckeys, carrays, P, need});
    }
    return LS_OK;
}

// ---------------------------------------------------- no-allocation sorts --
//
// ls_sort_noalloc runs the host-driven pipeline with every device buffer of
// the context pointed into this device's static array instead of grown by
// ensure().  The buffers are cut from bounds that hold for any input of n
// keys: the per-round tables from the same bounds as a graph class of n keys
// (one round's tasks, buckets, count-matrix entries, samples, leaves and
// models), the lists that grow over the rounds from the fact that they
// describe disjoint key ranges (a group holds at least one key, a group of
// class c > 0 more than the previous class cap, an all-equal bucket at least
// max(T/8, 2) keys and one piece per kFillPiece keys).  The layout and
// classify kernels check every capacity on the device, so a bound that did
// not hold would end the sort with an error, never write past a buffer.

// The context's device buffers, in one list (save, carve, restore, free).
constexpr size_t kCtxBufs = 32;
std::array<DevBuf*, kCtxBufs> ctx_bufs(ls_ctx* C)
{
    return {&C->scratch, &C->tune, &C->models, &C->sample, &C->sample2, &C->tbest, &C->tfirst,
            &C->tnf, &C->gjobs, &C->ljobs, &C->tasks, &C->next, &C->cnt, &C->pos, &C->scantmp, &C->bstat,
            &C->skip, &C->tflags, &C->fills, &C->ctl, &C->groups[0], &C->groups[1], &C->groups[2],
            &C->pcnt, &C->ppos, &C->ipb, &C->fullb, &C->ovf, &C->tags, &C->done, &C->sidebuf, &C->bidx};
}

struct Carve {
    DevBuf* b;
    size_t bytes;
};

// Buffers of a no-allocation sort of n keys with parameters P, and the
// total of their 256-byte aligned sizes.
std::vector<Carve> noalloc_plan(ls_ctx* C, uint64_t n, const Params& P, size_t* total)
{
    const Caps K = graph_caps(n, 1, P);
    const uint64_t fill_min = std::max<uint64_t>(P.base / 8, 2);
    const uint64_t samples = std::max(K.gsamples, K.samples);
    const uint64_t leafs = std::max(K.gleafs, K.leafs);
    const uint64_t tasks = std::max(K.tasks0, K.tasks);
    std::vector<Carve> v = {
        {&C->scratch, n * 8},
        {&C->ctl, sizeof(RoundCtl)},
        {&C->tasks, tasks * sizeof(Task)},
        {&C->next, tasks * sizeof(Task)},
        {&C->gjobs, K.tasks0 * sizeof(ModelJob)},
        {&C->ljobs, tasks * sizeof(ModelJob)},
        {&C->models, (K.gmodels + K.models) * sizeof(double)},
        {&C->sample, samples * 8},
        {&C->sample2, samples * 8},
        {&C->tbest, leafs * 8},
        {&C->tfirst, leafs * 8},
        {&C->tnf, tasks * 16},
        {&C->cnt, K.entries * 4},
        {&C->pos, K.entries * 8},
        {&C->scantmp, scan_tmp_entries(K.entries) * 8},
        {&C->bstat, K.buckets * 16},
        {&C->skip, K.buckets},
        {&C->tflags, tasks * 4},
        {&C->groups[0], (n + 1) * sizeof(Group)},
        {&C->groups[1], (n / (kGroupClassCap[0] + 1) + 1) * sizeof(Group)},
        {&C->groups[2], (n / (kGroupClassCap[1] + 1) + 1) * sizeof(Group)},
        {&C->fills, (n / fill_min + n / kFillPiece + 2) * sizeof(Fill)},
    };
    size_t off = 0;
    for (auto& c : v)
        off += (std::max<size_t>(c.bytes, 8) + 255) & ~(size_t)255;
    *total = off;
    return v;
}

// Capacities of the carved buffers, for the device-side checks.
LayoutParams noalloc_layout_params(ls_ctx* C, const Params& P, uint64_t model_base)
{
    LayoutParams lp = layout_params(P, model_base);
    lp.cap_tasks = std::min({C->next.cap / sizeof(Task), C->tasks.cap / sizeof(Task), C->ljobs.cap / sizeof(ModelJob),
                             C->tflags.cap / 4, C->tnf.cap / 16});
    lp.cap_fills = C->fills.cap / sizeof(Fill);
    for (uint32_t c = 0; c < kGroupClasses; ++c)
        lp.cap_groups[c] = C->groups[c].cap / sizeof(Group);
    lp.cap_keys = C->scratch.cap / 8;
    lp.cap_buckets = std::min(C->bstat.cap / 16, C->skip.cap);
    lp.cap_entries = std::min(C->cnt.cap / 4, C->pos.cap / 8);
    lp.cap_samples = std::min(C->sample.cap, C->sample2.cap) / 8;
    lp.cap_leafs = std::min(C->tbest.cap, C->tfirst.cap) / 8;
    const uint64_t pool = C->models.cap / sizeof(double);
    lp.cap_models = pool > model_base ? pool - model_base : 0;
    return lp;
}

// The whole pipeline for a batch of arrays.  msd_only: partition on the
// order-preserving bits alone (the touch-up repair path).
ls_status run_pipeline(ls_ctx* C, std::vector<Array>& arrays, hipStream_t st, const Params& P, bool msd_only)
{
    Batch B;
    uint64_t total = 0;
    for (auto& a : arrays)
        total += a.n;
    if (!msd_only && graph_eligible(total, arrays.size(), P)) {
        // the scratch buffer at the class size (the replay's sizing keeps it)
        TRY(ensure(C, C->scratch, std::max(pow2_ge(total), kGraphMinKeys) * 8, st));
        prepare(arrays, C->scratch.p, P, false, B);
        TRY(run_graph(C, arrays, st, P, B));
        return conclude(C, arrays, st, P, msd_only);
    }
    if (!(P.flags & LS_FLAG_INPLACE))
        TRY(ensure(C, C->scratch, std::max<uint64_t>(total, 1) * 8, st));
    TRY(ensure(C, C->ctl, sizeof(RoundCtl), st));
    prepare(arrays, C->scratch.p, P, msd_only, B);
    const uint64_t global_models = B.tr.models;
    Prof prof{C, st, (P.flags & LS_FLAG_PROFILE) != 0, {}};
    prof.only = (int)((P.flags >> 8) & 0xfu) - 1;

    // round-0 lists: staged in mapped host memory, copied by one kernel
    const uint64_t ng0[kGroupClasses] = {B.groups0[0].size(), B.groups0[1].size(), B.groups0[2].size()};
    const StageLayout SL = stage_layout(B.tasks.size(), B.tr.jobs.size(), ng0);
    for (uint32_t c = 0; c < kGroupClasses; ++c)
        TRY(ensure(C, C->groups[c], std::max<size_t>(B.groups0[c].size(), 1) * sizeof(Group), st));
    TRY(ensure(C, C->next, std::max<size_t>(B.tasks.size(), 1) * sizeof(Task), st));
    TRY(ensure(C, C->ljobs, std::max<size_t>(B.tasks.size(), 1) * sizeof(ModelJob), st));
    TRY(ensure(C, C->gjobs, std::max<size_t>(B.tr.jobs.size(), 1) * sizeof(ModelJob), st));
    TRY(ensure_pinned(C, C->estage, SL.bytes, st));
    fill_stage((unsigned char*)C->estage.p, SL, B);
    HIPCHECK(C, launch_upload(upload_plan(C, C->estage, SL), st));
    if (!B.tr.jobs.empty())
        TRY(train(C, C->gjobs, (uint32_t)B.tr.jobs.size(), B.tr.blocks, B.tr.samples, B.tr.leaves,
                  B.tr.max_sample, 0, B.tr.models, st, &prof));
    const LayoutParams lp = C->no_alloc ? noalloc_layout_params(C, P, global_models) : layout_params(P, global_models);
    if (!B.tasks.empty()) {
        LayoutParams lp0 = lp;
        lp0.host_flag = C->d_h_flag;
        arm_publish(C);
        HIPCHECK(C, launch_layout((Task*)C->next.p, (ModelJob*)C->ljobs.p, lp0, (RoundCtl*)C->ctl.p, C->d_h_ctl,
                                  st));
        TRY(wait_published(C, st));
    } else {
        TRY(read_ctl(C, st));
    }
    const uint32_t flags = msd_only ? 0u : (P.flags & LS_FLAG_NONMONOTONE);
    TRY(rounds_eager(C, st, P, lp, flags, prof));
    TRY(finish_eager(C, st, P, prof, B.group0_keys));
    return conclude(C, arrays, st, P, msd_only);
}

// Record the end of a sort's work on the caller's stream.
void mark_done(ls_ctx* C, hipStream_t st)
{
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (!C->ev_done || hipStreamIsCapturing(st, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone ||
        hipEventRecord(C->ev_done, st) != hipSuccess) {
        (void)hipGetLastError();
        return;
    }
    C->done_pending = true;
}

// Wait until the context's queued work (its last sort, its own streams) ends.
ls_status wait_ctx(ls_ctx* C)
{
    if (C->done_pending)
        HIPCHECK(C, hipEventSynchronize(C->ev_done));
    C->done_pending = false;
    if (C->cap_stream)
        HIPCHECK(C, hipStreamSynchronize(C->cap_stream));
    return LS_OK;
}

ls_status run_pipeline_marked(ls_ctx* C, std::vector<Array>& arrays, hipStream_t st, const Params& P,
                              bool msd_only)
{
    const ls_status s = run_pipeline(C, arrays, st, P, msd_only);
    mark_done(C, st);
    return s;
}

// A batch of segments described on the device: round 0 is prepared by a
// kernel from the device offsets (no host walk of the segments); the rest is
// the host-driven pipeline.  Two small reads: the total (to size the
// scratch) and round 0's counts.
ls_status run_segments_device(ls_ctx* C, uint64_t* keys, const uint64_t* d_off, uint64_t nseg,
                              const uint8_t* d_dtypes, uint32_t dtype, hipStream_t st, const Params& P)
{
    const bool inplace = (P.flags & LS_FLAG_INPLACE) != 0;
    uint64_t total = 0;
    if (nseg) {
        HIPCHECK(C, hipMemcpyAsync(&total, d_off + nseg, 8, hipMemcpyDeviceToHost, st));
        HIPCHECK(C, hipStreamSynchronize(st));
    }
    if (total && !keys)
        return fail(C, LS_ERR_INVALID, "null key pointer with keys to sort");
    if (!inplace)
        TRY(ensure(C, C->scratch, std::max<uint64_t>(total, 1) * 8, st));
    const size_t slots = std::max<uint64_t>(nseg, 1);
    TRY(ensure(C, C->ctl, sizeof(RoundCtl), st));
    TRY(ensure(C, C->next, slots * sizeof(Task), st));
    TRY(ensure(C, C->ljobs, slots * sizeof(ModelJob), st));
    TRY(ensure(C, C->gjobs, slots * sizeof(ModelJob), st));
    for (uint32_t c = 0; c < kGroupClasses; ++c)
        TRY(ensure(C, C->groups[c], slots * sizeof(Group), st));
    TRY(ensure(C, C->skip, kSegSummary * 8, st));
    SegPrepare A{};
    A.keys = keys;
    A.scratch = inplace ? nullptr : (uint64_t*)C->scratch.p;
    A.off = d_off;
    A.dtypes = d_dtypes;
    A.nseg = nseg;
    A.dtype = dtype;
    A.base = P.base;
    A.fanout = P.fanout;
    A.leaves = P.leaves;
    A.inplace = inplace ? 1u : 0u;
    A.rate = P.rate;
    A.cap = P.cap;
    A.seed = P.seed;
    A.tasks = (Task*)C->next.p;
    A.jobs = (ModelJob*)C->gjobs.p;
    for (uint32_t c = 0; c < kGroupClasses; ++c)
        A.groups[c] = (Group*)C->groups[c].p;
    A.ctl = (RoundCtl*)C->ctl.p;
    A.summary = (uint64_t*)C->skip.p;
    HIPCHECK(C, launch_seg_prepare(A, st));
    uint64_t sum[kSegSummary] = {};
    HIPCHECK(C, hipMemcpyAsync(sum, C->skip.p, sizeof sum, hipMemcpyDeviceToHost, st));
    TRY(read_ctl(C, st));
    if (sum[3])
        return fail(C, LS_ERR_INVALID, "offsets must start at 0 and be non-decreasing");
    const RoundCtl c0 = *C->h_ctl;
    Prof prof{C, st, (P.flags & LS_FLAG_PROFILE) != 0, {}};
    prof.only = (int)((P.flags >> 8) & 0xfu) - 1;
    if (c0.cur.njobs)
        TRY(train(C, C->gjobs, c0.cur.njobs, c0.cur.blocks, c0.cur.samples, sum[1], c0.cur.max_sample, 0, sum[2],
                  st, &prof));
    const LayoutParams lp = layout_params(P, sum[2]);
    if (c0.ntasks) {
        LayoutParams lp0 = lp;
        lp0.host_flag = C->d_h_flag;
        arm_publish(C);
        HIPCHECK(C, launch_layout((Task*)C->next.p, (ModelJob*)C->ljobs.p, lp0, (RoundCtl*)C->ctl.p, C->d_h_ctl,
                                  st));
        TRY(wait_published(C, st));
    }
    TRY(rounds_eager(C, st, P, lp, P.flags & LS_FLAG_NONMONOTONE, prof));
    TRY(finish_eager(C, st, P, prof, sum[0]));
    std::vector<Array> arrays;
    if (C->h_ctl->violations) {
        // the touch-up repair pass needs the segments on the host
        std::vector<uint64_t> off(nseg + 1);
        std::vector<uint8_t> dts(nseg, (uint8_t)dtype);
        HIPCHECK(C, hipMemcpyAsync(off.data(), d_off, off.size() * 8, hipMemcpyDeviceToHost, st));
        if (d_dtypes)
            HIPCHECK(C, hipMemcpyAsync(dts.data(), d_dtypes, nseg, hipMemcpyDeviceToHost, st));
        HIPCHECK(C, hipStreamSynchronize(st));
        for (uint64_t i = 0; i < nseg; ++i)
            arrays.push_back(Array{keys + off[i], nullptr, off[i + 1] - off[i], dts[i]});
    }
    return conclude(C, arrays, st, P, false);
}

ls_status sort_arrays(ls_ctx* C, std::vector<Array>& arrays, hipStream_t st, const ls_params* p)
{
    GateUse gate;
    Params P;
    TRY(resolve(C, p, P));
    for (auto& a : arrays) {
        if (a.n && !a.keys)
            return fail(C, LS_ERR_INVALID, "null key pointer with n > 0");
        if (a.dtype != LS_F64 && a.dtype != LS_U64)
            return fail(C, LS_ERR_INVALID, "unknown dtype");
        if (((uintptr_t)a.keys) & 7u)
            return fail(C, LS_ERR_INVALID, "key buffer must be 8-byte aligned");
    }
    HIPCHECK(C, hipSetDevice(C->device));
    C->dev_status = 0;
    std::memset(C->stats, 0, sizeof C->stats);
    return run_pipeline_marked(C, arrays, st, P, false);
}

}  // namespace

extern "C" {

void ls_default_params(ls_params* p)
{
    if (!p)
        return;
    std::memset(p, 0, sizeof *p);
    p->struct_size = sizeof(ls_params);
    p->fanout = kDefaultFanout;
    p->leaves = kDefaultLeaves;
    p->tile = 0;   // automatic
    p->base_threshold = kDefaultBase;
    p->sample_rate = 0.01;
    p->seed = kDefaultSeed;
    p->sample_cap = kDefaultSampleCap;
}

ls_status ls_create(ls_ctx** out, int device)
{
    GateUse gate;
    if (!out)
        return LS_ERR_INVALID;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count)
        return LS_ERR_INVALID;
    if (hipSetDevice(device) != hipSuccess)
        return LS_ERR_HIP;
    ls_ctx* C = new (std::nothrow) ls_ctx();
    if (!C)
        return LS_ERR_NOMEM;
    C->device = device;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess)
        C->lds_limit = prop.sharedMemPerBlock;
    if (hipHostMalloc((void**)&C->h_ctl, sizeof(RoundCtl), hipHostMallocMapped | hipHostMallocCoherent) !=
            hipSuccess ||
        hipHostGetDevicePointer((void**)&C->d_h_ctl, C->h_ctl, 0) != hipSuccess ||
        hipHostMalloc((void**)&C->h_flag, sizeof(uint64_t), hipHostMallocMapped | hipHostMallocCoherent) !=
            hipSuccess ||
        hipHostGetDevicePointer((void**)&C->d_h_flag, C->h_flag, 0) != hipSuccess) {
        if (C->h_ctl)
            (void)hipHostFree(C->h_ctl);
        if (C->h_flag)
            (void)hipHostFree(C->h_flag);
        delete C;
        return LS_ERR_NOMEM;
    }
    *C->h_flag = 0;
    // the no-allocation sort's static array on this device (the device is
    // current), and pinned staging for its round-0 lists
    if (noalloc_setup(device, &C->na_base, &C->na_bytes) != hipSuccess ||
        hipEventCreateWithFlags(&C->ev_done, hipEventDisableTiming) != hipSuccess ||
        ensure_pinned(C, C->estage, 65536, nullptr) != LS_OK) {
        (void)hipGetLastError();
        (void)hipHostFree(C->h_ctl);
        (void)hipHostFree(C->h_flag);
        if (C->estage.p)
            (void)hipHostFree(C->estage.p);
        if (C->ev_done)
            (void)hipEventDestroy(C->ev_done);
        delete C;
        return LS_ERR_HIP;
    }
    *out = C;
    return LS_OK;
}

ls_status ls_destroy(ls_ctx* C)
{
    GateUse gate;
    if (!C)
        return LS_ERR_INVALID;
    (void)hipSetDevice(C->device);
    (void)wait_ctx(C);
    (void)hipGetLastError();
    for (DevBuf* b : ctx_bufs(C))
        if (b->p)
            (void)hipFree(b->p);
    PinBuf* pins[] = {&C->pin_jobs, &C->estage, &C->gstage};
    for (PinBuf* b : pins)
        if (b->p)
            (void)hipHostFree(b->p);
    if (C->h_ctl)
        (void)hipHostFree(C->h_ctl);
    if (C->h_flag)
        (void)hipHostFree(C->h_flag);
    for (hipEvent_t e : C->ev_pool)
        (void)hipEventDestroy(e);
    drop_graphs(C, true);
    if (C->cap_stream)
        (void)hipStreamDestroy(C->cap_stream);
    if (C->ev_done)
        (void)hipEventDestroy(C->ev_done);
    delete C;
    return LS_OK;
}

ls_status ls_workspace_size(ls_ctx* C, ls_dtype dtype, size_t n, const ls_params* p, size_t* bytes)
{
    if (!bytes || (dtype != LS_F64 && dtype != LS_U64))
        return LS_ERR_INVALID;
    ls_ctx scratch_ctx;                 // parameter checks only (no HIP call, no LDS limit)
    scratch_ctx.lds_limit = ~(size_t)0 >> 1;
    Params P;
    TRY(resolve(C ? C : &scratch_ctx, p, P));
    size_t chunks = kTargetChunks + 64;
    size_t tables = (size_t)P.fanout * chunks * 12 + (size_t)P.fanout * 64 + model_doubles(P.leaves) * 8 * 4;
    size_t lists = (n / 2 + P.fanout) * (sizeof(Group) + sizeof(Fill)) / 8;
    // scratch keys (in place: side buffer, overflow blocks, tags and flags,
    // each a small fraction of the keys), round tables, output lists,
    // training sample
    const size_t keys = (P.flags & LS_FLAG_INPLACE) ? n : n * 8;
    *bytes = keys + tables + lists + (2 * std::min<size_t>(n / 50 + 4096, kDefaultSampleCap + 4096)) * 8;
    return LS_OK;
}

ls_status ls_reserve(ls_ctx* C, size_t n, const ls_params* p)
{
    GateUse gate;
    if (!C)
        return LS_ERR_INVALID;
    Params P;
    TRY(resolve(C, p, P));
    HIPCHECK(C, hipSetDevice(C->device));
    return ensure(C, C->scratch, std::max<size_t>(n, 1) * 8, nullptr);
}

ls_status ls_device_bytes(ls_ctx* C, size_t* bytes)
{
    if (!C || !bytes)
        return LS_ERR_INVALID;
    size_t s = 0;
    for (DevBuf* b : ctx_bufs(C))
        if (b->p)
            s += b->cap;
    *bytes = s;
    return LS_OK;
}

ls_status ls_trim(ls_ctx* C)
{
    GateUse gate;
    if (!C)
        return LS_ERR_INVALID;
    HIPCHECK(C, hipSetDevice(C->device));
    TRY(wait_ctx(C));
    drop_graphs(C, true);
    for (DevBuf* b : ctx_bufs(C)) {
        if (b->p)
            HIPCHECK(C, hipFree(b->p));
        b->p = nullptr;
        b->cap = 0;
    }
    ++C->gen;
    return LS_OK;
}

ls_status ls_sort_f64(ls_ctx* C, double* d_keys, size_t n, ls_stream_t stream, const ls_params* p)
{
    if (!C)
        return LS_ERR_INVALID;
    std::vector<Array> a{Array{(uint64_t*)d_keys, nullptr, n, LS_F64}};
    return sort_arrays(C, a, (hipStream_t)stream, p);
}

ls_status ls_sort_u64(ls_ctx* C, uint64_t* d_keys, size_t n, ls_stream_t stream, const ls_params* p)
{
    if (!C)
        return LS_ERR_INVALID;
    std::vector<Array> a{Array{d_keys, nullptr, n, LS_U64}};
    return sort_arrays(C, a, (hipStream_t)stream, p);
}

ls_status ls_sort_noalloc(ls_ctx* C, ls_dtype dtype, void* d_keys, size_t n, ls_stream_t stream,
                          const ls_params* p)
{
    GateUse gate;
    if (!C)
        return LS_ERR_INVALID;
    if (dtype != LS_F64 && dtype != LS_U64)
        return fail(C, LS_ERR_INVALID, "unknown dtype");
    if (n && !d_keys)
        return fail(C, LS_ERR_INVALID, "null key pointer with n > 0");
    if (((uintptr_t)d_keys) & 7u)
        return fail(C, LS_ERR_INVALID, "key buffer must be 8-byte aligned");
    if (n > LS_NOALLOC_MAX_KEYS)
        return fail(C, LS_ERR_UNSUPPORTED, "ls_sort_noalloc sorts at most " + std::to_string(LS_NOALLOC_MAX_KEYS) +
                                               " keys; got " + std::to_string(n));
    Params P;
    TRY(resolve(C, p, P));
    if (P.flags & (LS_FLAG_PROFILE | LS_FLAG_GRAPH | LS_FLAG_INPLACE))
        return fail(C, LS_ERR_UNSUPPORTED,
                    "ls_sort_noalloc takes none of LS_FLAG_PROFILE, LS_FLAG_GRAPH, LS_FLAG_INPLACE");
    if (!C->na_base)
        return fail(C, LS_ERR_HIP, "the no-allocation array of this device was not found");
    size_t need = 0;
    const std::vector<Carve> plan = noalloc_plan(C, n, P, &need);
    if (need > C->na_bytes)
        return fail(C, LS_ERR_UNSUPPORTED, "these parameters need " + std::to_string(need) +
                                               " bytes of scratch for " + std::to_string(n) + " keys; the static array "
                                               "holds " + std::to_string(C->na_bytes));
    HIPCHECK(C, hipSetDevice(C->device));
    C->dev_status = 0;
    std::memset(C->stats, 0, sizeof C->stats);
    if (n <= 1)
        return LS_OK;
    hipStream_t st = (hipStream_t)stream;
    // point every buffer of the context into the array; put them back after
    std::array<DevBuf, kCtxBufs> saved;
    const auto bufs = ctx_bufs(C);
    for (size_t i = 0; i < kCtxBufs; ++i) {
        saved[i] = *bufs[i];
        *bufs[i] = DevBuf{};
    }
    unsigned char* base = (unsigned char*)C->na_base;
    size_t off = 0;
    for (const Carve& c : plan) {
        const size_t sz = (std::max<size_t>(c.bytes, 8) + 255) & ~(size_t)255;
        c.b->p = base + off;
        c.b->cap = sz;
        off += sz;
    }
    C->no_alloc = true;
    std::vector<Array> a{Array{(uint64_t*)d_keys, nullptr, n, (uint32_t)dtype}};
    // the training tables must start at zero (the array keeps whatever the
    // last call on this device left there)
    ls_status rc = LS_OK;
    for (DevBuf* t : {&C->tbest, &C->tfirst, &C->tnf})
        if (rc == LS_OK && launch_zero(t->p, t->cap, st) != hipSuccess)
            rc = fail(C, LS_ERR_HIP, "clearing the training tables failed");
    if (rc == LS_OK)
        rc = run_pipeline_marked(C, a, st, P, false);
    C->no_alloc = false;
    for (size_t i = 0; i < kCtxBufs; ++i)
        *bufs[i] = saved[i];
    return rc;
}

ls_status ls_sort_segments(ls_ctx* C, ls_dtype dtype, void* d_keys, const uint64_t* h_offsets,
                           size_t num_segments, const uint8_t* h_dtypes, ls_stream_t stream,
                           const ls_params* p)
{
    if (!C)
        return LS_ERR_INVALID;
    if (num_segments && !h_offsets)
        return fail(C, LS_ERR_INVALID, "null offsets");
    if (num_segments && h_offsets[0] != 0)
        return fail(C, LS_ERR_INVALID, "offsets[0] must be 0");
    std::vector<Array> a;
    a.reserve(num_segments);
    for (size_t i = 0; i < num_segments; ++i) {
        if (h_offsets[i + 1] < h_offsets[i])
            return fail(C, LS_ERR_INVALID, "offsets must be non-decreasing");
        uint32_t dt = h_dtypes ? h_dtypes[i] : (uint32_t)dtype;
        uint64_t n = h_offsets[i + 1] - h_offsets[i];
        if (n && !d_keys)
            return fail(C, LS_ERR_INVALID, "null key pointer with keys to sort");
        a.push_back(Array{(uint64_t*)d_keys + h_offsets[i], nullptr, n, dt});
    }
    return sort_arrays(C, a, (hipStream_t)stream, p);
}

ls_status ls_sort_ls1(ls_ctx* C, ls_dtype dtype, void* d_keys, size_t n, double slack, ls_stream_t stream,
                      const ls_params* p, double* out8)
{
    GateUse gate;
    if (!C)
        return LS_ERR_INVALID;
    if ((dtype != LS_F64 && dtype != LS_U64) || (n && !d_keys) || !(slack >= 0.0) || slack > 64.0)
        return fail(C, LS_ERR_INVALID, "ls_sort_ls1: dtype, keys or slack (0..64) invalid");
    if (((uintptr_t)d_keys) & 7u)
        return fail(C, LS_ERR_INVALID, "key buffer must be 8-byte aligned");
    Params P;
    TRY(resolve(C, p, P));
    P.flags &= ~(uint32_t)(LS_FLAG_GRAPH | LS_FLAG_INPLACE | LS_FLAG_PROFILE);
    HIPCHECK(C, hipSetDevice(C->device));
    C->dev_status = 0;
    std::memset(C->stats, 0, sizeof C->stats);
    if (out8)
        std::fill(out8, out8 + 8, 0.0);
    if (n <= 1)
        return LS_OK;
    hipStream_t st = (hipStream_t)stream;
    const uint32_t f = P.fanout, L = P.leaves;
    if (ls1_scatter_lds_bytes(f, L) > C->lds_limit)
        return fail(C, LS_ERR_UNSUPPORTED, "ls_sort_ls1: fanout and leaves exceed the LDS of one workgroup");
    const uint64_t cap = std::max<uint64_t>(1, (uint64_t)std::ceil((double)n * (1.0 + slack) / (double)f));
    hipEvent_t ev[5] = {};
    for (auto& e : ev)
        HIPCHECK(C, hipEventCreate(&e));
    struct EvFree {
        hipEvent_t* e;
        ~EvFree()
        {
            for (int i = 0; i < 5; ++i)
                if (e[i])
                    (void)hipEventDestroy(e[i]);
        }
    } evfree{ev};
    HIPCHECK(C, hipEventRecord(ev[0], st));
    // 1. the global model (Sec. 2), 2. bucket counts per chunk and their scan
    Trainer tr;
    tr.add((const uint64_t*)d_keys, n, sample_size(n, P.rate, P.cap), P.seed, L, dtype);
    TRY(ensure(C, C->gjobs, sizeof(ModelJob), st));
    TRY(upload(C, C->pin_jobs, C->gjobs, tr.jobs, st));
    TRY(train(C, C->gjobs, 1, tr.blocks, tr.samples, tr.leaves, tr.max_sample, 0, tr.models, st, nullptr));
    const uint64_t chunk = std::max<uint64_t>(
        kLs1Tile * 4ull, ((n + kTargetChunks - 1) / kTargetChunks + kLs1Tile - 1) / kLs1Tile * kLs1Tile);
    Task t{};
    t.keys = (uint64_t*)d_keys;
    t.n = n;
    t.scale = (double)f;
    t.fanout = f;
    t.kind = kGlobal;
    t.dtype = dtype;
    t.leaves = L;
    t.nchunks = (uint32_t)((n + chunk - 1) / chunk);
    const uint64_t entries = (uint64_t)f * t.nchunks;
    TRY(ensure(C, C->tasks, sizeof(Task), st));
    TRY(ensure(C, C->ctl, sizeof(RoundCtl), st));
    TRY(ensure(C, C->cnt, entries * 4, st));
    TRY(ensure(C, C->pos, entries * 8, st));
    TRY(ensure(C, C->pcnt, entries * 4, st));
    TRY(ensure(C, C->ppos, entries * 8, st));
    TRY(ensure(C, C->scantmp, scan_tmp_entries(entries) * 8, st));
    TRY(ensure(C, C->bstat, (size_t)f * 16, st));
    TRY(ensure(C, C->fullb, ((size_t)f + 2) * 8, st));
    HIPCHECK(C, hipMemcpyAsync(C->tasks.p, &t, sizeof(Task), hipMemcpyHostToDevice, st));
    HIPCHECK(C, launch_round_init((uint64_t*)C->bstat.p, f, (RoundCtl*)C->ctl.p, false, st));
    HIPCHECK(C, launch_hist((const Task*)C->tasks.p, 1, t.nchunks, chunk, (const double*)C->models.p,
                            (uint32_t*)C->cnt.p, (uint64_t*)C->bstat.p, f, L, 0, nullptr, st));
    HIPCHECK(C, launch_scan((const uint32_t*)C->cnt.p, (uint64_t*)C->pos.p, entries, (uint64_t*)C->scantmp.p,
                            nullptr, st));
    // 3. what spills from each (bucket, chunk) entry, and where it goes
    HIPCHECK(C, launch_ls1_spill_counts((const uint64_t*)C->pos.p, (const uint32_t*)C->cnt.p, entries, t.nchunks,
                                        cap, (uint32_t*)C->pcnt.p, st));
    HIPCHECK(C, launch_scan((const uint32_t*)C->pcnt.p, (uint64_t*)C->ppos.p, entries, (uint64_t*)C->scantmp.p,
                            nullptr, st));
    HIPCHECK(C, launch_ls1_buckets((const uint64_t*)C->pos.p, (const uint64_t*)C->ppos.p,
                                   (const uint32_t*)C->pcnt.p, f, t.nchunks, n, (uint64_t*)C->fullb.p, st));
    std::vector<uint64_t> bt((size_t)f + 2);
    HIPCHECK(C, hipMemcpyAsync(bt.data(), C->fullb.p, bt.size() * 8, hipMemcpyDeviceToHost, st));
    HIPCHECK(C, hipStreamSynchronize(st));
    const uint64_t nspill = bt[f + 1], nkept = n - nspill;
    // 4. the ablation's own area: bucket slots, spill, sorted spill, packed
    // buckets, merged run, library temp
    size_t tb_sort = 0, tb_merge = 0;
    HIPCHECK(C, ls1_radix_sort(nullptr, &tb_sort, nullptr, nullptr, nspill, st));
    HIPCHECK(C, ls1_merge(nullptr, &tb_merge, nullptr, nkept, nullptr, nspill, nullptr, st));
    const uint64_t slots_n = (uint64_t)f * cap;
    const size_t temp = (std::max(tb_sort, tb_merge) + 255) & ~(size_t)255;
    TRY(ensure(C, C->tune, (slots_n + 2 * nspill + nkept + n) * 8 + temp, st));
    uint64_t* slots = (uint64_t*)C->tune.p;
    uint64_t* spill = slots + slots_n;
    uint64_t* sorted = spill + nspill;
    uint64_t* packed = sorted + nspill;
    uint64_t* merged = packed + nkept;
    void* tmp = merged + n;
    HIPCHECK(C, launch_scatter_ls1((const Task*)C->tasks.p, t.nchunks, chunk, (const double*)C->models.p,
                                   (const uint64_t*)C->pos.p, (const uint64_t*)C->ppos.p, cap, slots, spill, f, L,
                                   st));
    HIPCHECK(C, hipEventRecord(ev[1], st));
    // 5. each bucket sorted (the library's pipeline, buckets as segments)
    std::vector<Array> arrays;
    std::vector<uint64_t> fill((size_t)f + 1, 0);
    arrays.reserve(f);
    for (uint32_t b = 0; b < f; ++b) {
        const uint64_t m = std::min<uint64_t>(bt[b + 1] - bt[b], cap);
        fill[b + 1] = fill[b] + m;
        arrays.push_back(Array{slots + (uint64_t)b * cap, nullptr, m, (uint32_t)dtype});
    }
    TRY(run_pipeline(C, arrays, st, P, false));
    HIPCHECK(C, hipEventRecord(ev[2], st));
    // 6. the spill area sorted
    if (nspill)
        HIPCHECK(C, ls1_radix_sort(tmp, &tb_sort, spill, sorted, nspill, st));
    HIPCHECK(C, hipEventRecord(ev[3], st));
    // 7. buckets packed, merged with the spill area, converted back
    TRY(ensure(C, C->fullb, ((size_t)f + 2) * 8, st));
    HIPCHECK(C, hipMemcpyAsync(C->fullb.p, fill.data(), fill.size() * 8, hipMemcpyHostToDevice, st));
    HIPCHECK(C, launch_ls1_compact(slots, (const uint64_t*)C->fullb.p, cap, f, dtype, packed, st));
    HIPCHECK(C, ls1_merge(tmp, &tb_merge, packed, nkept, sorted, nspill, merged, st));
    HIPCHECK(C, launch_from_ord(merged, n, dtype, (uint64_t*)d_keys, st));
    HIPCHECK(C, hipEventRecord(ev[4], st));
    HIPCHECK(C, hipEventSynchronize(ev[4]));
    if (out8) {
        out8[0] = (double)nspill;
        out8[1] = (double)cap;
        for (int i = 0; i < 4; ++i) {
            float ms = 0.f;
            HIPCHECK(C, hipEventElapsedTime(&ms, ev[i], ev[i + 1]));
            out8[2 + i] = ms;
        }
        float all = 0.f;
        HIPCHECK(C, hipEventElapsedTime(&all, ev[0], ev[4]));
        out8[6] = all;
        out8[7] = (double)f;
    }
    return LS_OK;
}

ls_status ls_sort_segments_device(ls_ctx* C, ls_dtype dtype, void* d_keys, const uint64_t* d_offsets,
                                  size_t num_segments, const uint8_t* d_dtypes, ls_stream_t stream,
                                  const ls_params* p)
{
    GateUse gate;
    if (!C)
        return LS_ERR_INVALID;
    if (num_segments && !d_offsets)
        return fail(C, LS_ERR_INVALID, "null offsets");
    if (!d_dtypes && dtype != LS_F64 && dtype != LS_U64)
        return fail(C, LS_ERR_INVALID, "unknown dtype");
    if (((uintptr_t)d_keys) & 7u)
        return fail(C, LS_ERR_INVALID, "key buffer must be 8-byte aligned");
    Params P;
    TRY(resolve(C, p, P));
    P.flags &= ~(uint32_t)LS_FLAG_GRAPH;      // host-driven rounds only
    HIPCHECK(C, hipSetDevice(C->device));
    C->dev_status = 0;
    std::memset(C->stats, 0, sizeof C->stats);
    hipStream_t st = (hipStream_t)stream;
    const ls_status s = run_segments_device(C, (uint64_t*)d_keys, d_offsets, num_segments, d_dtypes,
                                            (uint32_t)dtype, st, P);
    mark_done(C, st);
    return s;
}

ls_status ls_sort_arrays(ls_ctx* C, const ls_array* h_arrays, size_t count, ls_stream_t stream,
                         const ls_params* p)
{
    if (!C)
        return LS_ERR_INVALID;
    if (count && !h_arrays)
        return fail(C, LS_ERR_INVALID, "null array list");
    std::vector<Array> a;
    a.reserve(count);
    for (size_t i = 0; i < count; ++i)
        a.push_back(Array{(uint64_t*)h_arrays[i].d_keys, nullptr, h_arrays[i].n, h_arrays[i].dtype});
    return sort_arrays(C, a, (hipStream_t)stream, p);
}

ls_status ls_autotune(ls_ctx* C, const ls_array* h_arrays, size_t count, ls_stream_t stream, const ls_params* base,
                      uint32_t reps, ls_params* best, ls_tune_result* results, size_t cap, size_t* n_results)
{
    GateUse gate;
    if (!C || !best || (count && !h_arrays))
        return LS_ERR_INVALID;
    ls_params bp;
    if (base) {
        if (base->struct_size != sizeof(ls_params))
            return fail(C, LS_ERR_INVALID, "ls_params.struct_size mismatch");
        bp = *base;
    } else {
        ls_default_params(&bp);
    }
    Params P0;
    TRY(resolve(C, &bp, P0));
    uint64_t total = 0;
    for (size_t i = 0; i < count; ++i) {
        if (h_arrays[i].n && !h_arrays[i].d_keys)
            return fail(C, LS_ERR_INVALID, "null key pointer with n > 0");
        if (h_arrays[i].dtype != LS_F64 && h_arrays[i].dtype != LS_U64)
            return fail(C, LS_ERR_INVALID, "unknown dtype");
        total += h_arrays[i].n;
    }
    reps = reps ? reps : 2;
    hipStream_t st = (hipStream_t)stream;
    HIPCHECK(C, hipSetDevice(C->device));
    TRY(ensure(C, C->tune, std::max<uint64_t>(total, 1) * 8, st));
    // the copies sit back to back in the tuning buffer; arrays that are
    // already back to back in the caller's memory are restored with one copy
    std::vector<ls_array> copies(count);
    std::vector<std::pair<size_t, size_t>> runs;  // [first, last) arrays contiguous in the source
    uint64_t off = 0;
    for (size_t i = 0; i < count; ++i) {
        copies[i] = h_arrays[i];
        copies[i].d_keys = (uint64_t*)C->tune.p + off;
        off += h_arrays[i].n;
        const bool joins = i > 0 && (const uint64_t*)h_arrays[i - 1].d_keys + h_arrays[i - 1].n ==
                                        (const uint64_t*)h_arrays[i].d_keys;
        if (joins)
            runs.back().second = i + 1;
        else
            runs.push_back({i, i + 1});
    }
    hipEvent_t e0, e1;
    HIPCHECK(C, hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(C, LS_ERR_HIP, "hipEventCreate failed");
    }
    static const uint32_t fanouts[] = {512, 1024, 2048, 4096};
    static const uint32_t tiles[] = {2048, 0};   // 0: automatic (4096, or 8192 in large rounds)
    static const uint32_t bases[] = {1024, 2048, 4096};
    size_t k = 0;
    double best_ms = -1.0;
    ls_status rc = LS_OK;
    for (uint32_t f : fanouts)
        for (uint32_t t : tiles)
            for (uint32_t b : bases) {
                ls_params cp = bp;
                cp.fanout = f;
                cp.tile = t;
                cp.base_threshold = b;
                cp.flags &= ~(LS_FLAG_PROFILE | LS_FLAG_SYNC);
                Params P;
                double ms = -1.0;
                if (resolve(C, &cp, P) == LS_OK) {
                    for (uint32_t r = 0; r < reps && rc == LS_OK; ++r) {
                        for (auto& run : runs) {
                            uint64_t n = 0;
                            for (size_t i = run.first; i < run.second; ++i)
                                n += h_arrays[i].n;
                            if (n && hipMemcpyAsync(copies[run.first].d_keys, h_arrays[run.first].d_keys, n * 8,
                                                    hipMemcpyDeviceToDevice, st) != hipSuccess)
                                rc = fail(C, LS_ERR_HIP, "copy for tuning failed");
                        }
                        std::vector<Array> a;
                        a.reserve(count);
                        for (auto& c : copies)
                            a.push_back(Array{(uint64_t*)c.d_keys, nullptr, c.n, c.dtype});
                        if (rc == LS_OK && hipEventRecord(e0, st) != hipSuccess)
                            rc = fail(C, LS_ERR_HIP, "hipEventRecord failed");
                        if (rc == LS_OK)
                            rc = sort_arrays(C, a, st, &cp);
                        float el = 0.f;
                        if (rc == LS_OK && (hipEventRecord(e1, st) != hipSuccess ||
                                            hipEventSynchronize(e1) != hipSuccess ||
                                            hipEventElapsedTime(&el, e0, e1) != hipSuccess))
                            rc = fail(C, LS_ERR_HIP, "timing failed");
                        if (rc == LS_OK && (ms < 0 || el < ms))
                            ms = el;
                    }
                }
                if (rc != LS_OK)
                    break;
                if (results && k < cap)
                    results[k] = ls_tune_result{f, t, b, 0, ms};
                ++k;
                if (ms >= 0 && (best_ms < 0 || ms < best_ms)) {
                    best_ms = ms;
                    *best = cp;
                    best->flags = bp.flags;
                }
            }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    TRY(rc);
    if (best_ms < 0)
        *best = bp;
    if (n_results)
        *n_results = k;
    return LS_OK;
}

ls_status ls_sync(ls_ctx* C, uint32_t* device_status)
{
    GateUse gate;
    if (!C)
        return LS_ERR_INVALID;
    HIPCHECK(C, hipSetDevice(C->device));
    TRY(wait_ctx(C));
    if (device_status)
        *device_status = C->dev_status;
    return LS_OK;
}

ls_status ls_last_stats(ls_ctx* C, uint64_t* out8)
{
    if (!C || !out8)
        return LS_ERR_INVALID;
    std::memcpy(out8, C->stats, sizeof C->stats);
    return LS_OK;
}

ls_status ls_last_profile(ls_ctx* C, double* out, size_t cap)
{
    if (!C || !out || cap < 24)
        return LS_ERR_INVALID;
    for (int k = 0; k < 8; ++k) {
        out[3 * k] = C->prof_ms[k];
        out[3 * k + 1] = C->prof_launch[k];
        out[3 * k + 2] = C->prof_bytes[k];
    }
    return LS_OK;
}

ls_status ls_profile_reset(ls_ctx* C)
{
    if (!C)
        return LS_ERR_INVALID;
    for (int k = 0; k < 8; ++k)
        C->prof_ms[k] = C->prof_launch[k] = C->prof_bytes[k] = 0;
    return LS_OK;
}

const char* ls_status_string(ls_status s)
{
    switch (s) {
    case LS_OK: return "ok";
    case LS_ERR_INVALID: return "invalid argument";
    case LS_ERR_NOMEM: return "out of memory";
    case LS_ERR_HIP: return "HIP runtime error";
    case LS_ERR_UNSUPPORTED: return "unsupported parameters";
    case LS_ERR_BUDGET: return "request exceeds the memory budget";
    case LS_ERR_TIMEOUT: return "timed out";
    case LS_ERR_NOTFOUND: return "unknown ticket";
    }
    return "unknown status";
}

const char* ls_last_error(ls_ctx* C)
{
    return C ? C->err.c_str() : "null context";
}

// ---------------------------------------------------------------- stage hooks

ls_status ls_model_train(ls_ctx* C, ls_dtype dtype, const void* d_keys, size_t n, const ls_params* p,
                         double* h_model_out, size_t cap)
{
    GateUse gate;
    if (!C || !d_keys || !n || !h_model_out || (dtype != LS_F64 && dtype != LS_U64))
        return LS_ERR_INVALID;
    Params P;
    TRY(resolve(C, p, P));
    const uint32_t L = P.leaves;
    if (cap < 4 + 7 * ((size_t)L + 1))
        return fail(C, LS_ERR_INVALID, "model output buffer too small");
    HIPCHECK(C, hipSetDevice(C->device));
    hipStream_t st = nullptr;
    Trainer tr;
    tr.add((const uint64_t*)d_keys, n, sample_size(n, P.rate, P.cap), P.seed, P.leaves, dtype);
    TRY(ensure(C, C->gjobs, sizeof(ModelJob), st));
    TRY(upload(C, C->pin_jobs, C->gjobs, tr.jobs, st));
    TRY(train(C, C->gjobs, 1, tr.blocks, tr.samples, tr.leaves, tr.max_sample, 0, tr.models, st, nullptr));
    HIPCHECK(C, hipStreamSynchronize(st));
    std::vector<double> dev(model_doubles(L));
    HIPCHECK(C, hipMemcpy(dev.data(), C->models.p, dev.size() * 8, hipMemcpyDeviceToHost));
    for (int i = 0; i < 4; ++i)
        h_model_out[i] = dev[i];
    for (uint32_t k = 0; k <= L; ++k) {
        double* o = h_model_out + 4 + 7 * (size_t)k;          // export knot: {X, y, ym, y1, ylo, yhi, s}
        const double* d = dev.data() + kModelSeg + 4 * (size_t)k;   // device knot: {X, ylo, s, yhi}
        o[0] = d[0];
        o[1] = dev[model_y_off(L) + k];
        o[2] = dev[model_ym_off(L) + k];
        o[3] = dev[model_y1_off(L) + k];
        o[4] = d[1];
        o[5] = d[3];
        o[6] = d[2];
    }
    return LS_OK;
}

ls_status ls_stage_hist(ls_ctx* C, ls_dtype dtype, const void* d_keys, size_t n, const double* h_model,
                        uint32_t leaves, double scale, int64_t offset, uint32_t fanout, uint64_t* h_counts,
                        uint64_t* h_min, uint64_t* h_max)
{
    GateUse gate;
    if (!C || !d_keys || !n || !h_model || !h_counts || (dtype != LS_F64 && dtype != LS_U64))
        return LS_ERR_INVALID;
    if (leaves < 1 || leaves > kMaxLeaves || fanout < 2 || fanout > kMaxFanout)
        return fail(C, LS_ERR_INVALID, "leaves or fanout out of range");
    HIPCHECK(C, hipSetDevice(C->device));
    hipStream_t st = nullptr;
    // model: export layout -> device layout with the previous-knot table
    std::vector<double> dev(model_doubles(leaves), 0.0);
    for (int i = 0; i < 4; ++i)
        dev[i] = h_model[i];
    uint32_t* prev = reinterpret_cast<uint32_t*>(dev.data() + model_prev_off(leaves));
    uint32_t last = kNoPrev;
    for (uint32_t k = 0; k <= leaves; ++k) {
        const double* o = h_model + 4 + 7 * (size_t)k;        // export knot: {X, y, ym, y1, ylo, yhi, s}
        double* d = dev.data() + kModelSeg + 4 * (size_t)k;   // device knot: {X, ylo, s, yhi}
        d[0] = o[0];
        d[1] = o[4];
        d[2] = o[6];
        d[3] = o[5];
        dev[model_ym_off(leaves) + k] = o[2];
        dev[model_y_off(leaves) + k] = o[1];
        dev[model_y1_off(leaves) + k] = o[3];
        if (k < leaves) {
            prev[k] = last;
            if (!std::isinf(o[0]))
                last = k;
        }
    }
    TRY(ensure(C, C->models, dev.size() * 8, st));
    TRY(ensure(C, C->ctl, sizeof(RoundCtl), st));
    HIPCHECK(C, hipMemcpy(C->models.p, dev.data(), dev.size() * 8, hipMemcpyHostToDevice));
    const uint32_t tile = kDefaultTile;
    uint64_t chunk = std::max<uint64_t>(tile * 4ull, ((n + kTargetChunks - 1) / kTargetChunks + tile - 1) / tile * tile);
    Task t{};
    t.keys = (uint64_t*)d_keys;
    t.n = n;
    t.scale = scale;
    t.offset = offset;
    t.fanout = fanout;
    t.kind = kGlobal;
    t.dtype = dtype;
    t.leaves = leaves;
    t.nchunks = (uint32_t)((n + chunk - 1) / chunk);
    TRY(ensure(C, C->tasks, sizeof(Task), st));
    TRY(ensure(C, C->cnt, (size_t)fanout * t.nchunks * 4, st));
    TRY(ensure(C, C->bstat, (size_t)fanout * 16, st));
    HIPCHECK(C, hipMemcpy(C->tasks.p, &t, sizeof(Task), hipMemcpyHostToDevice));
    HIPCHECK(C, launch_round_init((uint64_t*)C->bstat.p, fanout, (RoundCtl*)C->ctl.p, false, st));
    HIPCHECK(C, launch_hist((const Task*)C->tasks.p, 1, t.nchunks, chunk, (const double*)C->models.p,
                            (uint32_t*)C->cnt.p, (uint64_t*)C->bstat.p, fanout, leaves, 0, nullptr, st));
    HIPCHECK(C, hipDeviceSynchronize());
    std::vector<uint32_t> cnt((size_t)fanout * t.nchunks);
    std::vector<uint64_t> bs((size_t)fanout * 2);
    HIPCHECK(C, hipMemcpy(cnt.data(), C->cnt.p, cnt.size() * 4, hipMemcpyDeviceToHost));
    HIPCHECK(C, hipMemcpy(bs.data(), C->bstat.p, bs.size() * 8, hipMemcpyDeviceToHost));
    for (uint32_t b = 0; b < fanout; ++b) {
        uint64_t s = 0;
        for (uint32_t c = 0; c < t.nchunks; ++c)
            s += cnt[(size_t)b * t.nchunks + c];
        h_counts[b] = s;
        if (h_min) h_min[b] = bs[2 * b];
        if (h_max) h_max[b] = bs[2 * b + 1];
    }
    return LS_OK;
}

}  // extern "C"
