// Continuous-batching sort server (ls_server_* in include/lsort.h).
//
// Requests (device buffers, sorted in place) wait in a FIFO queue.  Each of
// `max_inflight` workers owns a library context and a HIP stream; when free
// it admits queued requests in arrival order while the accounted device
// memory stays within the budget, and sorts them as one batch.  The account
// holds the keys of the requests being sorted, what each idle worker's
// context keeps (it reuses its buffers from batch to batch), and for a busy
// worker that plus a bound on what its batch can add.  A worker whose own
// kept buffers stand in the way of the oldest request frees them first.  A
// batch's keys are capped relative to its oldest request, so a small request
// does not wait for a large one batched with it; a request over the cap stays
// queued for a later batch.  Requests that arrive while other batches run are
// picked up by the next free worker, so batches overlap on the GPU; while
// few requests wait, a request large enough to fill the device runs beside
// small batches only, not beside another large one.  The
// admission stops at the first request the budget cannot hold, and a request
// is only passed by later arrivals until it is the oldest, so none is
// overtaken indefinitely.
#include "lsort.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <numeric>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

namespace {

using Clock = std::chrono::steady_clock;

struct Request {
    uint64_t ticket;
    ls_dtype dtype;
    void* keys;
    uint64_t n;
    Clock::time_point submitted;
};

struct Done {
    ls_status status;
    double latency_s;
};

// A batch holds at most min(limit, max(kBatchFloorKeys, kBatchGrowth x its
// first request's keys)) keys, or its first request alone: batching pays for
// many small (launch-bound) requests, while a small request batched with a
// large one waits for the large one.  The limit is kLatencyBatchKeys, or
// kBacklogBatchKeys while more than kBacklog requests wait (then large
// batches keep the device full and raise throughput).
constexpr uint64_t kLatencyBatchKeys = 1ull << 25;
constexpr uint64_t kBacklogBatchKeys = 1ull << 29;
constexpr size_t kBacklog = 8;
constexpr uint64_t kBatchFloorKeys = 1ull << 22;
constexpr uint64_t kBatchGrowth = 4;
// Fixed part of a batch's bound (models, control blocks, smallest buffers).
constexpr uint64_t kBoundFloor = 8ull << 20;
// While at most kBacklog requests wait, a request of at least this many keys
// (one that fills the device by itself) runs in no batch beside another
// such batch: two of them side by side would each take about twice as long,
// which is the latency of the largest requests, while small requests still
// run beside it.
constexpr uint64_t kLargeRequestKeys = 1ull << 23;

}  // namespace

struct ls_server {
    int device = 0;
    uint64_t budget = 0;
    ls_params params{};
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Request> queue;
    std::unordered_map<uint64_t, Done> done;
    std::unordered_map<uint64_t, bool> pending;
    uint64_t next_ticket = 1;
    uint64_t keys_bytes = 0;           // keys of the requests being sorted
    uint32_t large_running = 0;        // batches running with a request of >= kLargeRequestKeys
    std::vector<uint64_t> held;        // per worker: its context's buffers (+ its batch's bound while busy)
    uint64_t peak = 0;
    uint64_t n_submitted = 0, n_completed = 0, n_batches = 0;
    bool stopping = false;
    std::vector<std::thread> workers;
    std::string last_error;   // message of the latest failed batch
};

namespace {

// Bound on the device memory a batch of `keys` keys can add to a context:
// every buffer grows to at most 1.5 x what the batch needs (a buffer grows
// by at least half of itself), plus the fixed part.
uint64_t batch_bound(const ls_server* S, uint64_t keys)
{
    size_t need = 0;
    if (ls_workspace_size(nullptr, LS_F64, keys, &S->params, &need) != LS_OK)
        need = keys * 8;
    return need + need / 2 + kBoundFloor;
}

uint64_t accounted(const ls_server* S)
{
    return S->keys_bytes + std::accumulate(S->held.begin(), S->held.end(), (uint64_t)0);
}

// Whether worker w can sort `keys` more keys now, with `own` bytes kept by
// its context (the caller holds the lock).
bool fits(const ls_server* S, uint32_t w, uint64_t keys, uint64_t own)
{
    const uint64_t others = accounted(S) - S->held[w];
    return others + own + keys * 8 + batch_bound(S, keys) <= S->budget;
}

// Whether request r may be admitted now as far as the large-request rule is
// concerned (the caller holds the lock).
bool may_run(const ls_server* S, const Request& r)
{
    return S->queue.size() > kBacklog || S->large_running == 0 || r.n < kLargeRequestKeys;
}

// The oldest request a batch may start with now, or nullptr.
const Request* lead(const ls_server* S)
{
    for (const Request& r : S->queue)
        if (may_run(S, r))
            return &r;
    return nullptr;
}

void worker_main(ls_server* S, uint32_t w)
{
    ls_ctx* ctx = nullptr;
    hipStream_t st = nullptr;
    bool ok = hipSetDevice(S->device) == hipSuccess && ls_create(&ctx, S->device) == LS_OK &&
              hipStreamCreateWithFlags(&st, hipStreamNonBlocking) == hipSuccess;
    std::vector<Request> batch;
    std::vector<ls_array> arrays;
    for (;;) {
        batch.clear();
        uint64_t keys = 0;
        bool trim = false, has_large = false;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            // wake to sort the oldest request, or to free this context's
            // buffers when they alone keep it out
            S->cv_work.wait(lk, [&] {
                if (S->queue.empty())
                    return S->stopping;
                const Request* r = lead(S);
                if (!r)
                    return false;   // only large requests wait, behind a large batch
                return fits(S, w, r->n, S->held[w]) || (S->held[w] > 0 && fits(S, w, r->n, 0));
            });
            if (S->queue.empty())
                break;
            const Request* first = lead(S);
            if (!fits(S, w, first->n, S->held[w])) {
                trim = true;
            } else {
                // The oldest request that may run leads; later ones join while
                // they fit the batch's key cap, and admission stops at the
                // first request the memory budget cannot hold.  A request
                // skipped for the cap or the large-request rule is only ever
                // passed by later arrivals until it leads a batch (a large one
                // waits at most for the large batch running).
                const uint64_t limit = S->queue.size() > kBacklog ? kBacklogBatchKeys : kLatencyBatchKeys;
                const uint64_t cap = std::min(limit, std::max(kBatchFloorKeys, kBatchGrowth * first->n));
                // (the first request is admitted whatever its size)
                std::deque<Request> keep;   // what stays queued, in order
                bool stop = false, large = false;
                for (const Request& r : S->queue) {
                    if (stop || !may_run(S, r)) {
                        keep.push_back(r);
                        continue;
                    }
                    if (!fits(S, w, keys + r.n, S->held[w])) {
                        stop = true;
                        keep.push_back(r);
                        continue;
                    }
                    if (!batch.empty() && keys + r.n > cap) {
                        keep.push_back(r);
                        continue;
                    }
                    keys += r.n;
                    large |= r.n >= kLargeRequestKeys;
                    batch.push_back(r);
                }
                S->queue.swap(keep);
                has_large = large;
                S->large_running += large ? 1u : 0u;
                S->keys_bytes += keys * 8;
                S->held[w] += batch_bound(S, keys);
                S->peak = std::max(S->peak, accounted(S));
                S->n_batches++;
            }
        }
        if (trim) {
            size_t b = 0;
            if (ctx && (ls_trim(ctx) != LS_OK || ls_device_bytes(ctx, &b) != LS_OK))
                b = 0;
            {
                std::lock_guard<std::mutex> lk(S->mu);
                S->held[w] = b;
            }
            S->cv_work.notify_all();
            continue;
        }
        ls_status status = ok ? LS_OK : LS_ERR_HIP;
        if (ok) {
            arrays.clear();
            for (auto& r : batch)
                arrays.push_back(ls_array{r.keys, r.n, (uint32_t)r.dtype, 0});
            status = ls_sort_arrays(ctx, arrays.data(), arrays.size(), (ls_stream_t)st,
                                    &S->params);
            if (status == LS_OK && hipStreamSynchronize(st) != hipSuccess)
                status = LS_ERR_HIP;
            if (status != LS_OK && batch.size() > 1) {
                // isolate the failure: retry each request on its own
                for (auto& r : batch) {
                    ls_array one{r.keys, r.n, (uint32_t)r.dtype, 0};
                    ls_status s1 = ls_sort_arrays(ctx, &one, 1, (ls_stream_t)st,
                                                  &S->params);
                    if (s1 == LS_OK)
                        s1 = hipStreamSynchronize(st) == hipSuccess ? LS_OK : LS_ERR_HIP;
                    r.n = (uint64_t)s1;     // reuse the field to carry the status below
                }
            }
        }
        size_t kept = 0;
        if (ok && ls_device_bytes(ctx, &kept) != LS_OK)
            kept = 0;
        const auto now = Clock::now();
        {
            std::lock_guard<std::mutex> lk(S->mu);
            if (status != LS_OK)
                S->last_error = ok ? ls_last_error(ctx) : "worker start-up failed (context or stream creation)";
            for (auto& r : batch) {
                ls_status s = status;
                if (status != LS_OK && batch.size() > 1)
                    s = (ls_status)r.n;
                S->done[r.ticket] = Done{s, std::chrono::duration<double>(now - r.submitted).count()};
                S->pending.erase(r.ticket);
                S->n_completed++;
            }
            S->keys_bytes -= keys * 8;
            S->large_running -= has_large ? 1u : 0u;
            // what the context keeps from now on (a bound that was too low
            // shows here, and the next admissions count it)
            S->held[w] = kept;
            S->peak = std::max(S->peak, accounted(S));
        }
        S->cv_done.notify_all();
        S->cv_work.notify_all();
    }
    if (st)
        (void)hipStreamDestroy(st);
    if (ctx)
        ls_destroy(ctx);
}

}  // namespace

extern "C" {

ls_status ls_server_create(ls_server** out, int device, size_t hbm_budget_bytes, uint32_t max_inflight,
                           const ls_params* p)
{
    if (!out || hbm_budget_bytes == 0 || max_inflight == 0 || max_inflight > 16)
        return LS_ERR_INVALID;
    if (p && p->struct_size != sizeof(ls_params))
        return LS_ERR_INVALID;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count)
        return LS_ERR_INVALID;
    ls_server* S = new (std::nothrow) ls_server();
    if (!S)
        return LS_ERR_NOMEM;
    S->device = device;
    S->budget = hbm_budget_bytes;
    if (p)
        S->params = *p;
    else
        ls_default_params(&S->params);
    size_t probe = 0;
    if (ls_workspace_size(nullptr, LS_F64, 1, &S->params, &probe) != LS_OK) {
        delete S;
        return LS_ERR_INVALID;
    }
    S->held.assign(max_inflight, 0);
    for (uint32_t i = 0; i < max_inflight; ++i)
        S->workers.emplace_back(worker_main, S, i);
    *out = S;
    return LS_OK;
}

ls_status ls_server_submit(ls_server* S, ls_dtype dtype, void* d_keys, size_t n, uint64_t* ticket)
{
    if (!S || !ticket || (dtype != LS_F64 && dtype != LS_U64) || (n && !d_keys))
        return LS_ERR_INVALID;
    if ((uint64_t)n * 8 + batch_bound(S, n) > S->budget)
        return LS_ERR_BUDGET;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        if (S->stopping)
            return LS_ERR_INVALID;
        *ticket = S->next_ticket++;
        S->queue.push_back(Request{*ticket, dtype, d_keys, (uint64_t)n, Clock::now()});
        S->pending[*ticket] = true;
        S->n_submitted++;
    }
    S->cv_work.notify_one();
    return LS_OK;
}

ls_status ls_server_wait(ls_server* S, uint64_t ticket, int timeout_ms, double* latency_s)
{
    if (!S)
        return LS_ERR_INVALID;
    std::unique_lock<std::mutex> lk(S->mu);
    auto ready = [&] { return S->done.count(ticket) > 0; };
    if (!ready() && !S->pending.count(ticket))
        return LS_ERR_NOTFOUND;
    if (timeout_ms < 0)
        S->cv_done.wait(lk, ready);
    else if (!S->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), ready))
        return LS_ERR_TIMEOUT;
    Done d = S->done[ticket];
    S->done.erase(ticket);
    if (latency_s)
        *latency_s = d.latency_s;
    return d.status;
}

ls_status ls_server_stats(ls_server* S, uint64_t* out6)
{
    if (!S || !out6)
        return LS_ERR_INVALID;
    std::lock_guard<std::mutex> lk(S->mu);
    out6[0] = S->n_submitted;
    out6[1] = S->n_completed;
    out6[2] = S->n_batches;
    out6[3] = S->peak;
    out6[4] = accounted(S);
    out6[5] = S->queue.size();
    return LS_OK;
}

ls_status ls_server_last_error(ls_server* S, char* buf, size_t cap)
{
    if (!S || !buf || !cap)
        return LS_ERR_INVALID;
    std::lock_guard<std::mutex> lk(S->mu);
    const size_t n = std::min(cap - 1, S->last_error.size());
    std::memcpy(buf, S->last_error.data(), n);
    buf[n] = 0;
    return LS_OK;
}

ls_status ls_server_destroy(ls_server* S)
{
    if (!S)
        return LS_ERR_INVALID;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stopping = true;
    }
    S->cv_work.notify_all();
    for (auto& t : S->workers)
        t.join();
    delete S;
    return LS_OK;
}

}  // extern "C"
