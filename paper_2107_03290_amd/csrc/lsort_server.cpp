// Continuous-batching sort server (ls_server_* in include/lsort.h).
//
// Requests (device buffers, sorted in place) wait in a FIFO queue.  Each of
// `max_inflight` workers owns a library context and a HIP stream; when free
// it admits queued requests in arrival order while the bytes they occupy on
// the device (keys + the scratch the sort needs) stay within the budget, and
// sorts them as one batch.  A batch's keys are capped relative to its oldest
// request, so a small request does not wait for a large one batched with it;
// a request over the cap stays queued for a later batch.  Requests that
// arrive while other batches run are picked up by the next free worker, so
// batches overlap on the GPU.  The admission stops at the first request the
// budget cannot hold, and a request is only passed by later arrivals until it
// is the oldest, so none is overtaken indefinitely.
#include "lsort.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
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

constexpr uint64_t kBytesPerKey = 16;             // the keys plus their scratch
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
    uint64_t admitted = 0, peak = 0;
    uint64_t n_submitted = 0, n_completed = 0, n_batches = 0;
    bool stopping = false;
    std::vector<std::thread> workers;
    ls_status fatal = LS_OK;
    std::string last_error;   // message of the latest failed batch
};

namespace {

void worker_main(ls_server* S)
{
    ls_ctx* ctx = nullptr;
    hipStream_t st = nullptr;
    bool ok = hipSetDevice(S->device) == hipSuccess && ls_create(&ctx, S->device) == LS_OK &&
              hipStreamCreateWithFlags(&st, hipStreamNonBlocking) == hipSuccess;
    std::vector<Request> batch;
    std::vector<ls_array> arrays;
    for (;;) {
        batch.clear();
        uint64_t bytes = 0;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            S->cv_work.wait(lk, [&] {
                if (S->stopping && S->queue.empty())
                    return true;
                if (S->queue.empty())
                    return false;
                return S->admitted + S->queue.front().n * kBytesPerKey <= S->budget;
            });
            if (S->queue.empty())
                break;
            // The oldest request leads; later ones join while they fit the
            // batch's key cap, and admission stops at the first request the
            // memory budget cannot hold.  A request skipped for the cap is
            // only ever passed by later arrivals until it leads a batch.
            const uint64_t limit = S->queue.size() > kBacklog ? kBacklogBatchKeys : kLatencyBatchKeys;
            const uint64_t cap = std::min(limit, std::max(kBatchFloorKeys, kBatchGrowth * S->queue.front().n));
            // (the first request is admitted whatever its size)
            uint64_t keys = 0;
            std::deque<Request> rest;
            while (!S->queue.empty()) {
                Request r = S->queue.front();
                const uint64_t b = r.n * kBytesPerKey;
                if (S->admitted + b > S->budget)
                    break;
                S->queue.pop_front();
                if (!batch.empty() && keys + r.n > cap) {
                    rest.push_back(r);
                    continue;
                }
                S->admitted += b;
                bytes += b;
                keys += r.n;
                batch.push_back(r);
            }
            // skipped requests go back in front, in their order
            while (!rest.empty()) {
                S->queue.push_front(rest.back());
                rest.pop_back();
            }
            S->peak = S->admitted > S->peak ? S->admitted : S->peak;
            S->n_batches++;
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
            S->admitted -= bytes;
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
    for (uint32_t i = 0; i < max_inflight; ++i)
        S->workers.emplace_back(worker_main, S);
    *out = S;
    return LS_OK;
}

ls_status ls_server_submit(ls_server* S, ls_dtype dtype, void* d_keys, size_t n, uint64_t* ticket)
{
    if (!S || !ticket || (dtype != LS_F64 && dtype != LS_U64) || (n && !d_keys))
        return LS_ERR_INVALID;
    if ((uint64_t)n * kBytesPerKey > S->budget)
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
    out6[4] = S->admitted;
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
