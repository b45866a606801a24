// server.cpp -- a continuous-batching sort server over the batched sort.
//
// Requests (a device input array, a device output array, a key count and a
// key type) arrive at any time.  A worker thread keeps up to `slots` batches
// in flight, each on its own stream with its own workspace: whenever a slot
// is free it admits waiting requests in arrival order while their memory
// footprint fits the budget, packs them into one batched launch per key type
// and records a completion event; finished batches are retired by polling
// those events, which frees their share of the budget for the next
// admissions.  Requests that arrive while a batch runs join the next batch,
// and with two slots two batches overlap on the device.  max_batch = 1 and
// slots = 1 turn the server into the plain path: one request per launch, in
// arrival order.
//
// Footprint of a request of n keys of w bytes: its input and output arrays
// (2 w n) plus its share of a batch workspace (w n of scratch keys and the
// per-tile bookkeeping, bounded here by w n + 64 bytes per 16 keys).

#include <hip/hip_runtime.h>

#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "intsort.h"
#include "internal.hpp"
#include "sort_plans.hpp"

namespace {

using clk = std::chrono::steady_clock;

struct Req {
    int kt;
    const void *in;
    void *out;
    uint64_t n;
    uint64_t bytes;
    clk::time_point t_submit, t_done;
    int state;   // 0 waiting, 1 running, 2 done, 3 failed
    bool listed, polled;   // a failed request is forgotten once both calls have reported it
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    void *ws = nullptr;
    size_t ws_bytes = 0;
    intsort_segment_desc *h_desc = nullptr;   // pinned, 2 * max_batch
    intsort_segment_desc *d_desc = nullptr;
    std::vector<uint64_t> tickets;
    bool busy = false;
};

uint64_t footprint(int kt, uint64_t n)
{
    const uint64_t w = kt == INTSORT_U64 ? 8 : 4;
    return 3 * w * n + 4 * n + 4096;
}

}  // namespace

struct intsort_server {
    intsort_ctx *ctx = nullptr;   // the server's own context
    int device = 0;
    uint64_t budget = 0, in_flight = 0;
    uint32_t max_batch = 1;
    uint64_t max_batch_keys = 0;
    std::vector<Slot> slots;
    std::mutex mu;
    std::condition_variable cv, idle;
    std::deque<uint64_t> queue;
    std::unordered_map<uint64_t, Req> reqs;
    std::vector<uint64_t> completed;
    uint64_t next_ticket = 1;
    uint64_t outstanding = 0;     // submitted and not done
    bool stop = false;
    uint64_t failed_since_drain = 0;   // requests that failed since the last intsort_server_drain
    uint32_t inject_failures = 0;      // batch launches still to fail on purpose
    std::thread worker;

    void run();
    bool launch(Slot &slot, const std::vector<Req> &batch);
    void finish(const std::vector<uint64_t> &tickets, bool ok);
};

// marks the requests of one batch finished (done or failed); called with the lock held
void intsort_server::finish(const std::vector<uint64_t> &tickets, bool ok)
{
    const clk::time_point now = clk::now();
    for (uint64_t t : tickets) {
        Req &r = reqs.at(t);
        r.state = ok ? 2 : 3;
        r.t_done = now;
        in_flight -= r.bytes;
        completed.push_back(t);
        outstanding--;
        if (!ok) failed_since_drain++;
    }
}

// runs without the lock: it sees only copies of the requests
bool intsort_server::launch(Slot &slot, const std::vector<Req> &batch)
{
    // split the batch by key type: u32 arrays first, u64 arrays after
    uint32_t a = 0, b = 0;
    uint64_t keys32 = 0, keys64 = 0;
    for (const Req &r : batch) {
        intsort_segment_desc d{r.in, r.out, r.n};
        if (r.kt == INTSORT_U32) {
            slot.h_desc[a++] = d;
            keys32 += r.n;
        } else {
            slot.h_desc[max_batch + b++] = d;
            keys64 += r.n;
        }
    }
    if (hipMemcpyAsync(slot.d_desc, slot.h_desc, sizeof(intsort_segment_desc) * 2 * max_batch,
                       hipMemcpyHostToDevice, slot.stream) != hipSuccess)
        return false;
    if (a && intsort_batched_sort_keys(ctx, INTSORT_U32, slot.d_desc, a, keys32, nullptr, slot.ws, slot.ws_bytes,
                                       slot.stream) != INTSORT_OK)
        return false;
    if (b && intsort_batched_sort_keys(ctx, INTSORT_U64, slot.d_desc + max_batch, b, keys64, nullptr, slot.ws,
                                       slot.ws_bytes, slot.stream) != INTSORT_OK)
        return false;
    return hipEventRecord(slot.done, slot.stream) == hipSuccess;
}

void intsort_server::run()
{
    (void)hipSetDevice(device);
    std::unique_lock<std::mutex> lk(mu);
    while (true) {
        bool progress = false;
        // retire finished batches
        for (Slot &sl : slots) {
            if (!sl.busy) continue;
            const hipError_t q = hipEventQuery(sl.done);
            if (q == hipErrorNotReady) continue;
            finish(sl.tickets, q == hipSuccess);
            sl.tickets.clear();
            sl.busy = false;
            progress = true;
        }
        if (outstanding == 0) idle.notify_all();
        if (stop && outstanding == 0) break;
        // admit waiting requests into a free slot
        for (Slot &sl : slots) {
            if (sl.busy || queue.empty()) continue;
            std::vector<uint64_t> batch;
            std::vector<Req> copies;
            uint64_t keys = 0;
            uint32_t n32 = 0, n64 = 0;
            while (!queue.empty()) {
                const Req &r = reqs.at(queue.front());
                if (in_flight + r.bytes > budget) break;   // wait for memory: arrival order is kept
                if (keys + r.n > max_batch_keys) break;
                if ((r.kt == INTSORT_U32 ? n32 : n64) >= max_batch) break;
                (r.kt == INTSORT_U32 ? n32 : n64)++;
                keys += r.n;
                in_flight += r.bytes;
                copies.push_back(r);
                batch.push_back(queue.front());
                queue.pop_front();
            }
            if (batch.empty()) break;
            for (uint64_t t : batch) reqs.at(t).state = 1;
            sl.busy = true;
            sl.tickets = batch;
            const bool inject = inject_failures > 0;
            if (inject) inject_failures--;
            lk.unlock();
            // an injected failure enqueues nothing, as when the first HIP call of the launch fails
            const bool ok = !inject && launch(sl, copies);
            // whatever part of a failed launch was enqueued finishes before the
            // requests are reported, so their arrays are free when the caller hears
            if (!ok) (void)hipStreamSynchronize(sl.stream);
            lk.lock();
            if (!ok) {
                finish(batch, false);
                sl.tickets.clear();
                sl.busy = false;
            }
            progress = true;
        }
        if (!progress) cv.wait_for(lk, std::chrono::microseconds(20));
    }
}

extern "C" {

intsort_status intsort_server_create(intsort_ctx *ctx, uint64_t hbm_budget_bytes, uint32_t max_batch,
                                     uint32_t slots, intsort_server **out)
{
    try {
        if (!out || !ctx || max_batch == 0 || slots == 0 || slots > 4 || hbm_budget_bytes == 0)
            return INTSORT_ERR_INVALID_ARGUMENT;
        *out = nullptr;
        const int dev = intsort::ctx_device(ctx);
        if (dev < 0) return INTSORT_ERR_UNSUPPORTED;
        if (hipSetDevice(dev) != hipSuccess) return INTSORT_ERR_HIP;
        intsort_server *s = new (std::nothrow) intsort_server;
        if (!s) return INTSORT_ERR_INTERNAL;
        s->device = dev;
        s->budget = hbm_budget_bytes;
        s->max_batch = max_batch;
        s->max_batch_keys = 1ull << 27;
        if (intsort_create(&s->ctx, dev) != INTSORT_OK) {
            delete s;
            return INTSORT_ERR_HIP;
        }
        size_t ws = 0;
        if (intsort_workspace_size(s->ctx, INTSORT_U64, 0, s->max_batch_keys, max_batch, nullptr, &ws) != INTSORT_OK) {
            intsort_destroy(s->ctx);
            delete s;
            return INTSORT_ERR_INTERNAL;
        }
        s->slots.resize(slots);
        bool ok = true;
        for (Slot &sl : s->slots) {
            sl.ws_bytes = ws;
            ok = ok && hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) == hipSuccess;
            ok = ok && hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) == hipSuccess;
            ok = ok && hipMalloc(&sl.ws, ws) == hipSuccess;
            ok = ok && hipHostMalloc((void **)&sl.h_desc, sizeof(intsort_segment_desc) * 2 * max_batch) == hipSuccess;
            ok = ok && hipMalloc((void **)&sl.d_desc, sizeof(intsort_segment_desc) * 2 * max_batch) == hipSuccess;
            if (!ok) break;
        }
        if (!ok) {
            for (Slot &sl : s->slots) {
                if (sl.stream) (void)hipStreamDestroy(sl.stream);
                if (sl.done) (void)hipEventDestroy(sl.done);
                if (sl.ws) (void)hipFree(sl.ws);
                if (sl.h_desc) (void)hipHostFree(sl.h_desc);
                if (sl.d_desc) (void)hipFree(sl.d_desc);
            }
            intsort_destroy(s->ctx);
            delete s;
            return INTSORT_ERR_HIP;
        }
        s->worker = std::thread([s] { s->run(); });
        *out = s;
        return INTSORT_OK;
    } catch (...) {
        return INTSORT_ERR_INTERNAL;
    }
}

intsort_status intsort_server_submit(intsort_server *s, intsort_key_type kt, const void *d_in, void *d_out,
                                     uint64_t n, uint64_t *ticket)
{
    try {
        if (!s || !ticket || (kt != INTSORT_U32 && kt != INTSORT_U64)) return INTSORT_ERR_INVALID_ARGUMENT;
        if (n > 0 && (!d_in || !d_out)) return INTSORT_ERR_INVALID_ARGUMENT;
        if (((reinterpret_cast<uintptr_t>(d_in) | reinterpret_cast<uintptr_t>(d_out)) & 15u) != 0)
            return INTSORT_ERR_MISALIGNED;
        const uint64_t bytes = footprint(kt, n);
        if (bytes > s->budget || n > s->max_batch_keys) return INTSORT_ERR_OVER_BUDGET;
        std::lock_guard<std::mutex> g(s->mu);
        if (s->stop) return INTSORT_ERR_INVALID_ARGUMENT;
        const uint64_t t = s->next_ticket++;
        Req r{};
        r.kt = kt;
        r.in = d_in;
        r.out = d_out;
        r.n = n;
        r.bytes = bytes;
        r.t_submit = clk::now();
        r.state = 0;
        s->reqs.emplace(t, r);
        s->queue.push_back(t);
        s->outstanding++;
        *ticket = t;
        s->cv.notify_one();
        return INTSORT_OK;
    } catch (...) {
        return INTSORT_ERR_INTERNAL;
    }
}

intsort_status intsort_server_poll(intsort_server *s, uint64_t ticket, int *done, double *latency_s)
{
    try {
        if (!s || !done) return INTSORT_ERR_INVALID_ARGUMENT;
        std::lock_guard<std::mutex> g(s->mu);
        auto it = s->reqs.find(ticket);
        if (it == s->reqs.end()) return INTSORT_ERR_INVALID_ARGUMENT;
        Req &r = it->second;
        *done = r.state >= 2;
        if (latency_s)
            *latency_s = *done ? std::chrono::duration<double>(r.t_done - r.t_submit).count() : 0.0;
        if (r.state == 3) {
            r.polled = true;
            if (r.listed) s->reqs.erase(it);
            return INTSORT_ERR_HIP;
        }
        return *done ? INTSORT_OK : INTSORT_ERR_NOT_READY;
    } catch (...) {
        return INTSORT_ERR_INTERNAL;
    }
}

intsort_status intsort_server_completed(intsort_server *s, uint64_t *tickets, double *latency_s, uint32_t capacity,
                                        uint32_t *count)
{
    try {
        if (!s || !count || (capacity > 0 && !tickets)) return INTSORT_ERR_INVALID_ARGUMENT;
        std::lock_guard<std::mutex> g(s->mu);
        uint32_t m = 0;
        size_t i = 0;
        bool failed = false;
        for (; i < s->completed.size() && m < capacity; i++, m++) {
            const uint64_t t = s->completed[i];
            Req &r = s->reqs.at(t);
            tickets[m] = t;
            if (latency_s) latency_s[m] = std::chrono::duration<double>(r.t_done - r.t_submit).count();
            // a failed request stays visible to poll until poll has reported it
            r.listed = true;
            if (r.state == 3) failed = true;
            if (r.state == 2 || r.polled) s->reqs.erase(t);
        }
        s->completed.erase(s->completed.begin(), s->completed.begin() + (long)i);
        *count = m;
        return failed ? INTSORT_ERR_HIP : INTSORT_OK;
    } catch (...) {
        return INTSORT_ERR_INTERNAL;
    }
}

intsort_status intsort_server_drain(intsort_server *s)
{
    try {
        if (!s) return INTSORT_ERR_INVALID_ARGUMENT;
        std::unique_lock<std::mutex> lk(s->mu);
        s->cv.notify_one();
        s->idle.wait(lk, [s] { return s->outstanding == 0; });
        const bool failed = s->failed_since_drain > 0;
        s->failed_since_drain = 0;
        return failed ? INTSORT_ERR_HIP : INTSORT_OK;
    } catch (...) {
        return INTSORT_ERR_INTERNAL;
    }
}

intsort_status intsort_server_fail_next_launches(intsort_server *s, uint32_t count)
{
    try {
        if (!s) return INTSORT_ERR_INVALID_ARGUMENT;
        std::lock_guard<std::mutex> g(s->mu);
        s->inject_failures = count;
        return INTSORT_OK;
    } catch (...) {
        return INTSORT_ERR_INTERNAL;
    }
}

intsort_status intsort_server_destroy(intsort_server *s)
{
    try {
        if (!s) return INTSORT_ERR_INVALID_ARGUMENT;
        {
            std::lock_guard<std::mutex> g(s->mu);
            s->stop = true;
            s->cv.notify_one();
        }
        if (s->worker.joinable()) s->worker.join();
        for (Slot &sl : s->slots) {
            (void)hipStreamSynchronize(sl.stream);
            (void)hipStreamDestroy(sl.stream);
            (void)hipEventDestroy(sl.done);
            (void)hipFree(sl.ws);
            (void)hipHostFree(sl.h_desc);
            (void)hipFree(sl.d_desc);
        }
        intsort_destroy(s->ctx);
        delete s;
        return INTSORT_OK;
    } catch (...) {
        return INTSORT_ERR_INTERNAL;
    }
}

}  // extern "C"
