// Serving engine: continuous batching of bootstrap requests.
//
// Callers submit requests (a batch of LWE samples of one parameter set, with
// per-sample tables) at any time from any thread.  A scheduler thread keeps a
// FIFO of waiting requests; whenever a stream slot is free it forms the next
// batch from the oldest waiting request and the later ones that share its
// context and flags (arrival order kept, up to max_batch samples), reserves the batch's device scratch against the
// memory budget (admission), gathers the inputs into the slot's staging
// buffers, enqueues the whole bootstrap on the slot's stream and scatters the
// outputs back.  Batches on different slots overlap on the device.  Keys stay
// resident; every result is bit-identical to a standalone call because each
// sample's bootstrap depends only on its own input.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "fdfb.h"
#include "internal.h"

using fdfbi::fail;

namespace {

using Clock = std::chrono::steady_clock;

struct Request {
    uint32_t ctx = 0, B = 0, flags = 0;
    const uint32_t *d_cts = nullptr;
    const int32_t *d_ids = nullptr;
    uint32_t *d_out = nullptr;
    int status = 0;  // 0 waiting or running, 1 done, < 0 error code
    Clock::time_point t_submit, t_done;
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    std::vector<fdfbi::Scratch> scratch;  // one per context
    uint32_t *in = nullptr, *out = nullptr;
    int32_t *ids = nullptr;
    bool busy = false;
    std::vector<uint64_t> reqs;
    size_t reserved = 0;
    uint32_t samples = 0;
};

}  // namespace

struct fdfb_server {
    std::vector<fdfb_ctx *> ctxs;
    uint32_t max_batch = 0;
    size_t budget = 0, in_flight = 0, max_in_flight = 0;
    std::vector<Slot> slots;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<uint64_t> waiting;
    std::unordered_map<uint64_t, Request> reqs;
    uint64_t next_id = 1;
    bool stop = false;
    int fatal = 0;
    std::thread worker;
    fdfb_serving_stats stats{};
    Clock::time_point t0 = Clock::now();

    size_t in_words() const
    {
        size_t w = 0;
        for (auto *c : ctxs) w = std::max<size_t>(w, c->P.n + 1);
        return w;
    }
    size_t out_words() const
    {
        size_t w = 0;
        for (auto *c : ctxs) w = std::max<size_t>(w, std::max(c->P.n, c->P.N) + 1);
        return w;
    }

    // Run one batch of requests on slot s (called without the lock held).
    int launch(Slot &s, uint32_t ci, const std::vector<Request *> &rs, uint32_t flags)
    {
        fdfb_ctx &c = *ctxs[ci];
        const size_t win = c.P.n + 1, wout = (flags & FDFB_OUT_EXTRACTED) ? c.P.N + 1 : c.P.n + 1;
        uint32_t off = 0;
        for (Request *r : rs) {
            if (hipMemcpyAsync(s.in + off * win, r->d_cts, 4 * win * r->B, hipMemcpyDeviceToDevice, s.stream) ||
                hipMemcpyAsync(s.ids + off, r->d_ids, 4 * (size_t)r->B, hipMemcpyDeviceToDevice, s.stream))
                return fail(FDFB_EDEVICE, "staging copy failed");
            off += r->B;
        }
        int rc = fdfbi::bootstrap_with(c, s.scratch[ci], s.in, s.ids, off, s.out, flags, s.stream);
        if (rc) return rc;
        off = 0;
        for (Request *r : rs) {
            if (hipMemcpyAsync(r->d_out, s.out + off * wout, 4 * wout * r->B, hipMemcpyDeviceToDevice, s.stream))
                return fail(FDFB_EDEVICE, "result copy failed");
            off += r->B;
        }
        if (hipEventRecord(s.done, s.stream)) return fail(FDFB_EDEVICE, "event record failed");
        return FDFB_OK;
    }

    void run()
    {
        std::unique_lock<std::mutex> lk(mu);
        while (true) {
            // retire finished batches
            bool any_busy = false;
            for (Slot &s : slots) {
                if (!s.busy) continue;
                const hipError_t q = hipEventQuery(s.done);
                if (q == hipErrorNotReady) {
                    any_busy = true;
                    continue;
                }
                // hipSuccess: the batch is done; any other result is a device
                // error: its requests fail instead of waiting forever
                if (q != hipSuccess) fatal = FDFB_EDEVICE;
                const auto now = Clock::now();
                for (uint64_t id : s.reqs) {
                    Request &r = reqs[id];
                    if (r.status == 0) r.status = (q == hipSuccess) ? 1 : FDFB_EDEVICE;
                    r.t_done = now;
                    stats.requests_done++;
                    stats.bootstraps_done += r.B;
                }
                s.reqs.clear();
                s.busy = false;
                in_flight -= s.reserved;
                s.reserved = 0;
                cv_done.notify_all();
            }
            if (stop && waiting.empty() && !any_busy) break;

            // admit the next batch into a free slot
            Slot *free_slot = nullptr;
            for (Slot &s : slots)
                if (!s.busy) { free_slot = &s; break; }
            if (free_slot && !waiting.empty()) {
                const Request &head = reqs[waiting.front()];
                const uint32_t ci = head.ctx, flags = head.flags;
                // the oldest request and the requests behind it that share its
                // context and flags, in arrival order, up to max_batch samples
                std::vector<uint64_t> take;
                uint32_t total = 0;
                for (auto it = waiting.begin(); it != waiting.end(); ++it) {
                    const Request &r = reqs[*it];
                    if (r.ctx != ci || r.flags != flags) continue;
                    if (total + r.B > max_batch) break;
                    take.push_back(*it);
                    total += r.B;
                }
                const size_t bytes = fdfbi::Scratch::bytes_for(ctxs[ci]->P, total);
                if (in_flight == 0 || in_flight + bytes <= budget) {
                    for (uint64_t id : take) waiting.erase(std::find(waiting.begin(), waiting.end(), id));
                    in_flight += bytes;
                    max_in_flight = std::max(max_in_flight, in_flight);
                    free_slot->busy = true;
                    free_slot->reserved = bytes;
                    free_slot->reqs = take;
                    free_slot->samples = total;
                    std::vector<Request *> rs;
                    for (uint64_t id : take) rs.push_back(&reqs[id]);
                    stats.batches++;
                    lk.unlock();
                    int rc = launch(*free_slot, ci, rs, flags);
                    lk.lock();
                    if (rc) {
                        fatal = rc;
                        for (uint64_t id : take) reqs[id].status = rc;
                        // let the event mark the slot free once queued work drains
                        (void)hipEventRecord(free_slot->done, free_slot->stream);
                        cv_done.notify_all();
                    }
                    continue;  // look for more work immediately
                }
            }
            cv_work.wait_for(lk, std::chrono::microseconds(any_busy ? 50 : 2000));
        }
    }
};

extern "C" {

int fdfb_server_create(fdfb_ctx *const *ctxs, uint32_t nctx, uint32_t max_batch, size_t mem_budget,
                       uint32_t nstreams, fdfb_server **out)
{
    if (!ctxs || !nctx || !out || !max_batch || !nstreams || nstreams > 8)
        return fail(FDFB_EINVAL, "need contexts, max_batch > 0 and 1..8 streams");
    *out = nullptr;
    auto *sv = new (std::nothrow) fdfb_server();
    if (!sv) return fail(FDFB_ENOMEM, "server allocation failed");
    sv->ctxs.assign(ctxs, ctxs + nctx);
    sv->max_batch = max_batch;
    sv->budget = mem_budget;
    for (fdfb_ctx *c : sv->ctxs) {
        if (!c) { delete sv; return fail(FDFB_EINVAL, "null context"); }
        if (int rc = fdfbi::ensure_device(*c)) { delete sv; return rc; }
    }
    sv->slots.resize(nstreams);
    for (Slot &s : sv->slots) {
        s.scratch.resize(nctx);
        if (hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking) ||
            hipEventCreateWithFlags(&s.done, hipEventDisableTiming) ||
            hipMalloc((void **)&s.in, 4 * sv->in_words() * max_batch) ||
            hipMalloc((void **)&s.ids, 4 * (size_t)max_batch) ||
            hipMalloc((void **)&s.out, 4 * sv->out_words() * max_batch)) {
            fdfb_server_destroy(sv);
            return fail(FDFB_ENOMEM, "server buffers");
        }
    }
    sv->worker = std::thread([sv] { sv->run(); });
    *out = sv;
    return FDFB_OK;
}

int fdfb_server_submit(fdfb_server *sv, uint32_t ctx_index, const uint32_t *d_cts, const int32_t *d_lut_ids,
                       uint32_t B, uint32_t *d_out, uint32_t flags, uint64_t *req_id)
{
    if (!sv || !req_id) return fail(FDFB_EINVAL, "null argument");
    if (ctx_index >= sv->ctxs.size()) return fail(FDFB_EINVAL, "context index out of range");
    if (B == 0 || B > sv->max_batch) return fail(FDFB_EINVAL, "request size must be in 1..max_batch");
    if (!d_cts || !d_lut_ids || !d_out) return fail(FDFB_EINVAL, "null buffer");
    if (flags & ~fdfbi::kAllFlags) return fail(FDFB_EINVAL, "unknown flag");
    if (int rc = fdfbi::check_form(*sv->ctxs[ctx_index], flags)) return rc;
    if (sv->ctxs[ctx_index]->nluts != sv->ctxs[ctx_index]->dev_nluts)
        return fail(FDFB_EINVAL, "tables must be registered before the server is created");
    std::lock_guard<std::mutex> lk(sv->mu);
    if (sv->fatal) return fail(sv->fatal, "server stopped after a device error");
    const uint64_t id = sv->next_id++;
    Request &r = sv->reqs[id];
    r.ctx = ctx_index;
    r.B = B;
    r.flags = flags;
    r.d_cts = d_cts;
    r.d_ids = d_lut_ids;
    r.d_out = d_out;
    r.t_submit = Clock::now();
    sv->waiting.push_back(id);
    *req_id = id;
    sv->cv_work.notify_one();
    return FDFB_OK;
}

int fdfb_server_poll(fdfb_server *sv, uint64_t req_id, int *done)
{
    if (!sv || !done) return fail(FDFB_EINVAL, "null argument");
    std::lock_guard<std::mutex> lk(sv->mu);
    auto it = sv->reqs.find(req_id);
    if (it == sv->reqs.end()) return fail(FDFB_EINVAL, "unknown request");
    if (it->second.status < 0) return it->second.status;
    *done = it->second.status == 1;
    return FDFB_OK;
}

int fdfb_server_wait(fdfb_server *sv, uint64_t req_id, double *latency_s)
{
    if (!sv) return fail(FDFB_EINVAL, "null server");
    std::unique_lock<std::mutex> lk(sv->mu);
    auto it = sv->reqs.find(req_id);
    if (it == sv->reqs.end()) return fail(FDFB_EINVAL, "unknown request");
    sv->cv_done.wait(lk, [&] { return it->second.status != 0; });
    const int st = it->second.status;
    if (latency_s)
        *latency_s = std::chrono::duration<double>(it->second.t_done - it->second.t_submit).count();
    sv->reqs.erase(it);
    return st < 0 ? fail(st, "request failed") : FDFB_OK;
}

int fdfb_server_stats(fdfb_server *sv, fdfb_serving_stats *out)
{
    if (!sv || !out) return fail(FDFB_EINVAL, "null argument");
    std::lock_guard<std::mutex> lk(sv->mu);
    *out = sv->stats;
    out->max_in_flight_bytes = sv->max_in_flight;
    out->seconds = std::chrono::duration<double>(Clock::now() - sv->t0).count();
    return FDFB_OK;
}

void fdfb_server_destroy(fdfb_server *sv)
{
    if (!sv) return;
    if (sv->worker.joinable()) {
        {
            std::lock_guard<std::mutex> lk(sv->mu);
            sv->stop = true;
        }
        sv->cv_work.notify_all();
        sv->worker.join();
    }
    for (Slot &s : sv->slots) {
        if (s.stream) (void)hipStreamSynchronize(s.stream);
        for (void *p : {(void *)s.in, (void *)s.ids, (void *)s.out})
            if (p) (void)hipFree(p);
        s.scratch.clear();
        if (s.done) (void)hipEventDestroy(s.done);
        if (s.stream) (void)hipStreamDestroy(s.stream);
    }
    delete sv;
}

}  // extern "C"
