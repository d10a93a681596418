// Serving engine: continuous batching of bootstrap requests.
//
// Callers submit requests (a batch of LWE samples of one parameter set, with
// per-sample tables) at any time from any thread; each submission records an
// event on the caller's stream, so the request's inputs may still be being
// written by earlier work there.  A scheduler thread keeps a FIFO of waiting
// requests; whenever a stream slot is free it forms the next batch from the
// oldest waiting request and the later ones that share its context and
// flags (arrival order kept, up to max_batch samples) and admits it by
// memory: the batch's staging buffers and bootstrap scratch are carved from
// one device arena of exactly the memory budget (first fit), so the budget
// bounds the device memory serving uses besides the keys.  A batch that does
// not fit is shortened to the requests that do, or waits for running batches
// to retire.  The slot's stream waits on the requests' events, gathers the
// inputs, runs the whole bootstrap and scatters the outputs.  Batches on
// different slots overlap on the device.  Keys stay resident; every result
// is bit-identical to a standalone call because each sample's bootstrap
// depends only on its own input.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "fdfb.h"
#include "arena.h"
#include "internal.h"

using fdfbi::fail;
using fdfbi::guarded;

namespace {

using Clock = std::chrono::steady_clock;

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct Request {
    uint32_t ctx = 0, B = 0, flags = 0;
    const uint32_t *d_cts = nullptr;
    const int32_t *d_ids = nullptr;
    uint32_t *d_out = nullptr;
    hipEvent_t ready = nullptr;  // recorded on the caller's stream at submission
    int status = 0;              // 0 waiting or running, 1 done, < 0 error code
    Clock::time_point t_submit, t_done;
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    bool busy = false;
    std::vector<uint64_t> reqs;
    size_t off = 0, bytes = 0;  // the batch's region of the arena
};


}  // namespace

struct fdfb_server {
    std::vector<fdfb_ctx *> ctxs;
    uint32_t max_batch = 0;
    size_t budget = 0, in_flight = 0, max_in_flight = 0;
    char *arena_base = nullptr;
    fdfbi::Arena arena;
    std::vector<Slot> slots;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<uint64_t> waiting;
    std::unordered_map<uint64_t, Request> reqs;
    std::vector<hipEvent_t> event_pool;
    uint64_t next_id = 1;
    bool stop = false;
    std::thread worker;
    fdfb_serving_stats stats{};
    Clock::time_point t0 = Clock::now();

    // Device resources (the scheduler thread has been joined by then).
    ~fdfb_server()
    {
        for (Slot &s : slots) {
            if (s.stream) (void)hipStreamSynchronize(s.stream);
            if (s.done) (void)hipEventDestroy(s.done);
            if (s.stream) (void)hipStreamDestroy(s.stream);
        }
        for (auto &kv : reqs)
            if (kv.second.ready) (void)hipEventDestroy(kv.second.ready);
        for (hipEvent_t e : event_pool) (void)hipEventDestroy(e);
        if (arena_base) (void)hipFree(arena_base);
    }

    static size_t out_width(const fdfb_ctx &c, uint32_t flags)
    {
        return (flags & FDFB_OUT_EXTRACTED) ? c.P.N + 1 : c.P.n + 1;
    }
    // Device bytes of a batch of `total` samples: staging (inputs, ids,
    // outputs) and the bootstrap's scratch.
    static size_t batch_bytes(const fdfb_ctx &c, uint32_t flags, uint32_t total)
    {
        return align256(4 * (size_t)total * (c.P.n + 1)) + align256(4 * (size_t)total) +
               align256(4 * (size_t)total * out_width(c, flags)) + fdfbi::scratch_bytes(c.P, total);
    }

    // Enqueue one batch on slot s, in its arena region (called without the lock).
    int launch(Slot &s, uint32_t ci, const std::vector<Request *> &rs, uint32_t flags, uint32_t total)
    {
        fdfb_ctx &c = *ctxs[ci];
        const size_t win = c.P.n + 1, wout = out_width(c, flags);
        char *p = arena_base + s.off;
        uint32_t *in = reinterpret_cast<uint32_t *>(p);
        p += align256(4 * (size_t)total * win);
        int32_t *ids = reinterpret_cast<int32_t *>(p);
        p += align256(4 * (size_t)total);
        uint32_t *out = reinterpret_cast<uint32_t *>(p);
        p += align256(4 * (size_t)total * wout);
        const fdfbi::ScratchView sc = fdfbi::carve_scratch(c.P, total, 1, p);
        uint32_t off = 0;
        for (Request *r : rs) {
            if (hipStreamWaitEvent(s.stream, r->ready, 0) ||
                hipMemcpyAsync(in + off * win, r->d_cts, 4 * win * r->B, hipMemcpyDeviceToDevice, s.stream) ||
                hipMemcpyAsync(ids + off, r->d_ids, 4 * (size_t)r->B, hipMemcpyDeviceToDevice, s.stream))
                return fail(FDFB_EDEVICE, "staging copy failed");
            off += r->B;
        }
        {
            std::lock_guard<std::recursive_mutex> lk(c.mu);
            int rc = fdfbi::ensure_device(c);  // tables registered since the last batch
            if (!rc) rc = fdfbi::ensure_form(c, flags);
            if (!rc) rc = fdfbi::enqueue_bootstrap(c, sc, in, ids, total, out, flags, s.stream);
            if (rc) return rc;
        }
        off = 0;
        for (Request *r : rs) {
            if (hipMemcpyAsync(r->d_out, out + off * wout, 4 * wout * r->B, hipMemcpyDeviceToDevice, s.stream))
                return fail(FDFB_EDEVICE, "result copy failed");
            off += r->B;
        }
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
                // error: the batch's requests fail instead of waiting forever
                const auto now = Clock::now();
                for (uint64_t id : s.reqs) {
                    Request &r = reqs[id];
                    if (r.status == 0) r.status = (q == hipSuccess) ? 1 : FDFB_EDEVICE;
                    r.t_done = now;
                    if (r.status == 1) {
                        stats.requests_done++;
                        stats.bootstraps_done += r.B;
                    }
                }
                s.reqs.clear();
                s.busy = false;
                arena.release(s.off, s.bytes);
                in_flight -= s.bytes;
                s.bytes = 0;
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
                std::vector<uint32_t> prefix;  // samples of take[0..k]
                uint32_t total = 0;
                for (auto it = waiting.begin(); it != waiting.end(); ++it) {
                    const Request &r = reqs[*it];
                    if (r.ctx != ci || r.flags != flags) continue;
                    if (total + r.B > max_batch) break;
                    take.push_back(*it);
                    total += r.B;
                    prefix.push_back(total);
                }
                // admission: the longest prefix of the batch whose memory fits
                // the arena now (every single request fits an empty arena)
                size_t off = 0, bytes = 0;
                size_t k = take.size();
                while (k > 0) {
                    bytes = batch_bytes(*ctxs[ci], flags, prefix[k - 1]);
                    if (arena.alloc(bytes, &off)) break;
                    --k;
                }
                if (k > 0) {
                    take.resize(k);
                    total = prefix[k - 1];
                    for (uint64_t id : take) waiting.erase(std::find(waiting.begin(), waiting.end(), id));
                    in_flight += bytes;
                    max_in_flight = std::max(max_in_flight, in_flight);
                    free_slot->busy = true;
                    free_slot->off = off;
                    free_slot->bytes = bytes;
                    free_slot->reqs = take;
                    std::vector<Request *> rs;
                    for (uint64_t id : take) rs.push_back(&reqs[id]);
                    stats.batches++;
                    lk.unlock();
                    int rc = launch(*free_slot, ci, rs, flags, total);
                    // the slot is free again once everything queued on it has run
                    const hipError_t er = hipEventRecord(free_slot->done, free_slot->stream);
                    lk.lock();
                    for (Request *r : rs) event_pool.push_back(r->ready);  // waits already enqueued
                    for (Request *r : rs) r->ready = nullptr;
                    if (rc || er != hipSuccess) {
                        if (!rc) rc = fail(FDFB_EDEVICE, "event record failed");
                        // only this batch fails; its region is released when the
                        // slot retires (or now, if the event could not be recorded)
                        for (uint64_t id : take) reqs[id].status = rc;
                        if (er != hipSuccess) {
                            (void)hipStreamSynchronize(free_slot->stream);
                            free_slot->busy = false;
                            free_slot->reqs.clear();
                            arena.release(free_slot->off, free_slot->bytes);
                            in_flight -= free_slot->bytes;
                            free_slot->bytes = 0;
                        }
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
    return guarded([&]() -> int {
        if (!ctxs || !nctx || !out || !max_batch || !nstreams || nstreams > 8)
            return fail(FDFB_EINVAL, "need contexts, max_batch > 0 and 1..8 streams");
        *out = nullptr;
        std::unique_ptr<fdfb_server> sv(new fdfb_server());
        sv->ctxs.assign(ctxs, ctxs + nctx);
        sv->max_batch = max_batch;
        size_t need = 0;
        for (fdfb_ctx *c : sv->ctxs) {
            if (!c) return fail(FDFB_EINVAL, "null context");
            std::lock_guard<std::recursive_mutex> lk(c->mu);
            if (int rc = fdfbi::ensure_device(*c)) return rc;
            need = std::max({need, fdfb_server::batch_bytes(*c, 0, max_batch),
                             fdfb_server::batch_bytes(*c, FDFB_OUT_EXTRACTED, max_batch)});
        }
        if (mem_budget < need)
            return fail(FDFB_EINVAL, "memory budget below one batch of max_batch samples (" + std::to_string(need) +
                                         " bytes)");
        sv->budget = mem_budget & ~(size_t)255;
        if (hipMalloc((void **)&sv->arena_base, sv->budget) != hipSuccess) {
            sv->arena_base = nullptr;
            return fail(FDFB_ENOMEM, "serving arena");
        }
        sv->arena.reset(sv->budget);
        sv->slots.resize(nstreams);
        for (Slot &s : sv->slots)
            if (hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking) ||
                hipEventCreateWithFlags(&s.done, hipEventDisableTiming))
                return fail(FDFB_EDEVICE, "server streams");
        fdfb_server *raw = sv.release();
        raw->worker = std::thread([raw] { raw->run(); });
        *out = raw;
        return FDFB_OK;
    });
}

int fdfb_server_submit(fdfb_server *sv, uint32_t ctx_index, const uint32_t *d_cts, const int32_t *d_lut_ids,
                       uint32_t B, uint32_t *d_out, uint32_t flags, void *stream, uint64_t *req_id)
{
    return guarded([&]() -> int {
        if (!sv || !req_id) return fail(FDFB_EINVAL, "null argument");
        if (ctx_index >= sv->ctxs.size()) return fail(FDFB_EINVAL, "context index out of range");
        if (B == 0 || B > sv->max_batch) return fail(FDFB_EINVAL, "request size must be in 1..max_batch");
        if (!d_cts || !d_lut_ids || !d_out) return fail(FDFB_EINVAL, "null buffer");
        if (flags & ~fdfbi::kAllFlags) return fail(FDFB_EINVAL, "unknown flag");
        if (int rc = fdfbi::check_form(*sv->ctxs[ctx_index], flags)) return rc;
        hipEvent_t ev = nullptr;
        {
            std::lock_guard<std::mutex> lk(sv->mu);
            if (!sv->event_pool.empty()) {
                ev = sv->event_pool.back();
                sv->event_pool.pop_back();
            }
        }
        if (!ev && hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess)
            return fail(FDFB_EDEVICE, "request event");
        if (hipEventRecord(ev, (hipStream_t)stream) != hipSuccess) {
            std::lock_guard<std::mutex> lk(sv->mu);
            sv->event_pool.push_back(ev);
            return fail(FDFB_EDEVICE, "request event record");
        }
        std::lock_guard<std::mutex> lk(sv->mu);
        const uint64_t id = sv->next_id++;
        Request &r = sv->reqs[id];
        r.ctx = ctx_index;
        r.B = B;
        r.flags = flags;
        r.d_cts = d_cts;
        r.d_ids = d_lut_ids;
        r.d_out = d_out;
        r.ready = ev;
        r.t_submit = Clock::now();
        sv->waiting.push_back(id);
        *req_id = id;
        sv->cv_work.notify_one();
        return FDFB_OK;
    });
}

int fdfb_server_poll(fdfb_server *sv, uint64_t req_id, int *done)
{
    return guarded([&]() -> int {
        if (!sv || !done) return fail(FDFB_EINVAL, "null argument");
        std::lock_guard<std::mutex> lk(sv->mu);
        auto it = sv->reqs.find(req_id);
        if (it == sv->reqs.end()) return fail(FDFB_EINVAL, "unknown request");
        if (it->second.status < 0) return fail(it->second.status, "request failed");
        *done = it->second.status == 1;
        return FDFB_OK;
    });
}

int fdfb_server_wait(fdfb_server *sv, uint64_t req_id, double *latency_s)
{
    return guarded([&]() -> int {
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
    });
}

int fdfb_server_stats(fdfb_server *sv, fdfb_serving_stats *out)
{
    return guarded([&]() -> int {
        if (!sv || !out) return fail(FDFB_EINVAL, "null argument");
        std::lock_guard<std::mutex> lk(sv->mu);
        *out = sv->stats;
        out->max_in_flight_bytes = sv->max_in_flight;
        out->arena_bytes = sv->budget;
        out->seconds = std::chrono::duration<double>(Clock::now() - sv->t0).count();
        return FDFB_OK;
    });
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
    delete sv;
}

}  // extern "C"
