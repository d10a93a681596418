// Internal interfaces of the FDFB host core shared by the C ABI (host.cpp)
// and the serving engine (server.cpp).  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>

#include <atomic>
#include <exception>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "fdfb.h"
#include "kernels.h"

namespace fdfbi {

// Device scratch of one bootstrap batch, carved from one block of memory:
// ModSwitched samples, sign accumulators, bit samples, switched RLWE samples,
// built accumulators, c_Q, and the work counters of the persistent blind
// rotation.  The block may be owned by a context's per-stream pool, a
// server's arena or the library's static no-allocation buffer.
struct ScratchView {
    uint32_t *ctN = nullptr, *acc_sign = nullptr, *cbits = nullptr, *rbits = nullptr, *accf = nullptr,
             *cq = nullptr;
    uint32_t *work = nullptr;  // kWorkWords counters, reset on the device before each use
};
constexpr size_t kWorkWords = 64;
// Jobs of one multi-job submission: each phase takes at most one queue
// launch per kQueueJobs jobs plus one per geometry pair, two counters each.
constexpr uint32_t kMaxJobs = 256;

// Bytes of scratch for B samples with L tables each (every buffer 256-byte aligned).
size_t scratch_bytes(const fdfb_params &P, uint32_t B, uint32_t L = 1);
// Lay out the buffers of scratch_bytes(P, B, L) bytes starting at base.
ScratchView carve_scratch(const fdfb_params &P, uint32_t B, uint32_t L, void *base);

// One stream's scratch block of a context.  Blocks are replaced, not resized:
// a larger batch allocates a new block (at least twice the old one) and the
// old block is kept until the context is freed or fdfb_release_scratch, so
// work already enqueued or captured in a HIP graph never sees freed memory.
struct StreamScratch {
    void *stream = nullptr;
    void *base = nullptr;
    size_t bytes = 0;
};

int fail(int code, const std::string &msg);

// Run an entry point's body, turning any C++ exception into an error code:
// no exception crosses the C ABI.
template <class F>
int guarded(F &&f) noexcept
{
    try {
        return f();
    } catch (const std::bad_alloc &) {
        return fail(FDFB_ENOMEM, "host allocation failed");
    } catch (const std::length_error &e) {
        return fail(FDFB_ENOMEM, std::string("host allocation failed: ") + e.what());
    } catch (const std::exception &e) {
        return fail(FDFB_EINVAL, std::string("unexpected error: ") + e.what());
    } catch (...) {
        return fail(FDFB_EINVAL, "unexpected error");
    }
}

}  // namespace fdfbi

struct fdfb_ctx {
    fdfb_params P{};
    uint64_t seed = 0;
    std::vector<uint32_t> s, sf, brk, pk, ksk;
    std::vector<uint32_t> lut_tables;  // [nluts][t]
    std::vector<int32_t> lut_polys;    // [nluts][2][N]: rotP_0, rotP_1
    int nluts = 0;

    fdfbk::Geometry geom{};
    bool mfma_ok = false;

    // Serialises every call on the context (host state, uploads, scratch
    // pools and the order of enqueued work); recursive for nested helpers.
    std::recursive_mutex mu;

    bool on_device = false;
    uint32_t *d_brk = nullptr, *d_pk = nullptr, *d_ksk = nullptr;
    void *d_brk_frag = nullptr;      // Karatsuba form: lane-ordered key fragments
    uint32_t *d_brk_corr = nullptr;  // Karatsuba form: offset correction per (i, j)
    void *d_brk_direct = nullptr;    // direct form (FDFB_DIRECT): key byte planes, built on first use
    void *d_pk_frag = nullptr, *d_ksk_frag = nullptr;  // int8 MFMA key-switch fragments
    uint32_t *d_err = nullptr;       // device error bits (FDFB_DEVERR_*), sticky until read
    int32_t *d_luts = nullptr;
    int dev_nluts = 0;
    size_t d_luts_cap = 0;           // tables the current d_luts buffer holds

    std::vector<fdfbi::StreamScratch> pools;  // direct calls: one scratch block per stream
    std::vector<void *> retired;              // replaced blocks, freed with the context

    std::atomic<int> abort_flag{0};

    bool profiling = false;
    bool trace = false;  // FDFB_TRACE: print the phase timings when the context is freed
    std::vector<hipEvent_t> prof_events;  // FDFB_NPHASES + 1 per recorded call

    void release_scratch();
    ~fdfb_ctx();
};

namespace fdfbi {

// Every flag an entry point accepts.
constexpr uint32_t kAllFlags = FDFB_OUT_EXTRACTED | FDFB_PLAIN | FDFB_DIRECT;
// Upload what the requested blind-rotation form needs beyond ensure_device.
int ensure_form(fdfb_ctx &c, uint32_t flags);
// Upload keys and registered tables on first use (or after new tables).
int ensure_device(fdfb_ctx &c);
// True when a call with these flags would enqueue kernels only: keys, tables
// and the requested form are resident.
bool device_ready(const fdfb_ctx &c, uint32_t flags);
// Scratch for B samples with L tables on `stream` from the context's pool.
int pool_scratch(fdfb_ctx &c, void *stream, uint32_t B, uint32_t L, ScratchView *out);
// A scratch block of at least `bytes` on `stream` from the context's pool.
int pool_block(fdfb_ctx &c, void *stream, size_t bytes, void **base);
// The requested blind-rotation form must exist for the context's parameters.
int check_form(const fdfb_ctx &c, uint32_t flags);
// Enqueue one full bootstrap batch on `st` using scratch `sc` (keys already
// resident): L tables per sample (ids [B][L], outputs [B][L][dim]) share the
// sign rotations.  Allocates nothing unless `profile` and the context
// records phase timings (events are created then).
int enqueue_bootstrap(fdfb_ctx &c, const ScratchView &sc, const uint32_t *d_cts, const int32_t *d_ids,
                      uint32_t B, uint32_t *d_out, uint32_t flags, hipStream_t st, uint32_t L = 1,
                      bool profile = true);
// The issue plan recorded by the autotuner for A accumulators of geometry G
// on the current device (kFormAuto if none).
fdfbk::BrPlan tuned_plan(const fdfbk::Geometry &G, uint32_t A);
// The persistent work-queue kernel can take this context's rotations with these flags.
bool queue_eligible(const fdfb_ctx &c, uint32_t flags);
// Enqueue several bootstrap jobs phase by phase: every job's ModSwitch and
// sign accumulators, the sign rotations of all jobs (the queue-eligible ones
// in persistent work-queue launches when use_queue), every job's bit samples,
// packing switch and public mux, the function rotations of all jobs, then
// every job's output.  views[k] is job k's scratch; counters: ncounters
// device words for the queue launches.
int enqueue_multi(const fdfb_job *jobs, uint32_t njobs, const ScratchView *views, uint32_t *counters,
                  uint32_t ncounters, bool use_queue, hipStream_t st);
// Enqueue queue-eligible jobs as a software pipeline: each persistent
// work-queue launch takes the function rotations of the jobs whose public
// mux is enqueued, then the next jobs' sign rotations (split at whole samples)
// up to `rounds` rounds of the kernel's resident capacity; after it, the
// outputs of those function rotations and the public mux of every job whose
// sign rotations are complete.  The counters are reused by every launch.
int enqueue_pipeline(const fdfb_job *jobs, uint32_t njobs, const ScratchView *views, uint32_t *counters,
                     uint32_t ncounters, uint32_t rounds, hipStream_t st);
constexpr uint32_t kMaxPipelineRounds = 64;

}  // namespace fdfbi
