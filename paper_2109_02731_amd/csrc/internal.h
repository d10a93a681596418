// Internal interfaces of the FDFB host core shared by the C ABI (host.cpp)
// and the serving engine (server.cpp).  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>

#include <atomic>
#include <string>
#include <vector>

#include "fdfb.h"
#include "kernels.h"

namespace fdfbi {

// Device scratch of one bootstrap batch: ModSwitched samples, sign
// accumulators, bit samples, switched RLWE samples, built accumulators, c_Q.
struct Scratch {
    uint32_t cap = 0;   // capacity in samples
    uint32_t capf = 0;  // capacity in table evaluations (samples x tables per sample)
    uint32_t *ctN = nullptr, *acc_sign = nullptr, *cbits = nullptr, *rbits = nullptr, *accf = nullptr,
             *cq = nullptr;
    static size_t bytes_for(const fdfb_params &P, uint32_t B, uint32_t L = 1);
    void release();
    ~Scratch() { release(); }
};

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

    bool on_device = false;
    uint32_t *d_brk = nullptr, *d_pk = nullptr, *d_ksk = nullptr;
    void *d_brk_frag = nullptr;      // Karatsuba form: lane-ordered key fragments
    uint32_t *d_brk_corr = nullptr;  // Karatsuba form: offset correction per (i, j)
    void *d_brk_direct = nullptr;    // direct form (FDFB_DIRECT): key byte planes, built on first use
    void *d_pk_frag = nullptr, *d_ksk_frag = nullptr;  // int8 MFMA key-switch fragments
    int32_t *d_luts = nullptr;
    int dev_nluts = 0;

    fdfbi::Scratch scratch;  // for direct (non-server) calls

    std::atomic<int> abort_flag{0};

    bool profiling = false;
    bool trace = false;  // FDFB_TRACE: print the phase timings when the context is freed
    std::vector<hipEvent_t> prof_events;  // FDFB_NPHASES + 1 per recorded call

    ~fdfb_ctx()
    {
        for (hipEvent_t e : prof_events) (void)hipEventDestroy(e);
        scratch.release();
        for (void *p : {(void *)d_brk, (void *)d_pk, (void *)d_ksk, d_brk_frag, (void *)d_brk_corr, d_brk_direct,
                        d_pk_frag, d_ksk_frag,
                        (void *)d_luts})
            if (p) (void)hipFree(p);
    }
};

namespace fdfbi {

int fail(int code, const std::string &msg);
// Every flag an entry point accepts.
constexpr uint32_t kAllFlags = FDFB_OUT_EXTRACTED | FDFB_PLAIN | FDFB_DIRECT;
// Upload what the requested blind-rotation form needs beyond ensure_device.
int ensure_form(fdfb_ctx &c, uint32_t flags);
// Upload keys and registered tables on first use (or after new tables).
int ensure_device(fdfb_ctx &c);
int ensure_scratch(fdfb_ctx &c, Scratch &sc, uint32_t B, uint32_t L = 1);
// The requested blind-rotation form must exist for the context's parameters.
int check_form(const fdfb_ctx &c, uint32_t flags);
// Enqueue one full bootstrap batch on `st` using scratch `sc`: L tables per
// sample (ids [B][L], outputs [B][L][dim]) share the sign rotations.
int bootstrap_with(fdfb_ctx &c, Scratch &sc, const uint32_t *d_cts, const int32_t *d_ids, uint32_t B,
                   uint32_t *d_out, uint32_t flags, hipStream_t st, uint32_t L = 1);

}  // namespace fdfbi
