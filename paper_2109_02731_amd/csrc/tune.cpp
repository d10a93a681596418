// Autotuner of the batched blind rotation: for a ring geometry and a number
// of accumulators it times every issue plan the kernels offer (kernel form,
// wavefronts per accumulator, accumulators per launch round, persistent work
// queue) on the device and records the fastest.  Every later rotation of
// that size and geometry is issued with the recorded plan.  All plans give
// the same bits (the arithmetic is exact and each plan runs the same
// per-accumulator chain), so the choice affects time only.
//
// The table is per process and keyed by (compute units, N, ell, digit
// chunks, n, accumulators).  With FDFB_TUNE_CACHE set to a file path, the
// table is read from that file at first use and written back after each
// tuning run; the file holds one JSON object per line inside a JSON list.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "fdfb.h"
#include "internal.h"

using fdfbi::fail;
using fdfbi::guarded;

namespace {

struct Entry {
    uint32_t cus, N, ell, ch, n, A;
    fdfbk::BrPlan plan;
    double ms;
};

std::mutex g_mu;
std::vector<Entry> g_table;
bool g_loaded = false;

uint32_t device_cus()
{
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    return (uint32_t)cus;
}

bool same_key(const Entry &e, uint32_t cus, const fdfbk::Geometry &G, uint32_t A)
{
    return e.cus == cus && e.N == (uint32_t)G.N && e.ell == (uint32_t)G.g_ell &&
           e.ch == (uint32_t)fdfbk::digit_chunks(G.g_log2B) && e.n == (uint32_t)G.n && e.A == A;
}

void put(const Entry &x)
{
    for (Entry &e : g_table)
        if (e.cus == x.cus && e.N == x.N && e.ell == x.ell && e.ch == x.ch && e.n == x.n && e.A == x.A) {
            e = x;
            return;
        }
    g_table.push_back(x);
}

// Read a cache file written by save_locked (lines that do not parse are skipped).
int load_locked(const char *path, bool must_exist)
{
    FILE *f = std::fopen(path, "r");
    if (!f) return must_exist ? fail(FDFB_EINVAL, std::string("cannot open tuning cache ") + path) : FDFB_OK;
    char line[512];
    while (std::fgets(line, sizeof line, f)) {
        Entry e{};
        unsigned cus, N, ell, ch, n, A, form, round;
        double ms;
        if (std::sscanf(line,
                        " {\"cus\": %u, \"N\": %u, \"ell\": %u, \"chunks\": %u, \"n\": %u, \"A\": %u, \"form\": %u, "
                        "\"round\": %u, \"ms\": %lf}",
                        &cus, &N, &ell, &ch, &n, &A, &form, &round, &ms) == 9) {
            e.cus = cus; e.N = N; e.ell = ell; e.ch = ch; e.n = n; e.A = A;
            e.plan.form = form;
            e.plan.round = round;
            e.ms = ms;
            if (form <= fdfbk::kFormSplit) put(e);
        }
    }
    std::fclose(f);
    return FDFB_OK;
}

int save_locked(const char *path)
{
    const std::string tmp = std::string(path) + ".tmp";
    FILE *f = std::fopen(tmp.c_str(), "w");
    if (!f) return fail(FDFB_EINVAL, std::string("cannot write tuning cache ") + path);
    std::fprintf(f, "[\n");
    for (size_t k = 0; k < g_table.size(); ++k) {
        const Entry &e = g_table[k];
        std::fprintf(f,
                     " {\"cus\": %u, \"N\": %u, \"ell\": %u, \"chunks\": %u, \"n\": %u, \"A\": %u, \"form\": %u, "
                     "\"round\": %u, \"ms\": %.4f}%s\n",
                     e.cus, e.N, e.ell, e.ch, e.n, e.A, e.plan.form, e.plan.round, e.ms,
                     k + 1 < g_table.size() ? "," : "");
    }
    std::fprintf(f, "]\n");
    const bool ok = std::fclose(f) == 0;
    if (!ok || std::rename(tmp.c_str(), path) != 0) return fail(FDFB_EINVAL, std::string("cannot write ") + path);
    return FDFB_OK;
}

void ensure_loaded_locked()
{
    if (g_loaded) return;
    g_loaded = true;
    if (const char *p = std::getenv("FDFB_TUNE_CACHE"))
        if (*p) (void)load_locked(p, false);
}

// Seeded fill for the timing buffers (SplitMix64 outputs; the values only
// have to look like accumulators and ModSwitched samples).
uint64_t mix(uint64_t z)
{
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

}  // namespace

namespace fdfbi {

fdfbk::BrPlan tuned_plan(const fdfbk::Geometry &G, uint32_t A)
{
    std::lock_guard<std::mutex> lk(g_mu);
    ensure_loaded_locked();
    if (g_table.empty()) return fdfbk::BrPlan{};
    const uint32_t cus = device_cus();
    for (const Entry &e : g_table)
        if (same_key(e, cus, G, A) && fdfbk::br_plan_valid(G, e.plan)) return e.plan;
    return fdfbk::BrPlan{};
}

}  // namespace fdfbi

static_assert(sizeof(fdfb_br_plan) == 16, "plan layout: form, round, ms");

extern "C" {

int fdfb_br_plans(fdfb_ctx *c, fdfb_br_plan *plans, uint32_t *count)
{
    return guarded([&]() -> int {
        if (!c || !count) return fail(FDFB_EINVAL, "null argument");
        if (!c->mfma_ok) return fail(FDFB_ENOTSUP, "no batched blind rotation for this parameter set");
        fdfbk::BrPlan buf[16];
        const int k = fdfbk::br_plan_candidates(c->geom, buf, 16);
        if (plans)
            for (int i = 0; i < k && i < (int)*count; ++i) plans[i] = fdfb_br_plan{buf[i].form, buf[i].round, 0.0};
        const bool fits = !plans || (uint32_t)k <= *count;
        *count = (uint32_t)k;
        return fits ? FDFB_OK : fail(FDFB_EINVAL, "plan buffer too small");
    });
}

int fdfb_br_set_plan(fdfb_ctx *c, uint32_t A, const fdfb_br_plan *plan)
{
    return guarded([&]() -> int {
        if (!c || !A) return fail(FDFB_EINVAL, "null context or A = 0");
        if (!c->mfma_ok) return fail(FDFB_ENOTSUP, "no batched blind rotation for this parameter set");
        const uint32_t cus = device_cus();
        std::lock_guard<std::mutex> lk(g_mu);
        ensure_loaded_locked();
        if (!plan) {
            g_table.erase(std::remove_if(g_table.begin(), g_table.end(),
                                         [&](const Entry &e) { return same_key(e, cus, c->geom, A); }),
                          g_table.end());
            return FDFB_OK;
        }
        const fdfbk::BrPlan p{plan->form, plan->round};
        if (!fdfbk::br_plan_valid(c->geom, p)) return fail(FDFB_EINVAL, "plan not available for this geometry");
        const fdfbk::Geometry &G = c->geom;
        put(Entry{cus, (uint32_t)G.N, (uint32_t)G.g_ell, (uint32_t)fdfbk::digit_chunks(G.g_log2B), (uint32_t)G.n, A, p,
                  plan->ms});
        return FDFB_OK;
    });
}

int fdfb_br_get_plan(fdfb_ctx *c, uint32_t A, fdfb_br_plan *plan)
{
    return guarded([&]() -> int {
        if (!c || !plan) return fail(FDFB_EINVAL, "null argument");
        const fdfbk::BrPlan p = fdfbi::tuned_plan(c->geom, A);
        double ms = 0.0;
        {
            std::lock_guard<std::mutex> lk(g_mu);
            const uint32_t cus = device_cus();
            for (const Entry &e : g_table)
                if (same_key(e, cus, c->geom, A)) ms = e.ms;
        }
        *plan = fdfb_br_plan{p.form, p.round, ms};
        return FDFB_OK;
    });
}

int fdfb_autotune(fdfb_ctx *c, uint32_t A, uint32_t per, uint32_t reps, fdfb_br_plan *best, fdfb_br_plan *tried,
                  uint32_t *ntried)
{
    return guarded([&]() -> int {
        if (!c || !best || !A || !per || !reps) return fail(FDFB_EINVAL, "null context or best, or A, per, reps = 0");
        std::lock_guard<std::recursive_mutex> lk(c->mu);
        if (!c->mfma_ok) return fail(FDFB_ENOTSUP, "no batched blind rotation for this parameter set");
        if (int rc = fdfbi::ensure_device(*c)) return rc;
        const fdfbk::Geometry &G = c->geom;
        fdfbk::BrPlan cand[16];
        const int nc = std::min(fdfbk::br_plan_candidates(G, cand, 16), 16);
        // timing buffers: A accumulators, their samples' rows, a work counter
        const size_t acc_words = (size_t)A * 2 * G.N, rows = (A + per - 1) / per, row_words = rows * (G.n + 1);
        std::vector<uint32_t> h(std::max(acc_words, row_words));
        uint32_t *d_acc = nullptr, *d_ctN = nullptr, *d_work = nullptr;
        hipStream_t st = nullptr;
        hipEvent_t e0 = nullptr, e1 = nullptr;
        auto done = [&](int rc) {
            if (st) (void)hipStreamSynchronize(st);
            for (void *p : {(void *)d_acc, (void *)d_ctN, (void *)d_work})
                if (p) (void)hipFree(p);
            if (e0) (void)hipEventDestroy(e0);
            if (e1) (void)hipEventDestroy(e1);
            if (st) (void)hipStreamDestroy(st);
            return rc;
        };
        hipError_t e = hipMalloc((void **)&d_acc, acc_words * 4);
        if (e == hipSuccess) e = hipMalloc((void **)&d_ctN, row_words * 4);
        if (e == hipSuccess) e = hipMalloc((void **)&d_work, fdfbi::kWorkWords * 4);
        if (e == hipSuccess) {
            for (size_t k = 0; k < acc_words; ++k) h[k] = (uint32_t)mix(k);
            e = hipMemcpy(d_acc, h.data(), acc_words * 4, hipMemcpyHostToDevice);
        }
        if (e == hipSuccess) {
            for (size_t k = 0; k < row_words; ++k) h[k] = (uint32_t)(mix(k + (1ull << 40)) % (2 * (uint64_t)G.N));
            e = hipMemcpy(d_ctN, h.data(), row_words * 4, hipMemcpyHostToDevice);
        }
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreate(&e0);
        if (e == hipSuccess) e = hipEventCreate(&e1);
        if (e != hipSuccess) return done(fail(FDFB_EDEVICE, std::string("autotune buffers: ") + hipGetErrorString(e)));
        int bi = -1;
        double bms = 0.0;
        std::vector<fdfb_br_plan> all;
        for (int k = 0; k < nc; ++k) {
            const fdfbk::BrPlan &p = cand[k];
            auto run = [&] {
                return fdfbk::launch_br_kara(G, d_acc, d_ctN, A, per, c->d_brk_frag, c->d_brk_corr, p, d_work, st);
            };
            e = run();  // warm-up (kernel attributes, caches)
            if (e == hipSuccess) e = hipEventRecord(e0, st);
            for (uint32_t r = 0; r < reps && e == hipSuccess; ++r) e = run();
            if (e == hipSuccess) e = hipEventRecord(e1, st);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float t = 0.f;
            if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
            if (e != hipSuccess) return done(fail(FDFB_EDEVICE, std::string("autotune run: ") + hipGetErrorString(e)));
            const double ms = (double)t / reps;
            all.push_back(fdfb_br_plan{p.form, p.round, ms});
            if (bi < 0 || ms < bms) {
                bi = k;
                bms = ms;
            }
        }
        *best = fdfb_br_plan{cand[bi].form, cand[bi].round, bms};
        if (ntried) {
            if (tried)
                for (size_t k = 0; k < all.size() && k < *ntried; ++k) tried[k] = all[k];
            *ntried = (uint32_t)all.size();
        }
        {
            std::lock_guard<std::mutex> tl(g_mu);
            ensure_loaded_locked();
            put(Entry{device_cus(), (uint32_t)G.N, (uint32_t)G.g_ell, (uint32_t)fdfbk::digit_chunks(G.g_log2B),
                      (uint32_t)G.n, A, cand[bi], bms});
            if (const char *path = std::getenv("FDFB_TUNE_CACHE"))
                if (*path)
                    if (int rc = save_locked(path)) return done(rc);
        }
        return done(FDFB_OK);
    });
}

int fdfb_autotune_bootstrap(fdfb_ctx *c, uint32_t B, uint32_t L, uint32_t reps, fdfb_br_plan *sign_best,
                            fdfb_br_plan *func_best, fdfb_br_plan *tried, uint32_t *ntried)
{
    return guarded([&]() -> int {
        if (!c || !sign_best || !func_best || !B || !L || !reps)
            return fail(FDFB_EINVAL, "null context or result, or B, L, reps = 0");
        std::lock_guard<std::recursive_mutex> lk(c->mu);
        if (!c->mfma_ok) return fail(FDFB_ENOTSUP, "no batched blind rotation for this parameter set");
        if (c->nluts < 1) return fail(FDFB_EINVAL, "register a table first (the timing batch uses table 0)");
        if ((uint64_t)B * L > 0xFFFFFFFFu) return fail(FDFB_EINVAL, "too many table evaluations");
        if (int rc = fdfbi::ensure_device(*c)) return rc;
        const fdfbk::Geometry &G = c->geom;
        const uint32_t As = B * (uint32_t)G.boot_ell, Af = B * L;
        fdfbk::BrPlan cand[16];
        const int nc = std::min(fdfbk::br_plan_candidates(G, cand, 16), 16);
        // a timing batch: random samples (their outputs are never read), table 0
        const size_t in_words = (size_t)B * (G.n + 1), out_words = (size_t)Af * (G.n + 1);
        const size_t sbytes = fdfbi::scratch_bytes(c->P, B, L);
        uint32_t *d_cts = nullptr, *d_out = nullptr;
        int32_t *d_ids = nullptr;
        void *d_scr = nullptr;
        hipStream_t st = nullptr;
        hipEvent_t e0 = nullptr, e1 = nullptr;
        const uint32_t cus = device_cus();
        // the table entries this search may overwrite, restored on failure
        std::vector<Entry> saved;
        {
            std::lock_guard<std::mutex> tl(g_mu);
            ensure_loaded_locked();
            saved = g_table;
        }
        auto done = [&](int rc) {
            if (st) (void)hipStreamSynchronize(st);
            for (void *p : {(void *)d_cts, (void *)d_out, (void *)d_ids, d_scr})
                if (p) (void)hipFree(p);
            if (e0) (void)hipEventDestroy(e0);
            if (e1) (void)hipEventDestroy(e1);
            if (st) (void)hipStreamDestroy(st);
            if (rc) {
                std::lock_guard<std::mutex> tl(g_mu);
                g_table = saved;
            }
            return rc;
        };
        hipError_t e = hipMalloc((void **)&d_cts, in_words * 4);
        if (e == hipSuccess) e = hipMalloc((void **)&d_out, out_words * 4);
        if (e == hipSuccess) e = hipMalloc((void **)&d_ids, (size_t)Af * 4);
        if (e == hipSuccess) e = hipMalloc(&d_scr, sbytes);
        if (e == hipSuccess) {
            std::vector<uint32_t> h(in_words);
            for (size_t k = 0; k < in_words; ++k) h[k] = (uint32_t)mix(k + (3ull << 40));
            e = hipMemcpy(d_cts, h.data(), in_words * 4, hipMemcpyHostToDevice);
        }
        if (e == hipSuccess) e = hipMemset(d_ids, 0, (size_t)Af * 4);
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreate(&e0);
        if (e == hipSuccess) e = hipEventCreate(&e1);
        if (e != hipSuccess) return done(fail(FDFB_EDEVICE, std::string("autotune buffers: ") + hipGetErrorString(e)));
        const fdfbi::ScratchView sc = fdfbi::carve_scratch(c->P, B, L, d_scr);
        auto set = [&](uint32_t A, const fdfbk::BrPlan &p, double ms) {
            std::lock_guard<std::mutex> tl(g_mu);
            put(Entry{cus, (uint32_t)G.N, (uint32_t)G.g_ell, (uint32_t)fdfbk::digit_chunks(G.g_log2B), (uint32_t)G.n,
                      A, p, ms});
        };
        // milliseconds per bootstrap batch with the current table
        auto time_batch = [&](double *ms) -> int {
            int rc = fdfbi::enqueue_bootstrap(*c, sc, d_cts, d_ids, B, d_out, 0, st, L, false);  // warm-up
            if (rc) return rc;
            if ((e = hipEventRecord(e0, st)) != hipSuccess) return fail(FDFB_EDEVICE, hipGetErrorString(e));
            for (uint32_t r = 0; r < reps; ++r)
                if ((rc = fdfbi::enqueue_bootstrap(*c, sc, d_cts, d_ids, B, d_out, 0, st, L, false))) return rc;
            if ((e = hipEventRecord(e1, st)) != hipSuccess || (e = hipEventSynchronize(e1)) != hipSuccess)
                return fail(FDFB_EDEVICE, hipGetErrorString(e));
            float t = 0.f;
            if ((e = hipEventElapsedTime(&t, e0, e1)) != hipSuccess) return fail(FDFB_EDEVICE, hipGetErrorString(e));
            *ms = (double)t / reps;
            return FDFB_OK;
        };
        {  // both phases start from the fixed rule
            std::lock_guard<std::mutex> tl(g_mu);
            g_table.erase(std::remove_if(g_table.begin(), g_table.end(),
                                         [&](const Entry &x) {
                                             return same_key(x, cus, G, As) || same_key(x, cus, G, Af);
                                         }),
                          g_table.end());
        }
        std::vector<fdfb_br_plan> all;
        // one phase at a time (the other keeps its current plan); with As == Af
        // one plan serves both phases and they are searched together
        const uint32_t phases[2] = {As, Af};
        fdfb_br_plan best[2] = {};
        for (int ph = 0; ph < (As == Af ? 1 : 2); ++ph) {
            int bi = -1;
            double bms = 0.0;
            for (int k = 0; k < nc; ++k) {
                set(phases[ph], cand[k], 0.0);
                double ms = 0.0;
                if (int rc = time_batch(&ms)) return done(rc);
                all.push_back(fdfb_br_plan{cand[k].form, cand[k].round, ms});
                if (bi < 0 || ms < bms) {
                    bi = k;
                    bms = ms;
                }
            }
            set(phases[ph], cand[bi], bms);
            best[ph] = fdfb_br_plan{cand[bi].form, cand[bi].round, bms};
        }
        if (As == Af) best[1] = best[0];
        *sign_best = best[0];
        *func_best = best[1];
        if (ntried) {
            if (tried)
                for (size_t k = 0; k < all.size() && k < *ntried; ++k) tried[k] = all[k];
            *ntried = (uint32_t)all.size();
        }
        if (const char *path = std::getenv("FDFB_TUNE_CACHE"))
            if (*path) {
                std::lock_guard<std::mutex> tl(g_mu);
                if (int rc = save_locked(path)) return done(rc);
            }
        return done(FDFB_OK);
    });
}

int fdfb_tune_save(const char *path)
{
    return guarded([&]() -> int {
        if (!path) return fail(FDFB_EINVAL, "null path");
        std::lock_guard<std::mutex> lk(g_mu);
        ensure_loaded_locked();
        return save_locked(path);
    });
}

int fdfb_tune_load(const char *path)
{
    return guarded([&]() -> int {
        if (!path) return fail(FDFB_EINVAL, "null path");
        std::lock_guard<std::mutex> lk(g_mu);
        ensure_loaded_locked();
        return load_locked(path, true);
    });
}

int fdfb_tune_clear(void)
{
    return guarded([&]() -> int {
        std::lock_guard<std::mutex> lk(g_mu);
        g_table.clear();
        g_loaded = true;  // an explicit clear also drops what the cache file held
        return FDFB_OK;
    });
}

}  // extern "C"
