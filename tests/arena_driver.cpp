// The serving engine's first-fit arena (fdfbi::Arena) against a shadow model
// of its block, over random allocation and release sequences; prints "ok"
// when every check holds.  Built and run by tests/test_host_logic.py on the CPU.
#include <cstdio>
#include <random>
#include <utility>
#include <vector>

#include "arena.h"

static int fails = 0;
#define CHECK(c, ...)                                           \
    do {                                                        \
        if (!(c)) {                                             \
            if (fails++ < 20) {                                 \
                std::printf("FAIL %s:%d: ", __FILE__, __LINE__); \
                std::printf(__VA_ARGS__);                       \
                std::printf("\n");                              \
            }                                                   \
        }                                                       \
    } while (0)

// lowest offset of a run of `units` free units in the shadow map, or -1
static long first_fit(const std::vector<char> &used, size_t units)
{
    size_t run = 0;
    for (size_t u = 0; u < used.size(); ++u) {
        run = used[u] ? 0 : run + 1;
        if (run == units) return (long)(u + 1 - units);
    }
    return -1;
}

int main()
{
    const size_t unit = 256;
    std::mt19937_64 rng(31);
    for (int c = 0; c < 400; ++c) {
        const size_t units = 1 + rng() % 200;
        fdfbi::Arena a;
        a.reset(units * unit);
        std::vector<char> used(units, 0);
        std::vector<std::pair<size_t, size_t>> live;  // (offset, bytes)
        for (int op = 0; op < 300; ++op) {
            if (live.empty() || rng() % 5 < 3) {
                const size_t want = 1 + rng() % std::max<size_t>(1, units / 3);
                size_t off = 0;
                const bool ok = a.alloc(want * unit, &off);
                const long ff = first_fit(used, want);
                CHECK(ok == (ff >= 0), "case %d op %d: alloc of %zu units %s, shadow %ld", c, op, want,
                      ok ? "succeeded" : "failed", ff);
                if (ok) {
                    CHECK(ff >= 0 && off == (size_t)ff * unit, "case %d op %d: offset %zu, first fit %ld", c, op,
                          off / unit, ff);
                    CHECK(off % unit == 0 && off + want * unit <= units * unit, "case %d: range outside", c);
                    for (size_t u = off / unit; u < off / unit + want && u < units; ++u) {
                        CHECK(!used[u], "case %d op %d: unit %zu handed out twice", c, op, u);
                        used[u] = 1;
                    }
                    live.push_back({off, want * unit});
                }
            } else {
                const size_t k = rng() % live.size();
                a.release(live[k].first, live[k].second);
                for (size_t u = live[k].first / unit; u < (live[k].first + live[k].second) / unit; ++u) used[u] = 0;
                live.erase(live.begin() + (long)k);
            }
            // the free ranges are exactly the maximal free runs of the shadow map
            std::vector<std::pair<size_t, size_t>> runs;
            for (size_t u = 0; u < units;) {
                if (used[u]) {
                    ++u;
                    continue;
                }
                size_t v = u;
                while (v < units && !used[v]) ++v;
                runs.push_back({u * unit, (v - u) * unit});
                u = v;
            }
            std::vector<std::pair<size_t, size_t>> got(a.free_ranges().begin(), a.free_ranges().end());
            CHECK(got == runs, "case %d op %d: %zu free ranges, shadow has %zu", c, op, got.size(), runs.size());
        }
        for (auto &l : live) a.release(l.first, l.second);
        CHECK(a.free_ranges().size() == 1 && a.free_ranges().begin()->first == 0 &&
                  a.free_ranges().begin()->second == units * unit,
              "case %d: not one block after releasing everything", c);
    }
    std::printf(fails ? "%d failures\n" : "ok\n", fails);
    return fails ? 1 : 0;
}
