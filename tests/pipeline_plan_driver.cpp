// Invariants of the software-pipeline schedule (fdfbp::schedule) over random
// job mixes; prints "ok" when every case holds.  Built and run by
// tests/test_host_logic.py on the CPU.
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "pipeline_plan.h"

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

static void check_case(const std::vector<fdfbp::Job> &jobs, uint32_t cap, uint32_t rounds, int id)
{
    const auto plan = fdfbp::schedule(jobs, cap, rounds);
    const size_t nj = jobs.size();
    const int NONE = -1;
    std::vector<int> front_at(nj, NONE), first_s(nj, NONE), last_s(nj, NONE), mid_at(nj, NONE), f_at(nj, NONE),
        back_at(nj, NONE);
    std::vector<uint64_t> covered(nj, 0);
    int prev_sign_job = -1;
    uint32_t max_per = 1;
    uint64_t total_items = 0, want_items = 0;
    for (const auto &j : jobs) {
        max_per = std::max(max_per, j.per);
        if (j.B) want_items += fdfbp::work_items(j.wide, j.B);
    }
    for (size_t L = 0; L < plan.size(); ++L) {
        const auto &l = plan[L];
        CHECK(!l.ranges.empty(), "case %d launch %zu empty", id, L);
        for (uint32_t k : l.fronts) {
            CHECK(front_at[k] == NONE, "case %d job %u front twice", id, k);
            front_at[k] = (int)L;
        }
        uint64_t items = 0;
        bool any_sign = false;
        for (const auto &r : l.ranges) {
            const auto &j = jobs[r.job];
            CHECK(j.B > 0, "case %d empty job %u scheduled", id, r.job);
            CHECK(r.A > 0, "case %d empty range", id);
            items += fdfbp::work_items(j.wide, r.A);
            if (r.sign) {
                any_sign = true;
                CHECK((int)r.job >= prev_sign_job, "case %d sign ranges out of job order", id);
                prev_sign_job = (int)r.job;
                CHECK(front_at[r.job] != NONE && front_at[r.job] <= (int)L, "case %d job %u rotated before its front",
                      id, r.job);
                CHECK(r.a0 == covered[r.job], "case %d job %u sign range not contiguous", id, r.job);
                CHECK(r.a0 % j.per == 0, "case %d job %u cut inside a sample", id, r.job);
                CHECK(j.wide || r.a0 % 4 == 0, "case %d job %u cut inside a work item", id, r.job);
                covered[r.job] += r.A;
                if (first_s[r.job] == NONE) first_s[r.job] = (int)L;
                last_s[r.job] = (int)L;
            } else {
                CHECK(r.a0 == 0 && r.A == j.B, "case %d job %u partial function rotation", id, r.job);
                CHECK(f_at[r.job] == NONE, "case %d job %u function rotation twice", id, r.job);
                CHECK(mid_at[r.job] != NONE && mid_at[r.job] < (int)L,
                      "case %d job %u function rotation before its public mux", id, r.job);
                f_at[r.job] = (int)L;
            }
        }
        for (uint32_t k : l.backs) {
            CHECK(f_at[k] == (int)L, "case %d job %u output not after its function rotation", id, k);
            back_at[k] = (int)L;
        }
        for (uint32_t k : l.mids) {
            CHECK(covered[k] == (uint64_t)jobs[k].B * jobs[k].per, "case %d job %u mux before its sign rotations end",
                  id, k);
            CHECK(last_s[k] == (int)L, "case %d job %u mux not after its last sign launch", id, k);
            CHECK(mid_at[k] == NONE, "case %d job %u mux twice", id, k);
            mid_at[k] = (int)L;
        }
        // a launch followed by more sign work holds at least `rounds` rounds,
        // short of one sample's accumulators at most
        bool more_sign = false;
        for (size_t L2 = L + 1; L2 < plan.size() && !more_sign; ++L2)
            for (const auto &r : plan[L2].ranges) more_sign |= r.sign;
        if (more_sign && any_sign)
            CHECK(items + max_per > (uint64_t)rounds * cap, "case %d launch %zu short: %llu items", id, L,
                  (unsigned long long)items);
        total_items += items;
    }
    for (size_t k = 0; k < nj; ++k) {
        if (!jobs[k].B) {
            CHECK(front_at[k] == NONE && f_at[k] == NONE, "case %d empty job %zu scheduled", id, k);
            continue;
        }
        CHECK(covered[k] == (uint64_t)jobs[k].B * jobs[k].per, "case %d job %zu sign coverage", id, k);
        CHECK(front_at[k] == first_s[k], "case %d job %zu front not with its first sign range", id, k);
        CHECK(f_at[k] != NONE && back_at[k] == f_at[k], "case %d job %zu function rotation or output missing", id, k);
    }
    uint64_t sign_items = 0;
    for (const auto &l : plan)
        for (const auto &r : l.ranges)
            if (r.sign) sign_items += fdfbp::work_items(jobs[r.job].wide, r.A);
    CHECK(total_items == want_items + sign_items, "case %d item total", id);
}

int main()
{
    std::mt19937_64 rng(2109);
    // the bench shape: 16 batches of 1024 at N = 1024 with two sign rotations per sample
    for (uint32_t rounds : {1u, 2u, 4u, 8u}) {
        std::vector<fdfbp::Job> jobs(16, fdfbp::Job{1024, 2, false});
        const auto plan = fdfbp::schedule(jobs, 512, rounds);
        size_t full = 0;
        for (const auto &l : plan) {
            uint64_t items = 0;
            for (const auto &r : l.ranges) items += fdfbp::work_items(false, r.A);
            full += items % 512 == 0;
        }
        // every launch but the first and last is whole rounds, and nothing is left over
        CHECK(full + 2 >= plan.size(), "bench shape rounds %u: %zu of %zu launches whole", rounds, full, plan.size());
        check_case(jobs, 512, rounds, -(int)rounds);
    }
    for (int id = 0; id < 3000; ++id) {
        const size_t nj = rng() % 24;
        std::vector<fdfbp::Job> jobs(nj);
        for (auto &j : jobs) {
            const uint32_t r = rng() % 10;
            j.B = r == 0 ? 0 : (r < 4 ? 1 + rng() % 8 : 1 + rng() % 3000);
            j.per = 1 + rng() % 5;
            j.wide = rng() % 3 == 0;
        }
        const uint32_t caps[] = {1, 2, 3, 7, 64, 512};
        check_case(jobs, caps[rng() % 6], 1 + rng() % 8, id);
    }
    std::printf(fails ? "%d failures\n" : "ok\n", fails);
    return fails ? 1 : 0;
}
