// Schedule of a sequence of bootstrap jobs as a software pipeline over
// persistent work-queue launches (host logic only, no device calls).
//
// Each launch takes the function rotations of the jobs whose public mux is
// already enqueued, then the sign rotations of the next jobs in job order, up
// to `rounds` rounds of the kernel's resident capacity.  A job's sign
// accumulators may be split between launches at whole samples and whole
// work items.  After a launch come the outputs of the jobs whose function
// rotation it ran, then the public mux of the jobs whose sign rotations it
// completed; their function rotations go into the next launch.
#pragma once
#include <algorithm>
#include <cstdint>
#include <numeric>
#include <vector>

namespace fdfbp {

// Work items of the persistent kernel for `accs` accumulators: four
// accumulators per item for a narrow geometry (N <= 1024), one for a wide one.
inline uint32_t work_items(bool wide, uint64_t accs) { return (uint32_t)(wide ? accs : (accs + 3) / 4); }

// A job as the schedule sees it: B samples, `per` sign accumulators per
// sample (ell_boot), and whether its geometry is wide.
struct Job {
    uint32_t B = 0, per = 1;
    bool wide = false;
};

// Accumulators [a0, a0 + A) of a job's sign rotations, or (sign false) its
// whole function rotation (a0 = 0, A = B).
struct Range {
    uint32_t job;
    bool sign;
    uint32_t a0, A;
};

// One launch: the jobs whose ModSwitch and sign accumulators are enqueued
// just before it, its ranges, then the jobs whose output follows it and the
// jobs whose public mux follows it (in that order).
struct Launch {
    std::vector<uint32_t> fronts;
    std::vector<Range> ranges;
    std::vector<uint32_t> backs, mids;
};

// cap: workgroups of the persistent kernel resident at once (> 0); rounds:
// rounds of cap per launch (> 0).  Jobs with B = 0 are skipped.
inline std::vector<Launch> schedule(const std::vector<Job> &jobs, uint32_t cap, uint32_t rounds)
{
    std::vector<Launch> plan;
    const uint32_t njobs = (uint32_t)jobs.size();
    const uint64_t target = (uint64_t)rounds * cap;
    std::vector<uint32_t> s_next(njobs, 0);  // sign accumulators of each job scheduled so far
    std::vector<uint32_t> ready;             // jobs whose public mux is enqueued
    uint32_t ks = 0;                         // first job with sign accumulators left to schedule
    for (;;) {
        Launch L;
        uint64_t items = 0;
        for (uint32_t k : ready) {
            L.ranges.push_back({k, false, 0, jobs[k].B});
            items += work_items(jobs[k].wide, jobs[k].B);
            L.backs.push_back(k);
        }
        ready.clear();
        const uint64_t goal = std::max(target, (items + cap - 1) / cap * cap);
        while (ks < njobs && items < goal) {
            const Job &j = jobs[ks];
            if (!j.B) {
                ++ks;
                continue;
            }
            const uint32_t total = j.B * j.per;
            // cut points: whole samples, and whole items of a narrow geometry
            const uint32_t gran = j.wide ? j.per : std::lcm(4u, j.per);
            const uint64_t room = j.wide ? goal - items : (goal - items) * 4;
            uint32_t take = total - s_next[ks];
            if (take > room) take = (uint32_t)(room / gran * gran);
            if (!take) {
                if (!L.ranges.empty()) break;                 // the launch is full to a cut point
                take = std::min(total - s_next[ks], gran);  // never an empty launch
            }
            if (s_next[ks] == 0) L.fronts.push_back(ks);  // the job's first sign accumulators
            L.ranges.push_back({ks, true, s_next[ks], take});
            items += work_items(j.wide, take);
            s_next[ks] += take;
            if (s_next[ks] == total) {
                L.mids.push_back(ks);
                ++ks;
            }
        }
        if (L.ranges.empty()) break;
        ready = L.mids;
        plan.push_back(std::move(L));
    }
    return plan;
}

}  // namespace fdfbp
