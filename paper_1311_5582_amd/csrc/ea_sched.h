// Sweeps per job for one step of the serving loop (host code only).
//
// A step is one launch over the running jobs' ladders, one workgroup per
// ladder at a time on each compute unit, the longest units first.  Every job
// first gets sweeps worth about the time T of `quantum` sweeps of the job with
// the most work per ladder sweep (work = L^3 x n_T), so that all units are of
// one length.  With more ladders than compute units the launch then takes
// ceil(ladders / CUs) rounds of T, the last one partly idle.  With packing on,
// the least urgent jobs (lowest response ratio first, never all of them) run
// units of T / m instead: the others then fit floor(ladders / CUs) rounds, and
// every idle slot of length T in those rounds holds m of the short units, m
// the smallest count that holds them all (at most 4: with fewer idle slots
// than that needs, the short units run past the full rounds, still in fewer
// rounds than equal units take).  The other jobs keep their full share.
#pragma once

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <numeric>
#include <vector>

namespace ea {

struct StepJob {
    int64_t ladders;   // units of the launch (2 x realizations)
    double work;       // work per ladder sweep (L^3 x n_T)
    int64_t left;      // sweeps the job has left (>= 1)
    double urgency;    // response ratio: the higher, the more it keeps its share
};

constexpr int kMaxUnitSplit = 4;   // a packed unit is at least T / 4

// Fraction of T given to each job's units (1 = full share).
inline std::vector<double> step_shares(const std::vector<StepJob> &jobs, int cus, bool pack)
{
    const size_t n = jobs.size();
    std::vector<double> share(n, 1.0);
    int64_t total = 0;
    for (const StepJob &j : jobs) total += j.ladders;
    if (!pack || n < 2 || cus <= 0 || total <= cus || total % cus == 0) return share;
    const int64_t cap = total / cus * cus;   // unit slots of the full rounds
    std::vector<size_t> order(n);
    std::iota(order.begin(), order.end(), (size_t)0);
    std::stable_sort(order.begin(), order.end(),
                     [&jobs](size_t a, size_t b) { return jobs[a].urgency < jobs[b].urgency; });
    int64_t kept = total, shrunk = 0;
    size_t k = 0;
    for (; k + 1 < n && kept > cap; ++k) {   // the most urgent job always keeps its share
        kept -= jobs[order[k]].ladders;
        shrunk += jobs[order[k]].ladders;
    }
    if (kept > cap || shrunk == 0) return share;   // no set of the others can make room
    const int64_t idle = cap - kept;                // slots of length T left in the full rounds
    const int64_t m = idle > 0 ? std::min<int64_t>(kMaxUnitSplit, (shrunk + idle - 1) / idle) : kMaxUnitSplit;
    if (m <= 1) return share;
    for (size_t i = 0; i < k; ++i) share[order[i]] = 1.0 / (double)m;
    return share;
}

// Sweeps of each job in the step: round(quantum x share x max work / work),
// at least 1, at most max_sweeps and the sweeps it has left.
inline std::vector<int> step_sweeps(const std::vector<StepJob> &jobs, int quantum, int cus, bool pack, int max_sweeps)
{
    double w_max = 0.0;
    for (const StepJob &j : jobs) w_max = std::max(w_max, j.work);
    const std::vector<double> share = step_shares(jobs, cus, pack);
    std::vector<int> q(jobs.size(), 0);
    for (size_t k = 0; k < jobs.size(); ++k) {
        const double want = std::min((double)max_sweeps, std::round(quantum * share[k] * w_max / jobs[k].work));
        q[k] = (int)std::min<int64_t>((int64_t)std::max(1.0, want), jobs[k].left);
    }
    return q;
}

}  // namespace ea
