// Reads server step cases on stdin and prints the sweeps ea::step_sweeps gives.
// Case: "n cus pack quantum max_sweeps", then n lines "ladders work left urgency".
#include <cstdio>
#include <vector>

#include "ea_sched.h"

int main()
{
    int n, cus, pack, quantum, max_sweeps;
    while (std::scanf("%d %d %d %d %d", &n, &cus, &pack, &quantum, &max_sweeps) == 5) {
        std::vector<ea::StepJob> jobs(n);
        for (ea::StepJob &j : jobs) {
            long long ladders, left;
            if (std::scanf("%lld %lf %lld %lf", &ladders, &j.work, &left, &j.urgency) != 4) return 1;
            j.ladders = ladders;
            j.left = left;
        }
        const std::vector<int> q = ea::step_sweeps(jobs, quantum, cus, pack != 0, max_sweeps);
        for (int k = 0; k < n; ++k) std::printf("%d%c", q[k], k + 1 < n ? ' ' : '\n');
    }
    return 0;
}
