"""Host logic of the serving loop's step sizes (ea_sched.h), on the CPU.

The server runs every job of a step for sweeps worth about one unit time T
(`quantum` sweeps of the job with the most work per ladder sweep), one
workgroup per ladder at a time on each compute unit, longest units first.  With
packing on and more ladders than compute units, the least urgent jobs run
units of T / m so that the step takes floor(ladders / CUs) rounds where equal
units need one more.  These tests drive ea::step_sweeps through a small
program built with g++ and check it against a list-scheduling simulation of
the launch written here."""
import heapq
import math
import os
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def stepper(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    out = tmp_path_factory.mktemp("sched") / "step_sweeps"
    subprocess.run([gxx, "-O1", "-std=c++17", "-I", os.path.join(ROOT, "paper_1311_5582_amd", "csrc"), "-o",
                    str(out), os.path.join(ROOT, "tests", "helpers", "step_sweeps.cpp")], check=True)

    def run(cases, cus, pack, quantum=200, max_sweeps=1 << 20):
        text = ""
        for jobs in cases:
            text += f"{len(jobs)} {cus} {int(pack)} {quantum} {max_sweeps}\n"
            for lad, work, left, urg in jobs:
                text += f"{lad} {work!r} {left} {urg!r}\n"
        res = subprocess.run([str(out)], input=text, capture_output=True, text=True, check=True)
        return [[int(x) for x in line.split()] for line in res.stdout.splitlines()]

    return run


def equal_units(jobs, quantum=200, max_sweeps=1 << 20):
    """Sweeps with every unit about T (halves round away from zero, as in C++)."""
    w_max = max(w for _, w, _, _ in jobs)
    return [min(left, max(1, min(max_sweeps, math.floor(quantum * w_max / w + 0.5)))) for _, w, left, _ in jobs]


def makespan(jobs, sweeps, cus, quantum=200):
    """Greedy list scheduling of the launch: units sorted by length (longest
    first), each started on the compute unit that frees first; time in units
    of T (quantum sweeps of the job with the most work per sweep)."""
    w_max = max(w for _, w, _, _ in jobs)
    units = []
    for (lad, w, _, _), q in zip(jobs, sweeps):
        units += [q * w / (quantum * w_max)] * lad
    units.sort(reverse=True)
    free = [0.0] * cus
    for u in units:
        heapq.heapreplace(free, free[0] + u)
    return max(free)


def test_equal_units_without_packing_or_spare_rounds(stepper):
    """Packing off, one round or less, or whole rounds: every unit about T."""
    mix = [(750, 19 ** 3 * 29.0, 10 ** 6, 1.3), (64, 10 ** 3 * 16.0, 10 ** 6, 1.0)]
    one_round = [(100, 8 ** 3 * 16.0, 10 ** 6, 2.0), (120, 12 ** 3 * 20.0, 10 ** 6, 1.0)]
    whole = [(256, 16 ** 3 * 32.0, 10 ** 6, 1.0), (256, 12 ** 3 * 32.0, 10 ** 6, 3.0)]
    assert stepper([mix], 256, False) == [equal_units(mix)]
    assert stepper([one_round, whole, [mix[0]]], 256, True) == [equal_units(one_round), equal_units(whole),
                                                                equal_units([mix[0]])]


def test_least_urgent_job_fills_the_last_round(stepper):
    """A 750-ladder job and a 64-ladder one on 256 CUs: equal units need 4
    rounds; packed, the small job (less urgent) runs units of T / 4 in the 18
    idle slots of the launch's third round (18 x 4 >= 64), the big one keeps
    its full share.
    Made more urgent, the small job keeps its share and the big one is cut."""
    big, small = 19 ** 3 * 29.0, 10 ** 3 * 16.0
    jobs = [(750, big, 10 ** 6, 1.3), (64, small, 10 ** 6, 1.0)]
    q = stepper([jobs], 256, True)[0]
    base = equal_units(jobs)
    assert q[0] == base[0] == 200
    assert q[1] == math.floor(200 * big / small / 4 + 0.5)
    assert makespan(jobs, base, 256) == pytest.approx(4.0, rel=0.01)
    assert makespan(jobs, q, 256) <= 3.0 * 1.01
    flipped = [(750, big, 10 ** 6, 1.0), (64, small, 10 ** 6, 1.3)]
    q2 = stepper([flipped], 256, True)[0]
    # idle slots 768 - 64 = 704 < 750 -> the big job's units are halved
    assert q2 == [100, math.floor(200 * big / small + 0.5)]
    assert makespan(flipped, q2, 256) <= 3.0 * 1.01


def test_sweeps_bounded_by_what_is_left(stepper):
    jobs = [(750, 19 ** 3 * 29.0, 37, 1.3), (64, 10 ** 3 * 16.0, 5, 1.0)]
    q = stepper([jobs], 256, True)[0]
    assert q == [37, 5]


@pytest.mark.parametrize("seed", range(6))
def test_packing_never_lengthens_a_step_and_keeps_the_most_urgent(stepper, seed):
    """Random job sets (2..8 jobs, 32..1024 ladders, L 6..20, n_T 16..48) on
    256 and 64 CUs: the packed step is never longer than the equal-unit one,
    is shorter whenever it packs and takes floor(ladders / CUs) rounds when the
    idle slots of those rounds hold the short units, the most urgent job keeps
    its full sweeps, and every cut job is cut to T / m with m in 2..4, the same
    m for all of them."""
    rng = np.random.default_rng(1000 + seed)
    sets = []
    for _ in range(40):
        n = int(rng.integers(2, 9))
        sets.append([(int(rng.integers(16, 513)) * 2, float(int(rng.integers(6, 21)) ** 3 * int(rng.integers(16, 49))),
                      10 ** 7, float(rng.uniform(1.0, 5.0))) for _ in range(n)])
    for cus in (256, 64):
        for jobs, q in zip(sets, stepper(sets, cus, True)):
            base = equal_units(jobs)
            total = sum(j[0] for j in jobs)
            t_base = makespan(jobs, base, cus)
            t_pack = makespan(jobs, q, cus)
            assert t_pack <= t_base * 1.01 + 1e-9
            top = max(range(len(jobs)), key=lambda k: jobs[k][3])
            assert q[top] == base[top]
            cut = [k for k in range(len(jobs)) if q[k] != base[k]]
            if cut:
                ratios = {round(base[k] / q[k]) for k in cut}
                assert len(ratios) == 1 and ratios <= {2, 3, 4}, ratios
                # the cut jobs are the least urgent ones
                assert max(jobs[k][3] for k in cut) <= min(jobs[k][3] for k in range(len(jobs)) if k not in cut)
                assert t_pack < t_base
                m = ratios.pop()
                kept = sum(jobs[k][0] for k in range(len(jobs)) if k not in cut)
                idle = total // cus * cus - kept
                if total - kept <= m * idle:
                    assert t_pack <= (total // cus) * 1.02 + 1e-9
            else:
                assert q == base
