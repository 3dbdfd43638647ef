"""Parity at volume: the benchmark workloads run on the GPU in their benchmark
launch configurations, and the stored oracle results of
tests/golden/parity_volumes.json (written by make_parity_volumes.py, which
calls only the CPU oracle) are compared bit for bit for every realization the
file holds: final spins (SHA-256 of the int8 array by slot), permutation,
energies and overlaps.

  L16_R64_1000   all 64 realizations, 1000 sweeps, PT every sweep (one launch, split ladders)
  L16_R64_10000  4 realizations of the same job after 10^4 sweeps (ten 1000-sweep launches)
  batched_5000   4 realizations of each of the five uneven jobs after 5000 sweeps of
                 the autotuned graph-captured plan (20 replays of 250 sweeps)
  L24_R256_2000  2 realizations after 2000 sweeps with PT every 10 (200 swap points)
  serving_2000   the 64-job serving trace with sweeps cut to min(sweeps, 2000), through
                 the server; one realization of every job
"""
import hashlib
import json
import os

import numpy as np
import pytest

from paper_1311_5582_amd import binding as B
from paper_1311_5582_amd import inputs
from paper_1311_5582_amd import serve

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "parity_volumes.json")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    B.lib()


@pytest.fixture(scope="module")
def golden():
    with open(GOLDEN) as f:
        return json.load(f)["cases"]


def _sha(a):
    return hashlib.sha256(np.ascontiguousarray(a, dtype=np.int8).tobytes()).hexdigest()


def _check(name, case, spins, perm, E, q, t):
    assert t == case["sweeps"], f"{name}: {t} sweeps done"
    for g in case["realizations"]:
        r = g["r"]
        assert g["t"] == case["sweeps"]
        assert np.array_equal(perm[r], np.array(g["perm"], dtype=np.int32)), f"{name} r={r}: permutation differs"
        assert np.array_equal(E[r], np.array(g["E"], dtype=np.int32)), f"{name} r={r}: energies differ"
        assert np.array_equal(q[r], np.array(g["q"], dtype=np.int32)), f"{name} r={r}: overlaps differ"
        assert _sha(spins[r]) == g["spins_sha256"], f"{name} r={r}: spins differ"


def _job(case):
    J = inputs.couplings(case["L"], case["R"], case["seed"])
    betas = inputs.geometric_betas(case["n_T"], case["t_min"], case["t_max"])
    return J, betas


@pytest.mark.parametrize("name,launch", [("L16_R64_1000", 1000), ("L16_R64_10000", 1000), ("L24_R256_2000", 200)])
def test_single_job_volume(golden, name, launch):
    case = golden[name]
    J, betas = _job(case)
    sim = B.Sim(case["L"], J, betas, case["seed"])
    print(f"[volume] {name}: launches of {launch} sweeps, {sim.info()}", flush=True)
    for _ in range(case["sweeps"] // launch):
        sim.sweep(launch, case["swap_every"])
    s, perm, t = sim.state()
    E, q = sim.observables()
    _check(name, case, s, perm, E, q, t)
    sim.close()


def test_batched_plan_volume(golden):
    names = sorted(k for k in golden if k.startswith("batched_5000/"))
    assert len(names) == len(inputs.BATCHED_JOBS)
    cases = [golden[n] for n in names]
    sims = []
    for c in cases:
        J, betas = _job(c)
        sims.append(B.Sim(c["L"], J, betas, c["seed"]))
    plan = B.Plan(sims, 250, [c["swap_every"] for c in cases], autotune=True)
    print(f"[volume] batched plan {plan.info()}", flush=True)
    plan.run(cases[0]["sweeps"] // 250)
    for n, c, sim in zip(names, cases, sims):
        s, perm, t = sim.state()
        E, q = sim.observables()
        _check(n, c, s, perm, E, q, t)
    plan.close()
    for sim in sims:
        sim.close()


def test_serving_trace_volume(golden):
    trace = inputs.serving_trace(n_jobs=64, rate_per_s=20.0)
    for j in trace:
        j["sweeps"] = min(j["sweeps"], 2000)
    srv = B.Server(quantum_sweeps=200, keep_state=True)
    checked = []

    def on_done(jid, j, st):
        assert st == B.JOB_DONE, (jid, j)
        name = f"serving_2000/job{j['job_id']}"
        case = golden[name]
        assert (case["L"], case["R"], case["n_T"], case["sweeps"]) == (j["L"], j["R"], j["n_T"], j["sweeps"])
        spins, perm = srv.final_state(jid)
        E, q = srv.result(jid)
        _check(name, case, spins, perm, E, q, j["sweeps"])
        srv.release(jid)
        checked.append(name)

    recs, wall = serve.run_trace(trace, srv, on_done=on_done)
    print(f"[volume] serving trace: {len(checked)} jobs checked, wall {wall:.2f} s, stats {srv.stats()}", flush=True)
    assert len(checked) == len(trace)
    srv.close()
