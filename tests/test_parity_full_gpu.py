"""Parity at the benchmarked sizes, in the launch configurations bench.py
times: the GPU runs every realization of the workload, the oracle re-runs
sampled realizations by themselves (one thread each), and the comparison is
bit for bit.  Every other realization is checked against the Hamiltonian
(energies) and the two copies (overlaps), which holds at any size.
"""
import threading

import numpy as np
import pytest

from paper_1311_5582_amd import binding as B
from paper_1311_5582_amd import inputs
from tests.test_parity_gpu import check_observables_properties

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    B.lib()


def _oracles(oracle_lib, L, J, betas, seed, rids, sweeps, swap_every):
    """Run the oracle on each sampled realization in its own thread (the C
    library releases the GIL)."""
    sims = [oracle_lib.OracleSim(L, J[[r]], betas, seed, rid=np.array([r])) for r in rids]
    ths = [threading.Thread(target=o.sweep, args=(sweeps, swap_every)) for o in sims]
    for th in ths:
        th.start()
    for th in ths:
        th.join()
    return sims


def _compare(rids, orcs, s, perm, E, q, sweeps):
    for r, o in zip(rids, orcs):
        assert o.t == sweeps
        assert np.array_equal(perm[r], o.temp_of_slot[0]), f"realization {r}: permutation differs"
        assert np.array_equal(s[r], o.spins[0]), f"realization {r}: spins differ"
        Eo, qo = o.observables()
        assert np.array_equal(E[r], Eo[0]) and np.array_equal(q[r], qo[0]), f"realization {r}: observables differ"


def test_L16_R64_bench_launch(oracle_lib):
    """64 realizations at L=16 with 32 temperatures, PT every sweep, 1000
    sweeps in one launch as the benchmark issues it (split ladders)."""
    cfg = inputs.CONFIGS["L16_R64"]
    L, R, n_T, seed = cfg["L"], cfg["R"], cfg["n_T"], cfg["seed"]
    J = inputs.couplings(L, R, seed)
    betas = inputs.geometric_betas(n_T, cfg["t_min"], cfg["t_max"])
    sim = B.Sim(L, J, betas, seed)
    print(f"[parity-full] L16_R64 launch {sim.info()}", flush=True)
    sim.sweep(1000, cfg["swap_every"])
    s, perm, t = sim.state()
    E, q = sim.observables()
    assert t == 1000
    rids = [0, 41, 63]
    _compare(rids, _oracles(oracle_lib, L, J, betas, seed, rids, 1000, cfg["swap_every"]), s, perm, E, q, 1000)
    check_observables_properties(L, J, betas, s, perm, E, q)


def test_batched_plan_bench_launch(oracle_lib):
    """The five uneven jobs (L = 8..20, 16..40 temperatures, 128 realizations
    each) in one autotuned, graph-captured plan as the benchmark runs it: two
    replays of 250 sweeps; the oracle re-runs one realization of every job."""
    jobs = inputs.BATCHED_JOBS
    Js = [inputs.couplings(j["L"], j["R"], j["seed"]) for j in jobs]
    bs = [inputs.geometric_betas(j["n_T"], j["t_min"], j["t_max"]) for j in jobs]
    sims = [B.Sim(j["L"], J, b, j["seed"]) for j, J, b in zip(jobs, Js, bs)]
    plan = B.Plan(sims, 250, [j["swap_every"] for j in jobs], autotune=True)
    print(f"[parity-full] batched plan {plan.info()}", flush=True)
    plan.run(2)
    results = []
    for sim in sims:
        s, perm, t = sim.state()
        assert t == 500
        results.append((s, perm) + tuple(sim.observables()))
    plan.close()
    picks = [(k, (37 * k + 5) % j["R"]) for k, j in enumerate(jobs)]
    orcs, ths = [], []
    for k, r in picks:
        j = jobs[k]
        o = oracle_lib.OracleSim(j["L"], Js[k][[r]], bs[k], j["seed"], rid=np.array([r]))
        orcs.append(o)
        ths.append(threading.Thread(target=o.sweep, args=(500, j["swap_every"])))
    for th in ths:
        th.start()
    for th in ths:
        th.join()
    for (k, r), o in zip(picks, orcs):
        s, perm, E, q = results[k]
        _compare([r], [o], s, perm, E, q, 500)
    for k in (0, 2):   # the cheaper jobs: every realization against the Hamiltonian
        s, perm, E, q = results[k]
        check_observables_properties(jobs[k]["L"], Js[k], bs[k], s, perm, E, q)


def test_L24_R256_bench_launch(oracle_lib):
    """256 realizations at L=24 with 48 temperatures, PT every 10 sweeps, 200
    sweeps (20 swap points) in the benchmark's launch."""
    cfg = inputs.CONFIGS["L24_R256"]
    L, R, n_T, seed = cfg["L"], cfg["R"], cfg["n_T"], cfg["seed"]
    J = inputs.couplings(L, R, seed)
    betas = inputs.geometric_betas(n_T, cfg["t_min"], cfg["t_max"])
    sim = B.Sim(L, J, betas, seed)
    print(f"[parity-full] L24_R256 launch {sim.info()}", flush=True)
    sim.sweep(200, cfg["swap_every"])
    s, perm, t = sim.state()
    E, q = sim.observables()
    rids = [0, 255]
    _compare(rids, _oracles(oracle_lib, L, J, betas, seed, rids, 200, cfg["swap_every"]), s, perm, E, q, 200)
    # Hamiltonian / overlap consistency on a spread of realizations
    sub = np.arange(0, R, 17)
    check_observables_properties(L, J[sub], betas, s[sub], perm[sub], E[sub], q[sub])
