"""Batching runtime and serving loop on the GPU: graph-captured plans against
eager runs, and the server's results alone vs in a mix, bit for bit."""
import numpy as np
import pytest

from paper_1311_5582_amd import binding as B
from paper_1311_5582_amd import inputs
from paper_1311_5582_amd import serve

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    B.lib()


JOBS = [  # L, R, n_T, seed, swap_every
    (6, 3, 16, 11, 1), (5, 2, 22, 12, 2), (8, 2, 40, 13, 0), (4, 4, 7, 14, 3), (10, 1, 33, 15, 1),
]


def _make(L, R, n_T, seed, layout="camsc", words_resident=0, split=True, rng="words"):
    return B.Sim(L, inputs.couplings(L, R, seed), inputs.geometric_betas(n_T, 0.4, 2.0), seed, layout=layout,
                 words_resident=words_resident, split=split, rng=rng)


@pytest.mark.parametrize("use_graph,autotune", [(True, True), (False, False), (True, False)])
def test_plan_replays_equal_eager(use_graph, autotune):
    sims = [_make(L, R, n_T, seed) for L, R, n_T, seed, _ in JOBS]
    refs = [_make(L, R, n_T, seed) for L, R, n_T, seed, _ in JOBS]
    se = [j[4] for j in JOBS]
    plan = B.Plan(sims, 3, se, autotune=autotune, use_graph=use_graph)
    info = plan.info()
    print(f"[runtime] plan info {info}", flush=True)
    assert info["uses_graph"] == use_graph
    assert info["units"] == sum(2 * j[1] for j in JOBS)
    for rep in range(4):
        plan.run(1)
        for ref, (_, _, _, _, s) in zip(refs, JOBS):
            ref.sweep(3, s)
        for sim, ref in zip(sims, refs):
            a, b = sim.state(), ref.state()
            assert a[2] == b[2] == 3 * (rep + 1)
            assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]), f"replay {rep}"
            # eager work on the planned jobs between replays
            assert np.array_equal(sim.observables()[0], ref.observables()[0])
    plan.run(2)
    for ref, (_, _, _, _, s) in zip(refs, JOBS):
        ref.sweep(6, s)
    for sim, ref in zip(sims, refs):
        assert np.array_equal(sim.state()[0], ref.state()[0])
    plan.close()


def test_plan_amsc4_staged_equal_eager():
    # the first job keeps 2 of its 6 AMSC4 words in LDS and stages the rest
    jobs = [(8, 2, 48, 21, 2), (6, 3, 20, 22, 0)]
    sims = [_make(L, R, n_T, s, layout="amsc4", words_resident=w) for L, R, n_T, s, w in jobs]
    refs = [_make(L, R, n_T, s, layout="amsc4") for L, R, n_T, s, _ in jobs]
    plan = B.Plan(sims, 4, [2, 1], autotune=True)
    plan.run(3)
    refs[0].sweep(12, 2)
    refs[1].sweep(12, 1)
    for a, b in zip(sims, refs):
        assert np.array_equal(a.state()[0], b.state()[0]) and np.array_equal(a.state()[1], b.state()[1])


def test_footprint_matches_allocation():
    for L, R, n_T, seed, _ in JOBS:
        for layout in ("camsc", "amsc4"):
            betas = inputs.geometric_betas(n_T, 0.4, 2.0)
            sim = B.Sim(L, inputs.couplings(L, R, seed), betas, seed, layout=layout)
            assert sim.footprint() == B.job_footprint(L, betas, R, layout)
            sim.close()


def _trace(n, seed=9):
    rng = np.random.default_rng(seed)
    out, t = [], 0.0
    for j in range(n):
        t += rng.exponential(0.002)
        out.append(dict(arrival_s=t, L=int(rng.integers(4, 9)), R=int(rng.integers(1, 5)),
                        n_T=int(rng.integers(4, 40)), t_min=0.4, t_max=2.0,
                        sweeps=int(rng.integers(5, 60)), swap_every=int(rng.integers(0, 4)), seed=1000 + j))
    return out


@pytest.mark.parametrize("autotune,split,rng", [(False, True, "words"), (True, True, "words"), (False, "slots", "words"),
                                                (False, True, "planes")])
def test_split_plan_and_batch_equal_alone(oracle_lib, autotune, split, rng):
    """Jobs that together hold fewer ladders than the device has compute
    units run with split ladders (by lattice halves, or by slot groups when
    asked) in a graph-captured plan and in a batch; every replay equals the
    same jobs run one at a time without splitting, and one realization of each
    job equals the oracle."""
    jobs = [(16, 8, 32, 61, 1), (12, 6, 16, 62, 3), (16, 4, 24, 63, 0)]   # L, R, n_T, seed, swap_every
    if split == "slots":   # slot groups need a count every part divides
        jobs = [(16, 8, 32, 61, 1), (12, 6, 16, 62, 3), (16, 4, 32, 63, 0)]
    sims = [_make(L, R, n_T, seed, split=split, rng=rng) for L, R, n_T, seed, _ in jobs]
    bats = [_make(L, R, n_T, seed, split=split, rng=rng) for L, R, n_T, seed, _ in jobs]
    refs = [B.Sim(L, inputs.couplings(L, R, seed), inputs.geometric_betas(n_T, 0.4, 2.0), seed, split=False, rng=rng)
            for L, R, n_T, seed, _ in jobs]
    se = [j[4] for j in jobs]
    plan = B.Plan(sims, 6, se, autotune=autotune)
    info = plan.info()
    print(f"[runtime] split plan info {info}", flush=True)
    if not autotune:
        assert info["split_parts"] > 1
    for rep in range(3):
        plan.run(1)
        B.sweep_batch(bats, [6, 6, 6], se)
        for ref, s in zip(refs, se):
            ref.sweep(6, s)
        for k, (a, b, c) in enumerate(zip(sims, bats, refs)):
            sa, pa, ta = a.state()
            sb, pb, tb = b.state()
            sc, pc, tc = c.state()
            assert ta == tb == tc == 6 * (rep + 1)
            assert np.array_equal(pa, pc) and np.array_equal(sa, sc), f"plan replay {rep} job {k}"
            assert np.array_equal(pb, pc) and np.array_equal(sb, sc), f"batch {rep} job {k}"
    plan.close()
    for (L, R, n_T, seed, swe), sim in zip(jobs, sims):
        r = R - 1
        o = oracle_lib.OracleSim(L, inputs.couplings(L, R, seed)[[r]], inputs.geometric_betas(n_T, 0.4, 2.0), seed,
                                 rid=np.array([r]), rng=rng)
        o.sweep(18, swe)
        s, perm, t = sim.state()
        assert np.array_equal(s[r], o.spins[0]) and np.array_equal(perm[r], o.temp_of_slot[0])
        E, q = sim.observables()
        Eo, qo = o.observables()
        assert np.array_equal(E[r], Eo[0]) and np.array_equal(q[r], qo[0])
    for x in sims + bats + refs:
        x.close()


@pytest.mark.parametrize("policy", ["shortest", "fifo", "ratio"])
def test_server_results_alone_equal_mix(oracle_lib, policy):
    """Jobs admitted under a budget that holds only a few at a time, with a
    small quantum so they interleave: each final state equals the job run
    alone, and the energies/overlaps equal ea_observables of that run; one
    realization of every job equals the oracle's."""
    trace = _trace(8)
    fps = [B.job_footprint(j["L"], inputs.geometric_betas(j["n_T"], 0.4, 2.0), j["R"]) for j in trace]
    budget = sum(sorted(fps)[-3:])
    srv = B.Server(hbm_budget_bytes=budget, quantum_sweeps=7, keep_state=True, policy=policy)

    recs, wall = serve.run_trace(trace, srv, on_done=lambda jid, j, st: None)
    assert len(recs) == len(trace)
    for jid, rec in recs.items():
        j = rec["job"]
        assert rec["status"] == B.JOB_DONE, rec
        spins, perm = srv.final_state(jid)
        E, q = srv.result(jid)
        alone = _make(j["L"], j["R"], j["n_T"], j["seed"])
        alone.sweep(j["sweeps"], j["swap_every"])
        s2, p2, t2 = alone.state()
        assert t2 == j["sweeps"]
        assert np.array_equal(spins, s2) and np.array_equal(perm, p2), f"job {jid} differs from alone"
        E2, q2 = alone.observables()
        assert np.array_equal(E, E2) and np.array_equal(q, q2)
        r = j["seed"] % j["R"]
        betas = inputs.geometric_betas(j["n_T"], 0.4, 2.0)
        orc = oracle_lib.OracleSim(j["L"], inputs.couplings(j["L"], j["R"], j["seed"])[[r]], betas, j["seed"],
                                   rid=np.array([r]))
        orc.sweep(j["sweeps"], j["swap_every"])
        assert np.array_equal(spins[r], orc.spins[0]) and np.array_equal(perm[r], orc.temp_of_slot[0])
        Eo, qo = orc.observables()
        assert np.array_equal(E[r], Eo[0]) and np.array_equal(q[r], qo[0])
    st = srv.stats()
    print(f"[runtime] server stats {st} wall {wall:.3f}s", flush=True)
    assert st["hbm_used"] == 0
    assert st["steps"] > len(trace) // 2
    srv.close()


@pytest.mark.parametrize("pack", [True, False])
def test_server_packed_steps_equal_alone(oracle_lib, pack):
    """Jobs that together hold more ladders than the device has compute units
    (400 against 256 on MI355X), all arriving at once with a small quantum:
    with packing the least urgent jobs run shorter steps that fill the last
    round, so the per-job sweep counts of a step change as the jobs' response
    ratios move; every job's final state still equals the job run alone, and
    one realization of each equals the oracle's."""
    jobs = [dict(arrival_s=0.0, L=6, R=96, n_T=16, t_min=0.4, t_max=2.0, sweeps=61, swap_every=1, seed=2101),
            dict(arrival_s=0.0, L=8, R=64, n_T=20, t_min=0.4, t_max=2.0, sweeps=47, swap_every=2, seed=2102),
            dict(arrival_s=0.0, L=5, R=40, n_T=24, t_min=0.4, t_max=2.0, sweeps=33, swap_every=1, seed=2103)]
    srv = B.Server(quantum_sweeps=9, keep_state=True, pack_rounds=pack)
    recs, wall = serve.run_trace(jobs, srv, on_done=lambda jid, j, st: None)
    assert len(recs) == len(jobs)
    for jid, rec in recs.items():
        j = rec["job"]
        assert rec["status"] == B.JOB_DONE, rec
        spins, perm = srv.final_state(jid)
        alone = _make(j["L"], j["R"], j["n_T"], j["seed"])
        alone.sweep(j["sweeps"], j["swap_every"])
        s2, p2, _ = alone.state()
        assert np.array_equal(spins, s2) and np.array_equal(perm, p2), f"job {jid} differs from alone (pack={pack})"
        alone.close()
        r = j["seed"] % j["R"]
        orc = oracle_lib.OracleSim(j["L"], inputs.couplings(j["L"], j["R"], j["seed"])[[r]],
                                   inputs.geometric_betas(j["n_T"], 0.4, 2.0), j["seed"], rid=np.array([r]))
        orc.sweep(j["sweeps"], j["swap_every"])
        assert np.array_equal(spins[r], orc.spins[0]) and np.array_equal(perm[r], orc.temp_of_slot[0])
    st = srv.stats()
    print(f"[runtime] packed server stats pack={pack} {st} wall {wall:.3f}s", flush=True)
    srv.close()


def test_server_admission_respects_budget_and_cancel():
    trace = _trace(6, seed=3)
    betas = [inputs.geometric_betas(j["n_T"], 0.4, 2.0) for j in trace]
    fps = [B.job_footprint(j["L"], b, j["R"]) for j, b in zip(trace, betas)]
    budget = max(fps) + min(fps)
    srv = B.Server(hbm_budget_bytes=budget, quantum_sweeps=5)
    ids = [srv.submit(j["L"], inputs.couplings(j["L"], j["R"], j["seed"]), b, j["seed"], j["sweeps"], j["swap_every"])
           for j, b in zip(trace, betas)]
    srv.cancel(ids[-1])                               # cancel while queued
    assert srv.status(ids[-1])[0] == B.JOB_CANCELLED
    running_cancelled = False
    for _ in range(1000):
        running, queued, _ = srv.step()
        st = srv.stats()
        assert st["hbm_used"] <= budget
        if not running_cancelled and srv.status(ids[0])[0] == B.JOB_RUNNING and srv.status(ids[0])[1] < trace[0]["sweeps"]:
            srv.cancel(ids[0])                        # cancel while running
            running_cancelled = True
        if running == 0 and queued == 0:
            break
    assert srv.stats()["hbm_used"] == 0
    for jid, j in zip(ids[1:-1], trace[1:-1]):
        assert srv.status(jid)[0] == B.JOB_DONE
        E, q = srv.result(jid)
        alone = _make(j["L"], j["R"], j["n_T"], j["seed"])
        alone.sweep(j["sweeps"], j["swap_every"])
        E2, q2 = alone.observables()
        assert np.array_equal(E, E2) and np.array_equal(q, q2)
    with pytest.raises(B.EAError):
        srv.result(ids[-1])
    srv.close()


def test_server_rejects_job_larger_than_budget():
    srv = B.Server(hbm_budget_bytes=4096, quantum_sweeps=5)
    with pytest.raises(B.EAError):
        srv.submit(8, inputs.couplings(8, 2, 1), inputs.geometric_betas(8, 0.5, 2.0), 1, 10, 1)
    srv.close()


@pytest.mark.parametrize("rng,n_jobs", [("words", 12), ("planes", 6)])
def test_server_serving_trace_shapes(oracle_lib, rng, n_jobs):
    """The first jobs of the benchmark's serving trace at their real shapes
    (L 6..20 with odd L, 32..512 realizations, 16..48 temperatures so some
    ladders span two words), sweeps cut by 50x, through the server with a
    quantum that divides none of them and the default HBM budget.  One
    realization of every job, chosen by its seed, is re-run by the oracle
    (one thread per job) and compared bit for bit."""
    import threading
    trace = inputs.serving_trace(n_jobs=n_jobs, rate_per_s=200.0)
    for j in trace:
        j["sweeps"] = max(1, j["sweeps"] // 50)
    print(f"[runtime] serving shapes rng={rng} " +
          " ".join(f"L{j['L']}R{j['R']}T{j['n_T']}x{j['sweeps']}" for j in trace), flush=True)
    srv = B.Server(quantum_sweeps=37, keep_state=True, rng=rng)
    recs, wall = serve.run_trace(trace, srv)
    assert len(recs) == len(trace)
    picks = []
    for jid, rec in recs.items():
        j = rec["job"]
        assert rec["status"] == B.JOB_DONE, rec
        r = j["seed"] % j["R"]
        betas = inputs.geometric_betas(j["n_T"], j["t_min"], j["t_max"])
        J = inputs.couplings(j["L"], j["R"], j["seed"])
        spins, perm = srv.final_state(jid)
        E, q = srv.result(jid)
        orc = oracle_lib.OracleSim(j["L"], J[[r]], betas, j["seed"], rid=np.array([r]), rng=rng)
        picks.append((jid, j, r, spins, perm, E, q, orc))
    ths = [threading.Thread(target=p[-1].sweep, args=(p[1]["sweeps"], p[1]["swap_every"])) for p in picks]
    for th in ths:
        th.start()
    for th in ths:
        th.join()
    for jid, j, r, spins, perm, E, q, orc in picks:
        assert orc.t == j["sweeps"]
        assert np.array_equal(perm[r], orc.temp_of_slot[0]), f"job {jid} realization {r}: permutation differs"
        assert np.array_equal(spins[r], orc.spins[0]), f"job {jid} realization {r}: spins differ"
        Eo, qo = orc.observables()
        assert np.array_equal(E[r], Eo[0]) and np.array_equal(q[r], qo[0]), f"job {jid}: observables differ"
    st = srv.stats()
    print(f"[runtime] serving shapes stats {st} wall {wall:.3f}s", flush=True)
    assert st["hbm_used"] == 0
    srv.close()


def test_exit_hook_closes_live_handles():
    """The binding's exit hook closes every live server, plan and job in that
    order (it runs before interpreter teardown, while torch is intact), and a
    handle closed there is left inert for its own finaliser."""
    sims = [_make(8, 2, 16, s) for s in (1, 2)]
    plan = B.Plan(sims, 5, [1, 1], autotune=False)
    plan.run(1)
    srv = B.Server(quantum_sweeps=3)
    srv.submit(6, inputs.couplings(6, 1, 3), inputs.geometric_betas(8, 0.5, 2.0), 3, 7, 1)
    srv.step()
    assert plan in B._LIVE["plan"] and srv in B._LIVE["server"] and all(x in B._LIVE["sim"] for x in sims)
    B._close_live_handles()
    assert not srv._h.value and not plan._h.value and not any(x._h.value for x in sims)
    for x in (srv, plan, *sims):
        x.close()   # a second close is a no-op
