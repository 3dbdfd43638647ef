"""GPU path vs the CPU oracle, bit for bit, through the C ABI.

The method is an exact Markov chain over a counter-based random stream, so
the spins, the temperature permutations, the energies and the overlaps must
match the oracle exactly (integer results: bit-exact is the bar).  Large
launches are checked on sampled realizations the oracle can run by
themselves, plus properties that hold at any size.
"""
import numpy as np
import pytest

from paper_1311_5582_amd import binding as B
from paper_1311_5582_amd import inputs
from tests import bruteforce as bf

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    B.lib()


def _report(tag, **kw):
    print(f"[parity] {tag} " + " ".join(f"{k}={v}" for k, v in kw.items()), flush=True)


def run_pair(oracle_lib, L, R, n_T, seed, sweeps, swap_every, layout="camsc", t_min=0.4, t_max=2.0,
             rids=None, block_threads=0, words_resident=0, couplings=None, splits=None, rng="words", split=True,
             h=0.0, site_order="natural", betas=None):
    """Run the GPU on all R realizations and the oracle on `rids`; compare."""
    _report("run", L=L, R=R, n_T=n_T, seed=seed, sweeps=sweeps, swap_every=swap_every, layout=layout,
            bt=block_threads, wr=words_resident, rng=rng, split=split, h=h)
    J = inputs.couplings(L, R, seed) if couplings is None else couplings
    betas = inputs.geometric_betas(n_T, t_min, t_max) if betas is None else betas
    rids = list(range(R)) if rids is None else list(rids)
    sim = B.Sim(L, J, betas, seed, layout=layout, block_threads=block_threads, words_resident=words_resident,
                rng=rng, split=split, h=h, site_order=site_order)
    orc = oracle_lib.OracleSim(L, J[rids], betas, seed, rid=np.array(rids), rng=rng, h=h)
    s0, p0, t0 = sim.state()
    assert t0 == 0
    assert np.array_equal(s0[rids], orc.spins), "initial spins differ"
    for n in (splits or [sweeps]):
        sim.sweep(n, swap_every)
        orc.sweep(n, swap_every)
    s, perm, t = sim.state()
    assert t == orc.t == sweeps
    assert np.array_equal(perm[rids], orc.temp_of_slot), "temperature permutation differs"
    assert np.array_equal(s[rids], orc.spins), "spins differ"
    E, q = sim.observables()
    Eo, qo = orc.observables()
    assert np.array_equal(E[rids], Eo) and np.array_equal(q[rids], qo)
    return sim, orc, (s, perm, E, q), J, betas


def check_observables_properties(L, J, betas, s, perm, E, q):
    """At any size: E is the Hamiltonian of the configuration at each
    temperature index, q the overlap of the two copies there."""
    R, _, n_T, N = s.shape
    for r in range(R):
        for c in range(2):
            sot = np.argsort(perm[r, c])
            for k in range(n_T):
                assert E[r, c, k] == bf.energy(L, J[r], s[r, c, sot[k]])
        sot0, sot1 = np.argsort(perm[r, 0]), np.argsort(perm[r, 1])
        qq = np.sum(s[r, 0, sot0].astype(np.int64) * s[r, 1, sot1].astype(np.int64), axis=1)
        assert np.array_equal(q[r], qq)


@pytest.mark.parametrize("layout", ["camsc", "amsc4", "amsc3", "amsc1"])
def test_plain_L8_full_run(oracle_lib, layout):
    """The single-job workload in full: L=8, 1 realization, 16 temperatures in
    [0.5, 2.0], 1000 sweeps, PT after every sweep."""
    cfg = inputs.CONFIGS["plain_L8"]
    sim, orc, (s, perm, E, q), J, betas = run_pair(oracle_lib, cfg["L"], cfg["R"], cfg["n_T"], cfg["seed"],
                                                   cfg["sweeps"], cfg["swap_every"], layout=layout,
                                                   t_min=cfg["t_min"], t_max=cfg["t_max"])
    check_observables_properties(cfg["L"], J, betas, s, perm, E, q)
    acc = sim.swap_acceptance()
    assert acc.sum() > 0


@pytest.mark.parametrize("L,n_T,layout", [(2, 4, "camsc"), (3, 5, "camsc"), (5, 22, "camsc"), (6, 34, "camsc"),
                                          (7, 40, "amsc4"), (4, 64, "camsc"), (4, 1, "camsc"), (5, 2, "amsc4"),
                                          (6, 13, "amsc4"), (9, 33, "camsc"), (3, 7, "amsc3"), (6, 10, "amsc3"),
                                          (5, 23, "amsc3"), (4, 64, "amsc3"), (7, 33, "amsc1"), (4, 5, "amsc1")])
def test_shapes_and_ragged_slots(oracle_lib, L, n_T, layout):
    """Even and odd L (two and three colour classes), ladders that fill a
    word exactly or leave a ragged tail, the smallest lattice and ladder."""
    run_pair(oracle_lib, L, 3, n_T, 1000 + L * 7 + n_T, 25, 1, layout=layout)


@pytest.mark.parametrize("swap_every", [0, 1, 3, 10])
def test_swap_schedules(oracle_lib, swap_every):
    run_pair(oracle_lib, 6, 2, 12, 77, 31, swap_every)


def test_split_calls_equal_one_call(oracle_lib):
    # swap points follow the global sweep index, so any split gives the same chain
    run_pair(oracle_lib, 6, 2, 20, 5, 37, 4, splits=[1, 9, 0, 13, 14])


@pytest.mark.parametrize("layout", ["camsc", "amsc4", "amsc3", "amsc1"])
@pytest.mark.parametrize("block_threads,words_resident", [(64, 0), (256, 0), (1024, 0), (128, 1), (64, 2)])
def test_launch_shape_invariance(oracle_lib, layout, block_threads, words_resident):
    """Any workgroup size and any number of LDS-resident words (staging the
    rest through HBM) gives the same chain."""
    run_pair(oracle_lib, 8, 2, 48, 31, 12, 3, layout=layout, block_threads=block_threads,
             words_resident=words_resident)


def test_L16_R64_sampled(oracle_lib):
    """The paper's lattice size with 64 realizations in one launch; the oracle
    reruns three sampled realizations; every realization is checked for
    energy/overlap consistency."""
    cfg = inputs.CONFIGS["L16_R64"]
    sim, orc, (s, perm, E, q), J, betas = run_pair(oracle_lib, cfg["L"], cfg["R"], cfg["n_T"], cfg["seed"], 6, 1,
                                                   rids=[0, 37, 63])
    check_observables_properties(cfg["L"], J, betas, s, perm, E, q)


def test_L24_sampled_staged_amsc4(oracle_lib):
    """L=24 with 48 temperatures: AMSC4 needs 6 words per site and AMSC3 5,
    staged through HBM; CAMSC keeps its 2 words resident."""
    L, n_T, seed = 24, 48, 4
    J = inputs.couplings(L, 4, seed)
    ref = None
    for layout in ("camsc", "amsc4", "amsc3"):
        sim, orc, st, _, _ = run_pair(oracle_lib, L, 4, n_T, seed, 3, 2, layout=layout, t_min=0.35, rids=[2],
                                      couplings=J)
        if ref is None:
            ref = st
        else:
            for a, b in zip(ref, st):
                assert np.array_equal(a, b)


def test_batched_uneven_jobs_equal_alone(oracle_lib):
    """One launch over jobs of different L and ladder length gives each job
    exactly the chain it has alone."""
    jobs = [(6, 3, 16, 11), (5, 2, 22, 12), (8, 2, 40, 13), (4, 4, 7, 14)]
    sims, refs = [], []
    for L, R, n_T, seed in jobs:
        J = inputs.couplings(L, R, seed)
        betas = inputs.geometric_betas(n_T, 0.4, 2.0)
        sims.append(B.Sim(L, J, betas, seed))
        alone = B.Sim(L, J, betas, seed)
        alone.sweep(9, 2)
        refs.append(alone.state())
    B.sweep_batch(sims, [9] * len(sims), [2] * len(sims))
    for sim, ref, (L, R, n_T, seed) in zip(sims, refs, jobs):
        got = sim.state()
        assert got[2] == ref[2] == 9
        assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1])
    # and the alone result is the oracle's
    L, R, n_T, seed = jobs[1]
    orc = oracle_lib.OracleSim(L, inputs.couplings(L, R, seed), inputs.geometric_betas(n_T, 0.4, 2.0), seed)
    orc.sweep(9, 2)
    assert np.array_equal(sims[1].state()[0], orc.spins)


def test_checkpoint_resume(oracle_lib):
    L, R, n_T, seed = 6, 2, 10, 99
    J = inputs.couplings(L, R, seed)
    betas = inputs.geometric_betas(n_T, 0.4, 2.0)
    a = B.Sim(L, J, betas, seed)
    a.sweep(17, 3)
    snap = a.state()
    a.sweep(20, 3)
    b = B.Sim(L, J, betas, seed, layout="amsc4")
    b.set_state(*snap)
    b.sweep(20, 3)
    sa, sb = a.state(), b.state()
    assert sa[2] == sb[2] == 37
    assert np.array_equal(sa[0], sb[0]) and np.array_equal(sa[1], sb[1])


def test_frozen_ferromagnet_gpu():
    L = 8
    J = inputs.ferro_couplings(L, 2)
    betas = inputs.geometric_betas(6, 0.3, 0.54)
    sim = B.Sim(L, J, betas, 3)
    s, perm, t = sim.state()
    sim.set_state(np.ones_like(s), perm, t)
    sim.sweep(50, 1)
    E, q = sim.observables()
    assert np.all(E == -3 * L ** 3) and np.all(q == L ** 3)


def test_set_state_rejects_bad_permutation():
    sim = B.Sim(4, inputs.couplings(4, 1, 1), inputs.geometric_betas(4, 0.5, 2.0), 1)
    s, perm, t = sim.state()
    perm[0, 1, 2] = perm[0, 1, 3]
    with pytest.raises(B.EAError):
        sim.set_state(s, perm, t)


@pytest.mark.parametrize("mode", ["always", "slots"])
@pytest.mark.parametrize("L,R,n_T,swap_every", [(8, 1, 16, 1), (16, 2, 32, 1), (6, 3, 24, 3), (4, 2, 8, 2),
                                                (10, 1, 32, 0)])
def test_split_ladders_equal_unsplit(oracle_lib, L, R, n_T, swap_every, mode):
    """A job with few ladders spreads each ladder over 2 or 4 workgroups: by
    lattice halves (two parts, mode "always") or by slot groups that meet only
    at swap points; the chain is the same as one workgroup per ladder, and the
    oracle's."""
    seed = 500 + L + n_T
    J = inputs.couplings(L, R, seed)
    betas = inputs.geometric_betas(n_T, 0.4, 2.0)
    a = B.Sim(L, J, betas, seed, split=mode)
    b = B.Sim(L, J, betas, seed, split=False)
    print(f"[parity] split info {a.info()} unsplit {b.info()}", flush=True)
    assert a.info()["split_parts"] > 1 and b.info()["split_parts"] == 1
    assert a.info()["split_by_halves"] == (mode == "always" and a.info()["split_parts"] == 2)
    for n in (5, 1, 14):
        a.sweep(n, swap_every)
        b.sweep(n, swap_every)
        sa, sb = a.state(), b.state()
        assert np.array_equal(sa[0], sb[0]) and np.array_equal(sa[1], sb[1]) and sa[2] == sb[2]
    assert np.array_equal(a.observables()[0], b.observables()[0])
    orc = oracle_lib.OracleSim(L, J, betas, seed)
    orc.sweep(20, swap_every)
    assert np.array_equal(a.state()[0], orc.spins)
    assert np.array_equal(a.swap_acceptance(), b.swap_acceptance())


@pytest.mark.parametrize("L,R,n_T,swap_every,bt,rids", [
    (8, 64, 32, 1, 64, [0, 37, 63]),   # 2 parts x 4 own groups, four class-0 sites per thread (two drawn ahead)
    (16, 1, 32, 1, 256, None),         # 4 parts, eight sites per thread: wider plane counters, generic reduction
    (12, 2, 24, 1, 512, None),         # 2 parts x 3 own groups, 864 sites per class: a ragged second site
    (10, 1, 16, 2, 128, None),         # 4 parts x 1 own group, PT every second sweep
])
def test_split_launch_shapes(oracle_lib, L, R, n_T, swap_every, bt, rids):
    """Split ladders by slot groups at workgroup sizes that give a thread more
    or fewer than the two class-0 sites whose next-sweep draws the swap step
    makes ahead of time, and every number of own slot groups: the oracle's
    chain, with calls that end right after a swap point and mid-interval."""
    sim, *_ = run_pair(oracle_lib, L, R, n_T, 7000 + 7 * L + n_T, 21, swap_every, split="slots", block_threads=bt,
                       rids=rids, splits=[1, 9, 11])
    info = sim.info()
    print(f"[parity] split launch {info}", flush=True)
    assert info["split_parts"] > 1 and info["block_threads"] == bt and not info["split_by_halves"]


@pytest.mark.parametrize("L,R,n_T,swap_every,bt,rids,rng", [
    (4, 1, 8, 1, 0, None, "words"),             # two planes per half: every site is on a boundary plane
    (16, 2, 24, 1, 1024, None, "words"),        # one site of a class per thread
    (20, 1, 20, 3, 256, None, "words"),         # five slot groups (no even split by groups), eight sites per thread
    (6, 3, 24, 0, 64, None, "words"),           # three planes per half, no PT, two sites per thread
    (8, 1, 1, 1, 0, None, "words"),             # one temperature: no swap pass
    (16, 40, 32, 1, 0, [0, 17, 39], "words"),   # the benchmark's shape with fewer realizations
    (4, 1, 8, 1, 0, None, "planes"),            # plane draws: every site on a boundary plane
    (16, 2, 24, 1, 1024, None, "planes"),       # plane draws, one site of a class per thread
    (20, 1, 20, 3, 256, None, "planes"),        # plane draws, a ragged last half, eight sites per thread
    (6, 3, 24, 0, 64, None, "planes"),          # plane draws, no PT
    (16, 40, 32, 1, 0, [0, 17, 39], "planes"),  # plane draws at the benchmark's shape
])
def test_split_by_halves_equals_oracle(oracle_lib, L, R, n_T, swap_every, bt, rids, rng):
    """Ladders split by lattice halves along z: each part owns half the planes
    with every slot and trades its first and last plane with the partner after
    every colour class, and the two halves' energy sums are added at swap
    points.  The oracle's chain (either draw stream), with calls ending right
    after a swap point and mid-interval."""
    sim, *_ = run_pair(oracle_lib, L, R, n_T, 9100 + 7 * L + n_T, 23, swap_every, split="always", block_threads=bt,
                       rids=rids, splits=[1, 9, 13], rng=rng)
    info = sim.info()
    print(f"[parity] split by halves {info}", flush=True)
    assert info["split_parts"] == 2 and info["split_by_halves"]
    if bt:
        assert info["block_threads"] == bt


@pytest.mark.parametrize("split,rng", [("always", "words"), ("always", "planes"), (False, "words"), (False, "planes")])
def test_swap_tables_in_hbm_equal_oracle(oracle_lib, split, rng):
    """Four pairs of nearly equal temperatures (d beta = 1e-7) give swap tables
    of 3N + 1 entries each, 4 x 12289 x 4 bytes at L=16: more than LDS holds,
    so the swap step reads the tables from HBM and the draws made ahead of it
    stay draws (with the tables in LDS, as in every other test, they become
    cuts).  Those pairs accept nearly always, the others at their usual rates.
    Split by lattice halves (either draw stream) and one workgroup per ladder."""
    L, R, n_T = 16, 2, 24
    betas = inputs.geometric_betas(n_T, 0.4, 2.0).copy()
    for k in (3, 9, 15, 21):
        betas[k + 1] = betas[k] - 1e-7
    sim, *_ = run_pair(oracle_lib, L, R, n_T, 9400 + (split is False) + 2 * (rng == "planes"), 23, 1, split=split,
                       rng=rng, betas=betas, splits=[1, 9, 13])
    info = sim.info()
    print(f"[parity] swap tables in HBM {info}", flush=True)
    assert info["split_by_halves"] == (split == "always")
    acc = sim.swap_acceptance().astype(np.int64)   # [R][copy][pair], 23 swap points each
    near = [3, 9, 15, 21]
    other = [k for k in range(n_T - 1) if k not in near]
    assert acc[:, :, near].min() >= 18, acc[:, :, near]   # nearly always accepted
    assert acc[:, :, other].sum() < 23 * R * 2 * len(other)   # and the table test rejects elsewhere


@pytest.mark.parametrize("L,R,n_T,swap_every,split,bt,wr", [
    (8, 1, 16, 1, True, 0, 0),        # the single small job
    (6, 3, 13, 1, False, 0, 0),       # ragged: one partial half
    (5, 2, 22, 1, True, 0, 0),        # odd L (three colour classes), two halves, ragged
    (4, 2, 40, 2, True, 0, 0),        # two words per site
    (8, 1, 64, 3, False, 64, 1),      # four halves, second word staged through HBM, 64 threads
    (16, 2, 32, 1, "always", 0, 0),   # split ladders, one half per part
    (10, 1, 32, 0, "always", 0, 0),   # split in 4 parts: quarter halves
    (6, 3, 24, 3, "always", 0, 0),    # split in 2: the second part spans both halves
    (2, 2, 4, 1, False, 0, 0),        # smallest lattice
])
def test_plane_draws_equal_oracle(oracle_lib, L, R, n_T, swap_every, split, bt, wr):
    """The bit-plane flip-draw stream: bit for bit the oracle's chain."""
    sim, *_ = run_pair(oracle_lib, L, R, n_T, 4000 + 13 * L + n_T, 21, swap_every, rng="planes", split=split,
                       block_threads=bt, words_resident=wr, splits=[1, 9, 11])
    info = sim.info()
    print(f"[parity] planes launch {info}", flush=True)
    if split == "always":
        assert info["split_parts"] > 1


@pytest.mark.parametrize("rng", ["words", "planes"])
def test_repeated_temperatures(oracle_lib, rng):
    """Equal neighbouring inverse temperatures: that pair's swap table is empty
    and every swap between them is accepted."""
    L, R, seed = 6, 2, 321
    J = inputs.couplings(L, R, seed)
    betas = np.array([0.5, 0.5, 0.7, 0.7, 0.7, 1.0, 1.4])
    sim = B.Sim(L, J, betas, seed, rng=rng)
    orc = oracle_lib.OracleSim(L, J, betas, seed, rng=rng)
    for n, se in ((7, 1), (5, 2)):
        sim.sweep(n, se)
        orc.sweep(n, se)
    s, perm, t = sim.state()
    assert np.array_equal(perm, orc.temp_of_slot) and np.array_equal(s, orc.spins)
    assert np.array_equal(sim.observables()[0], orc.observables()[0])


@pytest.mark.parametrize("L,R,n_T,layout,h,split", [
    (6, 3, 16, "camsc", 0.75, True),
    (5, 2, 22, "camsc", -1.25, True),      # odd L
    (4, 2, 40, "camsc", 0.25, True),       # two words per site
    (8, 1, 16, "camsc", 2.0, "always"),    # split ladders
    (6, 2, 13, "amsc4", -0.5, True),
    (5, 2, 23, "amsc3", 1.5, True),
    (6, 2, 33, "amsc1", -3.0, True),
    (4, 2, 12, "camsc", 8.0, True),        # every flip against the field is certain or impossible
])
def test_field_equals_oracle(oracle_lib, L, R, n_T, layout, h, split):
    """External field h (a multiple of 1/4): flips, swaps, energies, overlaps
    and magnetizations bit for bit the oracle's."""
    sim, orc, *_ = run_pair(oracle_lib, L, R, n_T, 6000 + 11 * L + n_T, 19, 1, layout=layout, h=h, split=split,
                            t_min=0.5, t_max=3.0, splits=[4, 15])
    assert np.array_equal(sim.magnetization(), orc.magnetization())
    print(f"[parity] field launch {sim.info()}", flush=True)


@pytest.mark.parametrize("L,R,n_T,parts,halves", [
    (16, 64, 32, 2, True),    # the benchmark job: 128 ladders, so 4 parts would exceed the CUs
    (8, 4, 32, 4, False),     # each of 4 parts keeps 2 groups x 512 sites
    (8, 1, 16, 1, False),     # too little work per part: the exchange would cost more than the split saves
    (24, 2, 48, 1, False),    # two words per site: split ladders need one
])
def test_split_choice(L, R, n_T, parts, halves):
    """The automatic choice of workgroups per ladder on a 256-CU device."""
    import torch
    if torch.cuda.get_device_properties(0).multi_processor_count != 256:
        pytest.skip("the choice depends on the number of compute units")
    sim = B.Sim(L, inputs.couplings(L, R, 3), inputs.geometric_betas(n_T, 0.5, 2.0), 3)
    assert sim.info()["split_parts"] == parts
    assert sim.info()["split_by_halves"] == halves
    sim.close()


@pytest.mark.parametrize("n_T,split", [(64, False), (32, "always")])
def test_plane_draws_deep_planes(oracle_lib, n_T, split):
    """Plane draws over enough flip attempts that halves needing planes 16..31
    occur (a slot's draw and threshold agree in their top 16 bits with
    probability 2^-16): L=2 with 16 realizations for 3 x 10^4 sweeps is up to
    5 x 10^8 flip attempts, a few thousand such halves and about ten past
    plane 24, all finished from the wave's list; every realization bit for bit
    the oracle's (one oracle thread per realization)."""
    import threading
    L, R, seed, sweeps = 2, 16, 8100 + n_T, 30_000
    J = inputs.couplings(L, R, seed)
    betas = inputs.geometric_betas(n_T, 0.3, 3.0)
    sim = B.Sim(L, J, betas, seed, rng="planes", split=split)
    print(f"[parity] deep planes {sim.info()}", flush=True)
    sim.sweep(sweeps, 1)
    s, perm, t = sim.state()
    E, q = sim.observables()
    orcs = [oracle_lib.OracleSim(L, J[[r]], betas, seed, rid=np.array([r]), rng="planes") for r in range(R)]
    ths = [threading.Thread(target=o.sweep, args=(sweeps, 1)) for o in orcs]
    for th in ths:
        th.start()
    for th in ths:
        th.join()
    for r, o in enumerate(orcs):
        assert o.t == t == sweeps
        assert np.array_equal(perm[r], o.temp_of_slot[0]), f"realization {r}: permutation differs"
        assert np.array_equal(s[r], o.spins[0]), f"realization {r}: spins differ"
        Eo, qo = o.observables()
        assert np.array_equal(E[r], Eo[0]) and np.array_equal(q[r], qo[0])


@pytest.mark.parametrize("L,R,n_T,swap_every,rng,split,bt,wr", [
    (8, 2, 16, 1, "words", False, 0, 0),       # unsplit, fused energy in the summing class
    (6, 3, 24, 3, "words", False, 0, 0),       # L/2 odd: rows of three class sites
    (16, 2, 32, 1, "words", "always", 0, 0),   # split ladders, paired sites, next-sweep draws
    (4, 2, 40, 2, "words", False, 0, 0),       # two words per site, energies from the separate count
    (8, 1, 64, 3, "words", False, 64, 1),      # second word staged through HBM, 64 threads
    (10, 1, 32, 0, "planes", "always", 0, 0),  # plane draws, split in 4
    (6, 2, 22, 1, "planes", False, 0, 0),      # plane draws, ragged halves
])
def test_class_order_equals_oracle(oracle_lib, L, R, n_T, swap_every, rng, split, bt, wr):
    """Spin words and couplings held by colour class in LDS (the separated
    allocation): the oracle's chain bit for bit in every launch shape."""
    sim, *_ = run_pair(oracle_lib, L, R, n_T, 9100 + 7 * L + n_T, 21, swap_every, rng=rng, split=split,
                       block_threads=bt, words_resident=wr, splits=[1, 9, 11], site_order="by_class")
    print(f"[parity] class order {sim.info()}", flush=True)


def test_class_order_field(oracle_lib):
    """The class order with a field (certain flips both ways, spins-up counts)."""
    sim, orc, *_ = run_pair(oracle_lib, 6, 3, 16, 9300, 19, 1, h=0.75, splits=[4, 15], site_order="by_class")
    assert np.array_equal(sim.magnetization(), orc.magnetization())
