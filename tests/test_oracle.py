"""Pins for the CPU oracle, against things other than the oracle itself.

Each test fixes a property that the paper or the mathematics determines:
an independent generator implementation (rocRAND), closed forms of the
threshold tables, the Hamiltonian written out with numpy, the exact Boltzmann
distribution by enumeration at L = 2, the zero- and infinite-temperature
limits, gauge invariance, and the ferromagnetic ground state -3N.
"""
import math
import os
import shutil
import subprocess

import numpy as np
import pytest

from paper_1311_5582_amd import inputs
from tests import bruteforce as bf

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


# --------------------------------------------------------------------------
# Philox4x32-10 (Sec. 4.3.2 evaluates the counter-based Philox family)
# --------------------------------------------------------------------------
@pytest.fixture(scope="module")
def rocrand_probe(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available to build the rocRAND probe")
    out = tmp_path_factory.mktemp("rr") / "rocrand_philox_blocks"
    src = os.path.join(ROOT, "tests", "helpers", "rocrand_philox_blocks.cpp")
    subprocess.run([hipcc, "--offload-arch=gfx950", "-O1", "-o", str(out), src], check=True,
                   capture_output=True)
    return str(out)


def test_philox_matches_rocrand(oracle_lib, rocrand_probe):
    rng = np.random.default_rng(123)
    rows = []
    for n in range(300):
        c = rng.integers(0, 2 ** 32, size=4, dtype=np.uint64)
        c[1] %= 2 ** 30            # reachable through rocRAND's public offset
        k = rng.integers(0, 2 ** 32, size=2, dtype=np.uint64)
        if n < 4:                  # small and extreme words too
            c = np.array([n, 0, 0, 0] if n < 2 else [2 ** 32 - 1, 2 ** 30 - 1, 2 ** 32 - 1, 2 ** 32 - 1],
                         dtype=np.uint64)
            k = np.array([0, 0] if n % 2 == 0 else [2 ** 32 - 1, 2 ** 32 - 1], dtype=np.uint64)
        rows.append((c, k))
    text = "\n".join(" ".join(str(int(v)) for v in list(c) + list(k)) for c, k in rows) + "\n"
    res = subprocess.run([rocrand_probe], input=text, capture_output=True, text=True, check=True)
    got = [list(map(int, line.split())) for line in res.stdout.strip().splitlines()]
    assert len(got) == len(rows)
    for (c, k), ref in zip(rows, got):
        assert list(oracle_lib.philox4x32_10(c, k)) == ref


def test_plane_draws_are_rocrand_blocks_transposed(oracle_lib, rocrand_probe):
    """The bit-plane stream: plane p of half h is a 16-bit field of a Philox
    block; transposing rocRAND's blocks with numpy must give each slot's
    uniform (bit 31 - p of the uniform = bit slot & 15 of plane p)."""
    rng = np.random.default_rng(7)
    cases = []
    for n in range(12):
        seed = int(rng.integers(0, 2 ** 63)) if n else 0
        i, t, r, c = (int(rng.integers(0, 2 ** 32)), int(rng.integers(0, 2 ** 30)), int(rng.integers(0, 2 ** 20)),
                      n & 1)
        cases.append((seed, i, t, r, c))
    rows = []
    for seed, i, t, r, c in cases:
        for h in range(4):
            for g in range(4):
                rows.append((i, t, r, (4 << 28) | (c << 24) | (h << 8) | g, seed & 0xFFFFFFFF, seed >> 32))
    text = "\n".join(" ".join(str(v) for v in row) for row in rows) + "\n"
    res = subprocess.run([rocrand_probe], input=text, capture_output=True, text=True, check=True)
    blocks = np.array([list(map(int, line.split())) for line in res.stdout.strip().splitlines()], dtype=np.uint64)
    blocks = blocks.reshape(len(cases), 4, 4, 4)          # case, half, group, word
    for n, (seed, i, t, r, c) in enumerate(cases):
        for h in range(4):
            words = blocks[n, h].reshape(16)              # plane pair p>>1 = 4 g + word
            planes = np.empty(32, dtype=np.uint64)
            planes[0::2] = words & 0xFFFF
            planes[1::2] = words >> 16
            bits = (planes[:, None] >> np.arange(16, dtype=np.uint64)[None, :]) & 1   # [plane][slot in half]
            uniform = (bits << (31 - np.arange(32, dtype=np.uint64))[:, None]).sum(axis=0)
            for q in range(16):
                assert oracle_lib.flip_draw(seed, "planes", i, t, r, c, 16 * h + q) == int(uniform[q])


def test_plane_draws_uniform_and_independent(oracle_lib):
    """Uniforms of the bit-plane stream: top bits equidistributed, slots of one
    site (inside a half and across halves) uncorrelated and distinct."""
    U = np.array([[oracle_lib.flip_draw(99, "planes", i, 3, 1, 0, s) for s in range(64)] for i in range(400)],
                 dtype=np.float64)
    top = (U // 2 ** 28).astype(int).ravel()
    counts = np.bincount(top, minlength=16)
    chi2 = float(((counts - top.size / 16) ** 2 / (top.size / 16)).sum())
    assert chi2 < 45.0                                   # 15 d.o.f., p ~ 1e-4
    x = U / 2 ** 32 - 0.5
    for a, b in ((0, 1), (14, 15), (15, 16), (0, 16), (31, 32), (5, 63)):
        corr = float(np.mean(x[:, a] * x[:, b]) / np.sqrt(np.mean(x[:, a] ** 2) * np.mean(x[:, b] ** 2)))
        assert abs(corr) < 0.2, (a, b, corr)
    assert all(len(set(row)) == 64 for row in U.astype(np.int64).tolist())
    # the other stream is untouched by the option
    assert oracle_lib.flip_draw(99, "words", 5, 3, 1, 0, 6) == int(
        oracle_lib.philox4x32_10([5, 3, 1, (0 << 28) | (0 << 24) | 1], [99, 0])[2])


# --------------------------------------------------------------------------
# Integer probability tables (Sec. 4.3.1, 4.3.2)
# --------------------------------------------------------------------------
def test_flip_threshold_closed_forms(oracle_lib):
    # beta = ln2/4: exp(-beta*dE) = 2^(-dE/4), so thresholds are 2^29, 2^30, 2^31
    # for u = 0, 1, 2 (dE = 12, 8, 4), up to one unit from rounding of ln 2
    beta = math.log(2.0) / 4.0
    for u, expo in ((0, 29), (1, 30), (2, 31)):
        assert abs(oracle_lib.flip_threshold(beta, u) - 2 ** expo) <= 1
    # infinite temperature: probability 1, clamped to 2^32 - 1
    assert oracle_lib.flip_threshold(0.0, 0) == 2 ** 32 - 1
    # large beta: below one part in 2^32 -> 0
    assert oracle_lib.flip_threshold(5.6, 2) == 0
    assert oracle_lib.flip_threshold(5.5, 2) > 0        # 2^32 e^-22 = 1.19
    # monotone in u at fixed beta (higher u = smaller cost)
    for beta in (0.3, 1.0, 2.5):
        t = [oracle_lib.flip_threshold(beta, u) for u in range(3)]
        assert t[0] <= t[1] <= t[2]


def test_swap_threshold_closed_forms(oracle_lib):
    # |dbeta| = ln2/2: exp(-2 |dbeta| n) = 2^-n
    db = math.log(2.0) / 2.0
    for n in range(1, 32):
        assert abs(oracle_lib.swap_threshold(db, n) - 2 ** (32 - n)) <= 1
    for n in range(33, 40):
        assert oracle_lib.swap_threshold(db, n) == 0
    assert oracle_lib.swap_threshold(db, 0) == 2 ** 32 - 1


# --------------------------------------------------------------------------
# Lattice, colouring and energy (Sec. 2.2, 3.1, 4.3 Eq. e)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("L", [2, 3, 4, 5, 6, 7, 9])
def test_colouring_is_proper(oracle_lib, L):
    n_col = oracle_lib.n_phases(L)
    assert n_col == (2 if L % 2 == 0 else 3)
    col = np.array([[[oracle_lib.colour(L, x, y, z) for x in range(L)] for y in range(L)] for z in range(L)])
    assert set(np.unique(col)) == set(range(n_col))
    for axis in range(3):
        assert np.all(col != np.roll(col, -1, axis=axis))


@pytest.mark.parametrize("L", [2, 3, 4, 5, 8])
def test_energy_matches_hamiltonian(oracle_lib, L):
    rng = np.random.default_rng(L)
    J = inputs.couplings(L, 1, seed=77)[0]
    for _ in range(5):
        s = rng.choice(np.array([-1, 1], dtype=np.int8), size=L ** 3)
        U = oracle_lib.unsat_bonds(L, J, s)
        assert 2 * U - 3 * L ** 3 == bf.energy(L, J, s)
        u = bf.local_field_unsat(L, J, s)
        assert sum(oracle_lib.local_unsat(L, J, s, i) for i in range(L ** 3)) == 2 * U
        assert [oracle_lib.local_unsat(L, J, s, i) for i in range(L ** 3)] == list(u)


def test_ferro_ground_state_energy(oracle_lib):
    for L in (2, 3, 4, 8):
        J = inputs.ferro_couplings(L, 1)[0]
        up = np.ones(L ** 3, dtype=np.int8)
        assert 2 * oracle_lib.unsat_bonds(L, J, up) - 3 * L ** 3 == -3 * L ** 3
        assert 2 * oracle_lib.unsat_bonds(L, -J, up) - 3 * L ** 3 == 3 * L ** 3


# --------------------------------------------------------------------------
# Dynamics
# --------------------------------------------------------------------------
def _sim(oracle_lib, L, J, betas, seed=11, **kw):
    return oracle_lib.OracleSim(L, J, betas, seed, **kw)


@pytest.mark.parametrize("L", [4, 5])
def test_running_energy_equals_recomputed(oracle_lib, L):
    J = inputs.couplings(L, 2, seed=5)
    sim = _sim(oracle_lib, L, J, inputs.geometric_betas(6, 0.5, 3.0), track_energy=True)
    sim.sweep(60, 1)      # raises if the running sum of 6 - 2u ever disagrees
    sim.sweep(30, 7)


@pytest.mark.parametrize("L", [4, 5])
def test_zero_temperature_limit(oracle_lib, L):
    # beta = 10: every threshold for u < 3 is 0, so the chain is the
    # deterministic quench "flip iff u >= 3", colour class by colour class
    J = inputs.couplings(L, 1, seed=9)
    sim = _sim(oracle_lib, L, J, np.array([10.0, 12.0]))
    s0 = sim.spins.copy()
    sim.sweep(5, 0)
    for c in range(2):
        for slot in range(2):
            assert np.array_equal(sim.spins[0, c, slot], bf.zero_temperature_sweeps(L, J[0], s0[0, c, slot], 5))


def test_infinite_temperature_limit(oracle_lib):
    # beta = 0: thresholds are 2^32 - 1, so a site flips unless the draw is
    # 2^32 - 1; every site belongs to one colour class, so a sweep negates
    # the whole configuration (with these seeds no draw equals 2^32 - 1)
    for L in (4, 5):
        J = inputs.couplings(L, 1, seed=3)
        sim = _sim(oracle_lib, L, J, np.array([0.0, 0.0, 0.0]))
        s0 = sim.spins.copy()
        sim.sweep(3, 0)
        assert np.array_equal(sim.spins, -s0)


def test_frozen_ferromagnet(oracle_lib):
    # all J = +1, aligned start, beta >= 1.85 makes the u = 0 threshold 0:
    # no spin can ever flip and E stays -3N through PT swaps
    L = 6
    J = inputs.ferro_couplings(L, 2)
    sim = _sim(oracle_lib, L, J, inputs.geometric_betas(4, 0.3, 0.54))
    sim.set_state(np.ones_like(sim.spins), sim.temp_of_slot, 0)
    sim.sweep(40, 1)
    assert np.all(sim.spins == 1)
    E, q = sim.observables()
    assert np.all(E == -3 * L ** 3)
    assert np.all(q == L ** 3)


def test_ferro_pt_reaches_ground_state(oracle_lib):
    # ferromagnet from a random start with a ladder down to T = 0.5: the
    # coldest temperature reaches the ground state E = -3N
    L = 4
    J = inputs.ferro_couplings(L, 1)
    sim = _sim(oracle_lib, L, J, inputs.geometric_betas(8, 0.5, 6.0), seed=21)
    sim.sweep(400, 1)
    E, _ = sim.observables()
    assert np.all(E[0, :, 0] == -3 * L ** 3)


def test_gauge_invariance(oracle_lib):
    # acceptance depends on u only and u is gauge invariant, so the gauge
    # image of a trajectory is the trajectory of the gauge image, bit for bit
    for L in (4, 5):
        rng = np.random.default_rng(100 + L)
        R = 2
        J = inputs.couplings(L, R, seed=8)
        betas = inputs.geometric_betas(9, 0.4, 2.0)
        a = _sim(oracle_lib, L, J, betas, seed=99)
        tau = rng.choice(np.array([-1, 1], dtype=np.int8), size=(R, L ** 3))
        Jg = np.empty_like(J)
        sg = np.empty_like(a.spins)
        for r in range(R):
            Jg[r], _ = bf.gauge(L, J[r], a.spins[r, 0, 0], tau[r])
            sg[r] = a.spins[r] * tau[r]
        b = _sim(oracle_lib, L, Jg, betas, seed=99)
        b.set_state(sg, a.temp_of_slot, 0)
        for _ in range(4):
            a.sweep(7, 2)
            b.sweep(7, 2)
            assert np.array_equal(b.spins, a.spins * tau[:, None, None, :])
            assert np.array_equal(b.temp_of_slot, a.temp_of_slot)
            assert np.array_equal(b.observables()[0], a.observables()[0])
        # global flip is the special case tau = -1 everywhere
        c = _sim(oracle_lib, L, J, betas, seed=99)
        d = _sim(oracle_lib, L, J, betas, seed=99)
        d.set_state(-c.spins, c.temp_of_slot, 0)
        c.sweep(10, 1)
        d.sweep(10, 1)
        assert np.array_equal(d.spins, -c.spins)


@pytest.mark.parametrize("stream", ["words", "planes"])
def test_exact_boltzmann_distribution_L2(oracle_lib, stream):
    """Time averages at every temperature index against exact enumeration of
    the 2^8 states of the L = 2 lattice (24 bonds), including the expected
    swap acceptance of every pair; the bound is 5 standard errors estimated
    from batch means.  Both flip-draw streams obey the same law."""
    L, R = 2, 24
    J1 = inputs.couplings(L, 1, seed=2024)[0]
    J = np.repeat(J1[None], R, axis=0)
    betas = np.array([1.1, 0.75, 0.5, 0.3])
    n_T = len(betas)
    sim = _sim(oracle_lib, L, J, betas, seed=7, stats=True, rng=stream)
    spectrum = bf.enumerate_energies(L, J1)
    sim.sweep(200, 1)                                       # burn-in
    sim.flip_tries[...] = 0
    sim.flip_acc[...] = 0
    sim.swap_tries[...] = 0
    sim.swap_acc[...] = 0
    n_batches, per_batch = 20, 600
    levels = np.unique(spectrum)
    hist = np.zeros((n_batches, n_T, len(levels)))
    swap_rate = np.zeros((n_batches, n_T - 1))
    for b in range(n_batches):
        tries0, acc0 = sim.swap_tries.copy(), sim.swap_acc.copy()
        for _ in range(per_batch):
            sim.sweep(1, 1)
            E, _ = sim.observables()
            for k in range(n_T):
                hist[b, k] += np.bincount(np.searchsorted(levels, E[:, :, k].ravel()), minlength=len(levels))
        swap_rate[b] = (sim.swap_acc - acc0) / (sim.swap_tries - tries0)
    hist /= hist.sum(axis=2, keepdims=True)
    for k in range(n_T):
        vals, p = bf.boltzmann_pdf(spectrum, betas[k])
        assert np.array_equal(vals, levels)
        mean = hist[:, k].mean(axis=0)
        err = hist[:, k].std(axis=0, ddof=1) / math.sqrt(n_batches)
        assert np.all(np.abs(mean - p) <= 5 * err + 2e-3), (k, mean, p)
    for k in range(n_T - 1):
        vals, pk = bf.boltzmann_pdf(spectrum, betas[k])
        _, pk1 = bf.boltzmann_pdf(spectrum, betas[k + 1])
        dE = vals[:, None] - vals[None, :]
        expect = float(np.sum(pk[:, None] * pk1[None, :] * np.minimum(1.0, np.exp((betas[k] - betas[k + 1]) * dE))))
        mean = swap_rate[:, k].mean()
        err = swap_rate[:, k].std(ddof=1) / math.sqrt(n_batches)
        assert abs(mean - expect) <= 5 * err + 2e-3, (k, mean, expect)
    # acceptance per (temperature, u) class equals threshold / 2^32
    for k in range(n_T):
        for u in range(7):
            n = sim.flip_tries[k, u]
            if n < 100:
                continue
            p = 1.0 if u >= 3 else oracle_lib.flip_threshold(betas[k], u) / 2 ** 32
            got = sim.flip_acc[k, u] / n
            assert abs(got - p) <= 5 * math.sqrt(max(p * (1 - p), 1e-12) / n) + 1e-9, (k, u, got, p)


# --------------------------------------------------------------------------
# Observables by temperature index and the initial-spin stream
# --------------------------------------------------------------------------
@pytest.mark.parametrize("L", [2, 3, 4])
def test_observables_by_temperature_index(oracle_lib, L):
    """Energy and overlap per temperature index (Sec. 4.1 measurement; the
    overlap between the two copies that enters the Binder ratio of Sec. 5.3)
    for random spins and a different random slot permutation in every
    ladder, against numpy: E[r][c][k] = H of copy c's slot at temperature k,
    q[r][k] = sum_i s_i(copy 0 at T_k) s_i(copy 1 at T_k).

    Plausible mistakes this catches, each checked by planting it in a copy of
    the oracle: looking copy 1's slot up through copy 0's permutation;
    summing s0 * s0 (or s1 * s1) in place of s0 * s1; indexing q or E by slot
    instead of by temperature; using temp_of_slot where its inverse is meant."""
    rng = np.random.default_rng(500 + L)
    R, n_T = 3, 7
    J = inputs.couplings(L, R, seed=40 + L)
    sim = _sim(oracle_lib, L, J, inputs.geometric_betas(n_T, 0.5, 2.0))
    for _ in range(3):
        spins = rng.choice(np.array([-1, 1], dtype=np.int8), size=sim.spins.shape)
        perm = np.stack([np.stack([rng.permutation(n_T) for _ in range(2)]) for _ in range(R)]).astype(np.int32)
        # the two copies of a realization never share a permutation here
        for r in range(R):
            while np.array_equal(perm[r, 0], perm[r, 1]):
                perm[r, 1] = rng.permutation(n_T)
        sim.set_state(spins, perm, 0)
        E, q = sim.observables()
        for r in range(R):
            slot_at = [np.empty(n_T, dtype=np.int64) for _ in range(2)]
            for c in range(2):
                for slot in range(n_T):
                    slot_at[c][perm[r, c, slot]] = slot
            for k in range(n_T):
                a, b = slot_at[0][k], slot_at[1][k]
                expect_q = int(np.dot(spins[r, 0, a].astype(np.int64), spins[r, 1, b].astype(np.int64)))
                assert q[r, k] == expect_q, (r, k)
                for c in range(2):
                    assert E[r, c, k] == bf.energy(L, J[r], spins[r, c, slot_at[c][k]]), (r, c, k)


def test_initial_spins_from_rocrand_blocks(oracle_lib, rocrand_probe):
    """orc_init's spins rebuilt from rocRAND's Philox4x32-10 blocks with the
    initial-spin stream of the library's header: spin (realization id r,
    copy c, slot s, site i) is +1 iff bit 0 of word s & 3 of
    block(c0 = i, c1 = 0, c2 = r, c3 = 2 << 28 | c << 24 | s >> 2) is set,
    key (lo32(seed), hi32(seed)); the permutation starts as the identity.

    Plausible mistakes this catches: a wrong domain or copy bit in c3;
    counting slot groups by slot instead of slot >> 2; the wrong output word
    or bit; the realization index in place of its id; the seed halves
    swapped."""
    L, n_T = 3, 6                     # a ragged last slot group
    rids = np.array([5, 9], dtype=np.int32)
    seed = 0x0123456789ABCDEF
    J = inputs.couplings(L, len(rids), seed=3)
    sim = _sim(oracle_lib, L, J, inputs.geometric_betas(n_T, 0.5, 2.0), seed=seed, rid=rids)
    N = L ** 3
    rows, index = [], []
    for r_idx, rid in enumerate(rids):
        for c in range(2):
            for g in range((n_T + 3) // 4):
                for i in range(N):
                    rows.append((i, 0, int(rid), (2 << 28) | (c << 24) | g, seed & 0xFFFFFFFF, seed >> 32))
                    index.append((r_idx, c, g, i))
    text = "\n".join(" ".join(str(v) for v in row) for row in rows) + "\n"
    res = subprocess.run([rocrand_probe], input=text, capture_output=True, text=True, check=True)
    blocks = [list(map(int, line.split())) for line in res.stdout.strip().splitlines()]
    assert len(blocks) == len(rows)
    expect = np.zeros_like(sim.spins)
    for (r_idx, c, g, i), blk in zip(index, blocks):
        for w in range(4):
            s = 4 * g + w
            if s < n_T:
                expect[r_idx, c, s, i] = 1 if blk[w] & 1 else -1
    assert np.array_equal(sim.spins, expect)
    assert np.array_equal(sim.temp_of_slot, np.tile(np.arange(n_T, dtype=np.int32), (len(rids), 2, 1)))
    assert sim.t == 0


# --------------------------------------------------------------------------
# Measurements: overlap moments and plane-sum autocorrelations (Sec. 5)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("L", [2, 3, 4, 5])
def test_measure_against_numpy_fft(oracle_lib, L):
    """Plane sums, their autocorrelation and the overlap moments against a
    numpy evaluation: |FFT of the plane sums|^2 summed over the axes equals
    sum_d C[d] cos(2 pi m d / L) for every m; q^4 exactly in 128 bits."""
    rng = np.random.default_rng(40 + L)
    R, n_T = 2, 5
    J = inputs.couplings(L, R, seed=L)
    sim = _sim(oracle_lib, L, J, inputs.geometric_betas(n_T, 0.5, 2.0))
    acc = sim.new_measurements()
    expect_q2 = np.zeros((R, n_T), dtype=object)
    expect_q4 = np.zeros((R, n_T), dtype=object)
    expect_c = np.zeros((R, n_T, L), dtype=np.int64)
    for rep in range(4):
        spins = rng.choice(np.array([-1, 1], dtype=np.int8), size=sim.spins.shape)
        perm = np.stack([np.stack([rng.permutation(n_T) for _ in range(2)]) for _ in range(R)]).astype(np.int32)
        sim.set_state(spins, perm, 0)
        sim.measure(acc)
        for r in range(R):
            sot = [np.argsort(perm[r, c]) for c in range(2)]
            for k in range(n_T):
                qf = (spins[r, 0, sot[0][k]].astype(np.int64) * spins[r, 1, sot[1][k]]).reshape(L, L, L)  # z, y, x
                planes = [qf.sum(axis=(0, 1)), qf.sum(axis=(0, 2)), qf.sum(axis=(1, 2))]          # x, y, z
                q = int(qf.sum())
                expect_q2[r, k] += q * q
                expect_q4[r, k] += q ** 4
                for Q in planes:
                    expect_c[r, k] += np.array([int(np.dot(Q, np.roll(Q, -d))) for d in range(L)])
                # the FFT identity on this single measurement
                c1 = sum(np.array([int(np.dot(Q, np.roll(Q, -d))) for d in range(L)]) for Q in planes)
                power = sum(np.abs(np.fft.fft(Q)) ** 2 for Q in planes)
                for m in range(L):
                    assert abs(float(np.dot(c1, np.cos(2 * math.pi * m * np.arange(L) / L))) - power[m]) < 1e-6
    count, q2, q4, c = acc
    assert np.all(count == 4)
    for r in range(R):
        for k in range(n_T):
            assert int(q2[r, k]) == expect_q2[r, k]
            assert int(q4[r, k, 0]) + (int(q4[r, k, 1]) << 64) == expect_q4[r, k]
    assert np.array_equal(c, expect_c)


def test_binder_and_xi_closed_forms(oracle_lib):
    """g = 1 when every measurement has |q| = N (identical copies); xi from an
    Ornstein-Zernike form chi(k) = chi(0) / (1 + (2 sin(k/2))^2 xi^2) is
    recovered exactly; a field uncorrelated between sites has xi = 0."""
    L, R, n_T = 4, 3, 2
    N = L ** 3
    J = inputs.couplings(L, R, seed=1)
    sim = _sim(oracle_lib, L, J, inputs.geometric_betas(n_T, 0.5, 2.0))
    s = sim.spins.copy()
    s[:, 1] = s[:, 0]
    sim.set_state(s, np.tile(np.arange(n_T, dtype=np.int32), (R, 2, 1)), 0)
    acc = sim.new_measurements()
    for _ in range(3):
        sim.measure(acc)
    g, _ = oracle_lib.binder_and_xi(acc, L)
    assert np.allclose(g, 1.0, rtol=0, atol=1e-12)
    # synthetic accumulators with a prescribed chi(0) / chi(k)
    k = 2 * math.pi / L
    for xi in (0.0, 0.7, 2.5):
        chi0 = 40.0
        chik = chi0 / (1 + (2 * math.sin(k / 2)) ** 2 * xi ** 2)
        # one realization, one temperature: C[d] = A + B cos(k d) gives sum_d C cos(k d) = B L / 2
        q2 = chi0 * N
        B = chik * 3 * N * 2 / L
        A = (q2 * 3 - B * sum(math.cos(k * d) for d in range(L))) / L   # sum_d C[d] = 3 q^2
        Cd = np.array([A + B * math.cos(k * d) for d in range(L)])
        acc2 = (np.ones((1, 1), np.int64), np.array([[q2]]), np.zeros((1, 1, 2), np.uint64), Cd[None, None, :])
        _, xl = oracle_lib.binder_and_xi(acc2, L)
        assert abs(xl[0] * L - xi) < 1e-9


# --------------------------------------------------------------------------
# External field h (Eq. 1), a multiple of 1/4
# --------------------------------------------------------------------------
@pytest.mark.parametrize("h", [0.75, -1.25])
def test_exact_boltzmann_with_field_L2(oracle_lib, h):
    """Joint distribution of (bond energy, magnetization) at every temperature
    index against exact enumeration of the 2^8 states with weights
    exp(-beta (E - h M)), and the expected swap acceptance of every pair."""
    L, R = 2, 24
    J1 = inputs.couplings(L, 1, seed=77)[0]
    J = np.repeat(J1[None], R, axis=0)
    betas = np.array([1.0, 0.7, 0.45, 0.3])
    n_T = len(betas)
    sim = _sim(oracle_lib, L, J, betas, seed=5, stats=True, h=h)
    Eb, Mg = bf.enumerate_energy_magnetization(L, J1)
    Etot = Eb - h * Mg
    keys = sorted(set(zip(Eb.tolist(), Mg.tolist())))
    index = {k: n for n, k in enumerate(keys)}
    sim.sweep(200, 1)
    sim.swap_tries[...] = 0
    sim.swap_acc[...] = 0
    n_batches, per_batch = 20, 500
    hist = np.zeros((n_batches, n_T, len(keys)))
    swap_rate = np.zeros((n_batches, n_T - 1))
    for b in range(n_batches):
        tries0, acc0 = sim.swap_tries.copy(), sim.swap_acc.copy()
        for _ in range(per_batch):
            sim.sweep(1, 1)
            E, _ = sim.observables()
            M = sim.magnetization()
            for k in range(n_T):
                for e, m in zip(E[:, :, k].ravel().tolist(), M[:, :, k].ravel().tolist()):
                    hist[b, k, index[(e, m)]] += 1
        swap_rate[b] = (sim.swap_acc - acc0) / (sim.swap_tries - tries0)
    hist /= hist.sum(axis=2, keepdims=True)
    state_key = np.array([index[(e, m)] for e, m in zip(Eb.tolist(), Mg.tolist())])
    for k in range(n_T):
        w = np.exp(-betas[k] * (Etot - Etot.min()))
        p = np.bincount(state_key, weights=w, minlength=len(keys))
        p /= p.sum()
        mean = hist[:, k].mean(axis=0)
        err = hist[:, k].std(axis=0, ddof=1) / math.sqrt(n_batches)
        assert np.all(np.abs(mean - p) <= 5 * err + 2e-3), (k, mean, p)
    for k in range(n_T - 1):
        wk = np.exp(-betas[k] * (Etot - Etot.min()))
        wk1 = np.exp(-betas[k + 1] * (Etot - Etot.min()))
        pk, pk1 = wk / wk.sum(), wk1 / wk1.sum()
        dE = Etot[:, None] - Etot[None, :]
        expect = float(np.sum(pk[:, None] * pk1[None, :] * np.minimum(1.0, np.exp((betas[k] - betas[k + 1]) * dE))))
        mean = swap_rate[:, k].mean()
        err = swap_rate[:, k].std(ddof=1) / math.sqrt(n_batches)
        assert abs(mean - expect) <= 5 * err + 2e-3, (k, mean, expect)


@pytest.mark.parametrize("L,h", [(4, 0.25), (5, -1.5), (4, 3.0)])
def test_zero_temperature_limit_with_field(oracle_lib, L, h):
    """beta = 60 makes every threshold of a positive cost (>= 1/2) zero: the
    chain is the quench 'flip iff 12 - 4u + 2 h s <= 0'."""
    J = inputs.couplings(L, 1, seed=19)
    sim = _sim(oracle_lib, L, J, np.array([60.0, 70.0]), h=h)
    s0 = sim.spins.copy()
    sim.sweep(4, 0)
    for c in range(2):
        for slot in range(2):
            assert np.array_equal(sim.spins[0, c, slot],
                                  bf.zero_temperature_sweeps_field(L, J[0], s0[0, c, slot], 4, h))


def test_field_reversal_symmetry(oracle_lib):
    """Reversing every spin and the field leaves every flip cost and every
    energy difference unchanged: the reversed chain is the reversed image of
    the original, swaps included, bit for bit."""
    for L in (4, 5):
        J = inputs.couplings(L, 2, seed=31)
        betas = inputs.geometric_betas(7, 0.4, 2.0)
        a = _sim(oracle_lib, L, J, betas, seed=8, h=0.75)
        b = _sim(oracle_lib, L, J, betas, seed=8, h=-0.75)
        b.set_state(-a.spins, a.temp_of_slot, 0)
        for _ in range(3):
            a.sweep(6, 2)
            b.sweep(6, 2)
            assert np.array_equal(b.spins, -a.spins)
            assert np.array_equal(b.temp_of_slot, a.temp_of_slot)
            assert np.array_equal(b.magnetization(), -a.magnetization())


@pytest.mark.parametrize("h,beta", [(2.0, 1.5), (-2.0, 3.0)])
def test_frozen_ferromagnet_in_field(oracle_lib, h, beta):
    """All J = +1, every spin +1: the cheapest flip costs 12 + 2h > 0, and at
    these beta its threshold is 0, so the state never changes: E = -3N,
    M = N through sweeps and swaps."""
    L = 4
    N = L ** 3
    assert oracle_lib.flip_threshold_h(beta, 0, 1, h) == 0
    J = inputs.ferro_couplings(L, 2)
    sim = _sim(oracle_lib, L, J, np.array([beta, beta * 1.2, beta * 1.5]), h=h)
    sim.set_state(np.ones_like(sim.spins), sim.temp_of_slot, 0)
    sim.sweep(30, 1)
    assert np.all(sim.spins == 1)
    assert np.all(sim.observables()[0] == -3 * N) and np.all(sim.magnetization() == N)
