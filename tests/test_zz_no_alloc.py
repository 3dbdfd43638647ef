"""The allocation-free batch entry point (ea_sweep_batch_noalloc) against the
allocating one (ea_sweep_batch): identical chains bit for bit, on two calls in
a row that reuse the library's static workspace, the second with a smaller
batch, plus the workspace limits and one realization against the oracle."""
import numpy as np
import pytest

from paper_1311_5582_amd import binding as B
from paper_1311_5582_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    B.lib()


def _make(L, R, n_T, seed):
    return B.Sim(L, inputs.couplings(L, R, seed), inputs.geometric_betas(n_T, 0.4, 2.0), seed)


def _same(a, b, what):
    sa, pa, ta = a.state()
    sb, pb, tb = b.state()
    assert ta == tb, f"{what}: sweep counters differ"
    assert np.array_equal(pa, pb), f"{what}: permutations differ"
    assert np.array_equal(sa, sb), f"{what}: spins differ"
    Ea, qa = a.observables()
    Eb, qb = b.observables()
    assert np.array_equal(Ea, Eb) and np.array_equal(qa, qb), f"{what}: observables differ"
    assert np.array_equal(a.swap_acceptance(), b.swap_acceptance()), f"{what}: swap counts differ"


def test_noalloc_batch_equals_batch(oracle_lib):
    # first call: three jobs (even and odd L, one and two words per site, PT on and off)
    first = [(8, 3, 16, 31), (7, 2, 22, 32), (10, 2, 40, 33)]
    ns1, se1 = [30, 25, 40], [1, 2, 0]
    ref = [_make(*j) for j in first]
    got = [_make(*j) for j in first]
    print(f"[noalloc] call 1: jobs {first} sweeps {ns1} swap_every {se1}", flush=True)
    B.sweep_batch(ref, ns1, se1)
    B.sweep_batch_noalloc(got, ns1, se1)
    for k, (a, b) in enumerate(zip(got, ref)):
        _same(a, b, f"call 1 job {k}")
    # second call: a smaller batch (fewer jobs and ladders) continuing two of the jobs
    ns2, se2 = [12, 9], [3, 1]
    print(f"[noalloc] call 2: jobs {first[:2]} sweeps {ns2} swap_every {se2}", flush=True)
    B.sweep_batch(ref[:2], ns2, se2)
    B.sweep_batch_noalloc(got[:2], ns2, se2)
    for k, (a, b) in enumerate(zip(got, ref)):
        _same(a, b, f"call 2 job {k}")
    # one realization of the continued odd-L job against the oracle
    L, R, n_T, seed = first[1]
    r = 1
    o = oracle_lib.OracleSim(L, inputs.couplings(L, R, seed)[[r]], inputs.geometric_betas(n_T, 0.4, 2.0), seed,
                             rid=np.array([r]))
    o.sweep(ns1[1], se1[1])
    o.sweep(ns2[1], se2[1])
    s, perm, t = got[1].state()
    assert t == ns1[1] + ns2[1] == o.t
    assert np.array_equal(s[r], o.spins[0]) and np.array_equal(perm[r], o.temp_of_slot[0])
    for x in got + ref:
        x.close()


def test_noalloc_limits():
    # more jobs than the workspace holds: refused, nothing runs
    sims = [_make(2, 1, 1, 40 + k) for k in range(257)]
    with pytest.raises(B.EAError) as ei:
        B.sweep_batch_noalloc(sims, [1] * len(sims), [0] * len(sims))
    assert ei.value.code == B.EA_EINVAL and "workspace" in str(ei.value)
    assert all(s.state()[2] == 0 for s in sims)
    # the same jobs within the limit run
    B.sweep_batch_noalloc(sims[:256], [1] * 256, [0] * 256)
    assert all(s.state()[2] == 1 for s in sims[:256])
    for s in sims:
        s.close()
    # more ladders than the workspace holds: refused
    big = [_make(2, 131072, 2, 50), _make(2, 1, 2, 51)]   # 262144 + 2 ladders
    with pytest.raises(B.EAError) as ei:
        B.sweep_batch_noalloc(big, [1, 1], [1, 1])
    assert ei.value.code == B.EA_EINVAL and "ladders" in str(ei.value)
    # jobs with no sweeps do not count against the limit
    B.sweep_batch_noalloc(big, [0, 2], [1, 1])
    assert big[0].state()[2] == 0 and big[1].state()[2] == 2
    for s in big:
        s.close()
