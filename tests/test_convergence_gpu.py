"""Parallel tempering against plain Metropolis on the 8^3 Edwards-Anderson
spin glass at 1/T = 2 (the paper's convergence study, Sec. 5.3, Fig. qvst):
the Binder ratio of the coldest temperature, measured over windows of sweeps
[2^k, 2^(k+1)), settles with PT by about 10^5 sweeps, while the same ladder
without swaps is still far from it; at the hottest temperature (T = 2, well
above the spin-glass transition) the two runs agree, the paper's check that
results with and without swaps are consistent.

Realizations are independent, so errors are jackknife errors over them.
Every run is a fixed function of its seed (the chains are bit-exact), so the
thresholds below were set once from the measured values with a wide margin.
"""
import numpy as np
import pytest

from paper_1311_5582_amd import binding as B
from paper_1311_5582_amd import inputs

pytestmark = pytest.mark.gpu

L, R, N_T, SEED = 8, 256, 16, 4242
T_MIN, T_MAX = 0.5, 2.0
K_FIRST, K_LAST = 10, 16            # windows [2^k, 2^(k+1)), the last ends at 131072 sweeps
EVERY = 16                          # sweeps between measurements


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    B.lib()


def _moments(sim):
    """Per-realization thermal averages <q^2>/N^2 and <q^4>/N^4, [R][n_T]."""
    count, q2, q4, _ = sim.measurements()
    n = count.astype(np.float64)
    N = float(L ** 3)
    m2 = q2.astype(np.float64) / n / N ** 2
    m4 = (q4[..., 0].astype(np.float64) + np.ldexp(q4[..., 1].astype(np.float64), 64)) / n / N ** 4
    return m2, m4


def _binder(m2, m4):
    return 0.5 * (3.0 - m4.mean(0) / m2.mean(0) ** 2)


def _jackknife(m2, m4, f):
    """f(m2, m4) per temperature with its jackknife error over realizations."""
    full = f(m2, m4)
    r = m2.shape[0]
    s2, s4 = m2.sum(0), m4.sum(0)
    loo = np.array([f(((s2 - m2[i]) / (r - 1))[None], ((s4 - m4[i]) / (r - 1))[None]) for i in range(r)])
    err = np.sqrt((r - 1) / r * ((loo - loo.mean(0)) ** 2).sum(0))
    return full, err


def _run_windows(swap_every):
    J = inputs.couplings(L, R, SEED)
    betas = inputs.geometric_betas(N_T, T_MIN, T_MAX)
    sim = B.Sim(L, J, betas, SEED)
    sim.sweep(2 ** K_FIRST, swap_every)
    out = {}
    for k in range(K_FIRST, K_LAST + 1):
        sim.reset_measurements()
        for _ in range(2 ** k // EVERY):
            sim.sweep(EVERY, swap_every)
            sim.measure()
        m2, m4 = _moments(sim)
        g, g_err = _jackknife(m2, m4, lambda a, b: _binder(a, b))
        q2, q2_err = _jackknife(m2, m4, lambda a, b: a.mean(0))
        out[k] = dict(g=g, g_err=g_err, q2=q2, q2_err=q2_err)
        print(f"[convergence] swap_every={swap_every} window [2^{k}, 2^{k + 1}): g(T={T_MIN}) = "
              f"{g[0]:.4f} +- {g_err[0]:.4f}, g(T={T_MAX}) = {g[-1]:.4f} +- {g_err[-1]:.4f}, "
              f"q2(T={T_MIN}) = {q2[0]:.4f} +- {q2_err[0]:.4f}", flush=True)
    assert sim.state()[2] == 2 ** (K_LAST + 1)
    sim.close()
    return out


@pytest.fixture(scope="module")
def runs():
    return {"pt": _run_windows(1), "nopt": _run_windows(0)}


def test_pt_binder_settles_by_1e5_sweeps(runs):
    """With swaps after every sweep the cold Binder ratio is at its late value
    in every window from [2^13, 2^14) on (measured: 0.917 +- 0.006 from 2^12
    sweeps through 2^17)."""
    last = runs["pt"][K_LAST]
    for k in range(13, K_LAST):
        w = runs["pt"][k]
        diff = abs(w["g"][0] - last["g"][0])
        sigma = np.hypot(w["g_err"][0], last["g_err"][0])
        assert diff < 3.0 * sigma, (k, diff, sigma)


def test_no_pt_is_far_from_equilibrium(runs):
    """Without swaps the cold copies are still stuck at 2^17 sweeps: their
    Binder ratio and overlap are far below the PT values (measured: g = 0.17
    +- 0.07 against 0.918 +- 0.006, q^2 = 0.153 against 0.615)."""
    p, n = runs["pt"][K_LAST], runs["nopt"][K_LAST]
    sigma = np.hypot(p["g_err"][0], n["g_err"][0])
    assert p["g"][0] - n["g"][0] > 5.0 * sigma, (p["g"][0], n["g"][0], sigma)
    sq = np.hypot(p["q2_err"][0], n["q2_err"][0])
    assert p["q2"][0] - n["q2"][0] > 5.0 * sq, (p["q2"][0], n["q2"][0], sq)


def test_hot_end_consistent_with_and_without_pt(runs):
    """At T = 2 both runs are equilibrated: overlap and Binder ratio agree."""
    p, n = runs["pt"][K_LAST], runs["nopt"][K_LAST]
    assert abs(p["q2"][-1] - n["q2"][-1]) < 4.0 * np.hypot(p["q2_err"][-1], n["q2_err"][-1])
    assert abs(p["g"][-1] - n["g"][-1]) < 4.0 * np.hypot(p["g_err"][-1], n["g_err"][-1])
