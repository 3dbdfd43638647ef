"""Seeded synthetic inputs: couplings, temperature ladders, workload shapes.

This module holds no part of the simulation's arithmetic.  It only draws the
inputs both sides receive (the HIP library and, in tests, the CPU oracle):
+-J couplings with p = 1/2 (the bimodal zero-mean distribution of Sec. 2.2),
geometric temperature ladders, and the job mix of the serving workload.
Realization r's couplings depend on (seed, r) only, so any subset of
realizations can be regenerated on its own.
"""
import math

import numpy as np


def couplings(L: int, R: int, seed: int, r0: int = 0) -> np.ndarray:
    """+-1 couplings, int8 [R][L^3][3]; entry [r][i][mu] is the bond between
    site i = x + L(y + Lz) and its +mu neighbour, for realizations r0..r0+R-1."""
    N = L ** 3
    out = np.empty((R, N, 3), dtype=np.int8)
    for k in range(R):
        rng = np.random.default_rng([int(seed) & 0xFFFFFFFF, int(seed) >> 32, r0 + k])
        bits = rng.integers(0, 2, size=(N, 3), dtype=np.int8)
        out[k] = 1 - 2 * bits
    return out


def ferro_couplings(L: int, R: int) -> np.ndarray:
    """All couplings +1 (ferromagnet in the H = -sum J s s convention)."""
    return np.ones((R, L ** 3, 3), dtype=np.int8)


def geometric_betas(n_T: int, t_min: float, t_max: float) -> np.ndarray:
    """Inverse temperatures of a geometric ladder T_k = t_min (t_max/t_min)^(k/(n_T-1)),
    k = 0 the coldest."""
    if n_T == 1:
        return np.array([1.0 / t_min])
    k = np.arange(n_T, dtype=np.float64)
    T = t_min * (t_max / t_min) ** (k / (n_T - 1))
    return 1.0 / T


# ---------------------------------------------------------------------------
# Workload shapes (all synthetic: no dataset exists for this method)
# ---------------------------------------------------------------------------
CONFIGS = {
    # single small job; the oracle runs all of it in seconds
    "plain_L8": dict(L=8, R=1, n_T=16, t_min=0.5, t_max=2.0, sweeps=1000, swap_every=1, seed=1),
    # the paper's lattice size (16^3) with 64 realizations
    "L16_R64": dict(L=16, R=64, n_T=32, t_min=0.4, t_max=2.0, sweeps=10_000, swap_every=1, seed=2),
    # large production lattice, PT every 10 sweeps
    "L24_R256": dict(L=24, R=256, n_T=48, t_min=0.35, t_max=2.0, sweeps=100_000, swap_every=10, seed=4),
}

# uneven jobs sharing one launch: L and ladder length spread together
BATCHED_JOBS = [
    dict(L=L, R=128, n_T=n_T, t_min=0.4, t_max=2.0, sweeps=5000, swap_every=1, seed=300 + j)
    for j, (L, n_T) in enumerate(zip((8, 10, 12, 16, 20), (16, 22, 28, 34, 40)))
]


def splitmix64(x: int) -> int:
    """SplitMix64 finaliser (Steele, Lea, Flood 2014), used to derive job seeds."""
    x = (x + 0x9E3779B97F4A7C15) & 0xFFFFFFFFFFFFFFFF
    x = ((x ^ (x >> 30)) * 0xBF58476D1CE4E5B9) & 0xFFFFFFFFFFFFFFFF
    x = ((x ^ (x >> 27)) * 0x94D049BB133111EB) & 0xFFFFFFFFFFFFFFFF
    return x ^ (x >> 31)


def serving_trace(n_jobs: int = 64, rate_per_s: float = 20.0, seed: int = 5,
                  sweep_median: float = 1e4, sweep_sigma: float = 0.9,
                  sweep_min: int = 1000, sweep_max: int = 100_000):
    """Poisson arrivals; L ~ U{6..20}, R ~ U{32..512}, n_T ~ U{16..48},
    sweeps ~ lognormal(median, sigma) clipped to [sweep_min, sweep_max]."""
    rng = np.random.default_rng(seed)
    t = 0.0
    jobs = []
    for j in range(n_jobs):
        t += rng.exponential(1.0 / rate_per_s)
        sweeps = int(round(math.exp(math.log(sweep_median) + sweep_sigma * rng.standard_normal())))
        jobs.append(dict(job_id=j, arrival_s=t,
                         L=int(rng.integers(6, 21)), R=int(rng.integers(32, 513)),
                         n_T=int(rng.integers(16, 49)), t_min=0.4, t_max=2.0,
                         sweeps=int(min(max(sweeps, sweep_min), sweep_max)), swap_every=1,
                         seed=splitmix64(seed * 1_000_003 + j)))
    return jobs
