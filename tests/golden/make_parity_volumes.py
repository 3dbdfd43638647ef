"""Write tests/golden/parity_volumes.json: expected results of the benchmark
workloads at parity-test volume, computed by the CPU oracle alone.

Only the oracle (oracle/) and the seeded input generators
(paper_1311_5582_amd.inputs, which hold none of the method's arithmetic) are
used here; nothing comes from the HIP library.  Every case runs one
realization per task (realization r of a job depends on (seed, r) only), so
any subset of a job's realizations is reproduced exactly.  Per realization
the file stores the energies E [2][n_T] and overlaps q [n_T] by temperature
index, the permutation temp_of_slot [2][n_T], and the SHA-256 of the final
spins (int8 [2][n_T][L^3], +1/-1, by slot).

Cases (sizes of the workloads the benchmark runs):
  L16_R64_1000   L=16, all 64 realizations, 32 temperatures, 1000 sweeps, PT every sweep
  L16_R64_10000  L=16, 4 realizations, the full 10^4 sweeps
  batched_5000   the five uneven jobs (L = 8..20), 4 realizations each, 5000 sweeps
  L24_R256_2000  L=24, 2 realizations, 48 temperatures, 2000 sweeps, PT every 10
  serving_2000   every job of the 64-job serving trace, one realization chosen from
                 its seed, min(sweeps, 2000) sweeps

Run: python tests/golden/make_parity_volumes.py [--jobs N] [--only CASE ...]
"""
import argparse
import concurrent.futures as cf
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1311_5582_amd import inputs  # noqa: E402

OUT = os.path.join(HERE, "parity_volumes.json")


def spins_sha256(spins):
    return hashlib.sha256(np.ascontiguousarray(spins, dtype=np.int8).tobytes()).hexdigest()


def pick(seed, R, m):
    """m-th realization drawn for a job from its seed (distinct for m < R)."""
    chosen = []
    k = 0
    while len(chosen) < m:
        r = inputs.splitmix64((int(seed) + k) & 0xFFFFFFFFFFFFFFFF) % R
        if r not in chosen:
            chosen.append(int(r))
        k += 1
    return chosen


def cases():
    out = []
    c = inputs.CONFIGS["L16_R64"]
    out.append(dict(name="L16_R64_1000", L=c["L"], R=c["R"], n_T=c["n_T"], t_min=c["t_min"], t_max=c["t_max"],
                    seed=c["seed"], sweeps=1000, swap_every=c["swap_every"], rids=list(range(c["R"]))))
    out.append(dict(name="L16_R64_10000", L=c["L"], R=c["R"], n_T=c["n_T"], t_min=c["t_min"], t_max=c["t_max"],
                    seed=c["seed"], sweeps=10_000, swap_every=c["swap_every"], rids=[0, 21, 42, 63]))
    for k, j in enumerate(inputs.BATCHED_JOBS):
        out.append(dict(name=f"batched_5000/job{k}", L=j["L"], R=j["R"], n_T=j["n_T"], t_min=j["t_min"],
                        t_max=j["t_max"], seed=j["seed"], sweeps=j["sweeps"], swap_every=j["swap_every"],
                        rids=pick(j["seed"], j["R"], 4)))
    c = inputs.CONFIGS["L24_R256"]
    out.append(dict(name="L24_R256_2000", L=c["L"], R=c["R"], n_T=c["n_T"], t_min=c["t_min"], t_max=c["t_max"],
                    seed=c["seed"], sweeps=2000, swap_every=c["swap_every"], rids=[0, 255]))
    for j in inputs.serving_trace(n_jobs=64, rate_per_s=20.0):
        out.append(dict(name=f"serving_2000/job{j['job_id']}", L=j["L"], R=j["R"], n_T=j["n_T"], t_min=j["t_min"],
                        t_max=j["t_max"], seed=j["seed"], sweeps=min(j["sweeps"], 2000), swap_every=j["swap_every"],
                        rids=pick(j["seed"], j["R"], 1)))
    return out


def run_one(case, r):
    L = case["L"]
    J = inputs.couplings(L, 1, case["seed"], r0=r)
    betas = inputs.geometric_betas(case["n_T"], case["t_min"], case["t_max"])
    o = oracle.OracleSim(L, J, betas, case["seed"], rid=np.array([r]))
    o.sweep(case["sweeps"], case["swap_every"])
    E, q = o.observables()
    return dict(r=r, t=o.t, E=E[0].tolist(), q=q[0].tolist(), perm=o.temp_of_slot[0].tolist(),
                spins_sha256=spins_sha256(o.spins[0]))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=os.cpu_count() or 1)
    ap.add_argument("--only", nargs="*", default=None, help="case-name prefixes to (re)compute")
    args = ap.parse_args()
    doc = json.load(open(OUT)) if os.path.exists(OUT) else {"cases": {}}
    todo = [c for c in cases() if args.only is None or any(c["name"].startswith(p) for p in args.only)]
    tasks = [(c, r) for c in todo for r in c["rids"]]
    # longest tasks first
    tasks.sort(key=lambda cr: -cr[0]["sweeps"] * cr[0]["L"] ** 3 * cr[0]["n_T"])
    results = {c["name"]: {} for c in todo}
    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(max_workers=args.jobs) as ex:
        futs = {ex.submit(run_one, c, r): (c["name"], r) for c, r in tasks}
        for n, f in enumerate(cf.as_completed(futs)):
            name, r = futs[f]
            results[name][r] = f.result()
            print(f"[{time.perf_counter() - t0:7.1f} s] {n + 1}/{len(tasks)} {name} r={r}", flush=True)
    for c in todo:
        meta = {k: c[k] for k in ("L", "R", "n_T", "t_min", "t_max", "seed", "sweeps", "swap_every")}
        meta["realizations"] = [results[c["name"]][r] for r in c["rids"]]
        doc["cases"][c["name"]] = meta
    doc["generator"] = "tests/golden/make_parity_volumes.py (CPU oracle only)"
    with open(OUT + ".tmp", "w") as f:
        json.dump(doc, f, separators=(",", ":"))
    os.replace(OUT + ".tmp", OUT)
    print(f"wrote {OUT}", flush=True)


if __name__ == "__main__":
    main()
