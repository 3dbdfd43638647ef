"""Replay a job trace against the continuous-batching server by wall clock.

Each job is submitted when its arrival time has passed; the server admits it
when its HBM footprint fits, runs it in the shared launch, and retires it.
Latency = completion time - arrival time (queueing included).
"""
import time

import numpy as np

from paper_1311_5582_amd import binding as B
from paper_1311_5582_amd import inputs


def run_trace(trace, server, realize=None, idle_sleep_s=0.0005, on_done=None):
    """trace: list of dicts with arrival_s, L, R, n_T, t_min, t_max, sweeps, swap_every, seed.
    realize(job) -> (couplings, betas); default draws them from the inputs module.
    Returns (records, wall_s): one record per job with arrival, admitted-by, done, latency."""
    realize = realize or (lambda j: (inputs.couplings(j["L"], j["R"], j["seed"]),
                                     inputs.geometric_betas(j["n_T"], j["t_min"], j["t_max"])))
    pending = sorted(trace, key=lambda j: j["arrival_s"])
    prepared = [realize(j) for j in pending]   # host-side input generation is not part of the service
    ids, records = {}, {}
    t0 = time.perf_counter()
    k = 0
    while k < len(pending) or len(records) < len(pending):
        now = time.perf_counter() - t0
        while k < len(pending) and pending[k]["arrival_s"] <= now:
            j = pending[k]
            J, betas = prepared[k]
            jid = server.submit(j["L"], J, betas, j["seed"], j["sweeps"], j["swap_every"])
            ids[jid] = j
            k += 1
        running, queued, finished = server.step()
        now = time.perf_counter() - t0
        for jid, j in ids.items():
            if jid in records:
                continue
            st, _ = server.status(jid)
            if st in (B.JOB_DONE, B.JOB_FAILED, B.JOB_CANCELLED):
                records[jid] = dict(job=j, status=st, done_s=now, latency_s=now - j["arrival_s"])
                if on_done:
                    on_done(jid, j, st)
        if running == 0 and queued == 0 and k < len(pending):
            time.sleep(min(max(pending[k]["arrival_s"] - (time.perf_counter() - t0), 0.0), 0.05) + idle_sleep_s)
    return records, time.perf_counter() - t0


def latency_summary(records):
    lat = np.array([r["latency_s"] for r in records.values()])
    flips = sum(r["job"]["sweeps"] * r["job"]["L"] ** 3 * r["job"]["n_T"] * r["job"]["R"] * 2 for r in records.values())
    done_last = max(r["done_s"] for r in records.values())
    worst = sorted(records.values(), key=lambda r: -r["latency_s"])[:3]
    worst = [dict(job_id=r["job"].get("job_id"), L=r["job"]["L"], R=r["job"]["R"], n_T=r["job"]["n_T"],
                  sweeps=r["job"]["sweeps"], arrival_s=round(r["job"]["arrival_s"], 3),
                  latency_s=round(r["latency_s"], 3)) for r in worst]
    return dict(jobs=len(lat), p50_s=float(np.percentile(lat, 50)), p99_s=float(np.percentile(lat, 99)),
                mean_s=float(lat.mean()), max_s=float(lat.max()), flips=float(flips), done_last_s=float(done_last),
                worst=worst)
