"""Benchmark: picoseconds per spin-flip attempt on one MI355X.

Workload (default): 3D +-J EA model, L = 16 (4096 spins), 64 disorder
realizations x 2 copies, 32 temperatures geometric in T in [0.4, 2.0],
parallel tempering after every sweep, CAMSC layout.  One step = one sweep
launch of --sweeps-per-step sweeps plus one measurement (energies and
overlaps); the default 10 steps x 1000 sweeps is the whole 10^4-sweep job.
ps/flip follows Eq. tsf of the paper: wall time / (sweeps x spins x
temperatures x samples), samples = realizations x 2 copies.

Prints one JSON line.  The roofline object prices the sweep kernel against
the integer issue rate of the chip; the cpu_baseline object times the CPU
oracle on a bounded sample of the same workload.
"""
import argparse
import json
import os
import sys
import threading
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "ps per spin-flip attempt (1 GPU, batched vs plain) + p50/p99 job latency"

# int32 operations per spin-flip attempt that the method itself needs (the
# count is derived in the design notes): a quarter of a Philox4x32-10 block
# (10 rounds x (2 v_mad_u64_u32 + 2 three-input xors) / 4 = 10), the table
# column, address, compare and insert (4), and the share of the bit-parallel
# bond energies (2).  On gfx950 every one of these issues at full rate
# (measured: v_mad_u64_u32 33.4 T/s, v_bitop3 36.1 T/s on 256 CUs).
ALG_OPS_PER_FLIP = 16
# The same for the bit-plane stream: a flip attempt needs the planes up to the
# first one where its draw and threshold differ.  Per 16-slot half a Philox
# block (40 ops) gives 8 planes and is needed 1.06 times on average (all 16
# slots decided within 8 planes with probability (1 - 2^-8)^16): 2.65 ops per
# flip; each plane costs 6 ops per 32 slots (select the threshold bit, compare,
# record, retire, place the plane) over about 8.5 planes: 1.6; bond words and
# their bit-sliced sum (6 xor3, a full-adder tree of 8, masks and the update,
# about 20 ops per 32 slots): 0.63.  About 5 in all.
ALG_OPS_PER_FLIP_PLANES = 5
# MI355X: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz int32 lane-operations per second
PEAK_OPS_PER_S = 256 * 4 * 16 * 2.4e9
KERNEL_SRC = os.path.join(ROOT, "paper_1311_5582_amd", "csrc", "ea_kernels.hip")
PROFILES = os.path.join(ROOT, "profiles")


def kernel_source_hash():
    import hashlib
    return hashlib.sha1(open(KERNEL_SRC, "rb").read()).hexdigest()[:12]


def measured_traffic(workload, layout, rng="words"):
    """HBM bytes per sweep launch from the committed rocprofv3 FETCH_SIZE /
    WRITE_SIZE summary, only if it was taken on the current kernel source."""
    import re
    suffix = "" if rng == "words" else "_" + rng
    path = os.path.join(PROFILES, f"sweep_kernel_{workload}_{layout}{suffix}.md")
    if not os.path.exists(path):
        return None
    m = re.search(r"traffic_bytes_per_launch:\s*(\d+)\s+kernel_sha1:\s*([0-9a-f]+)", open(path).read())
    if not m or m.group(2) != kernel_source_hash():
        return None
    return int(m.group(1))


def cpu_baseline(L, n_T, t_min, t_max, seed, sweeps, threads):
    """Time the oracle: `threads` realizations, one per thread, `sweeps` each."""
    import oracle
    from paper_1311_5582_amd import inputs
    betas = inputs.geometric_betas(n_T, t_min, t_max)
    sims = [oracle.OracleSim(L, inputs.couplings(L, 1, seed, r0=r), betas, seed, rid=np.array([r]))
            for r in range(threads)]
    ths = [threading.Thread(target=s.sweep, args=(sweeps, 1)) for s in sims]
    t0 = time.perf_counter()
    for th in ths:
        th.start()
    for th in ths:
        th.join()
    dt = time.perf_counter() - t0
    flips = sweeps * L ** 3 * n_T * 2 * threads
    return {"value": dt / flips * 1e12, "unit": "ps/flip", "cores": threads, "kind": "oracle",
            "sample": f"{threads} realizations x 2 copies x {n_T} temps, L={L}, {sweeps} sweeps, "
                      f"PT every sweep ({flips:.3g} flip attempts, {dt:.1f} s wall)"}


def bench_other_stream(B, torch, L, J, betas, seed, layout, block_threads, split, rng, sweeps, swap_every, steps):
    """The same workload and launch with the other flip-draw stream (kernel time
    from HIP events on the launch stream, wall time around the steps)."""
    stream = torch.cuda.Stream()
    sim = B.Sim(L, J, betas, seed, layout=layout, block_threads=block_threads, stream=stream, split=split, rng=rng)
    sim.sweep(sweeps, swap_every)
    sim.observables()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    t0 = time.perf_counter()
    for a, b in evs:
        a.record(stream)
        sim.sweep(sweeps, swap_every)
        b.record(stream)
        sim.observables()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    flips = sweeps * L ** 3 * len(betas) * J.shape[0] * 2
    kern = float(np.mean([a.elapsed_time(b) for a, b in evs])) / 1e3
    sim.close()
    return {"rng": rng, "steps": steps, "ps_per_flip": round(wall / (flips * steps) * 1e12, 4),
            "kernel_ps_per_flip": round(kern / flips * 1e12, 4)}


def bench_layout_study(B, torch, inputs, sweeps, steps):
    """The paper's layout comparison (16^3 lattice, PT every 10 sweeps) on the
    benchmark's L=16 job: every layout, one workgroup per ladder, plus CAMSC
    with split ladders and with bit-plane draws."""
    cfg = inputs.CONFIGS["L16_R64"]
    L, R, n_T = cfg["L"], cfg["R"], cfg["n_T"]
    J = inputs.couplings(L, R, cfg["seed"])
    betas = inputs.geometric_betas(n_T, cfg["t_min"], cfg["t_max"])
    flips = sweeps * L ** 3 * n_T * R * 2
    out = {"workload": "L=16, 64 realizations x 2 copies, 32 temperatures, PT every 10 sweeps",
           "sweeps_per_step": sweeps, "steps": steps}
    for name, layout, split, rng in (("amsc1", "amsc1", False, "words"), ("amsc3", "amsc3", False, "words"),
                                     ("amsc4", "amsc4", False, "words"), ("camsc", "camsc", False, "words"),
                                     ("camsc_split", "camsc", True, "words"),
                                     ("camsc_split_planes", "camsc", True, "planes")):
        stream = torch.cuda.Stream()
        sim = B.Sim(L, J, betas, cfg["seed"], layout=layout, stream=stream, split=split, rng=rng)
        sim.sweep(sweeps, 10)
        torch.cuda.synchronize()
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
        for a, b in evs:
            a.record(stream)
            sim.sweep(sweeps, 10)
            b.record(stream)
        torch.cuda.synchronize()
        kern = float(np.mean([a.elapsed_time(b) for a, b in evs])) / 1e3
        out[name] = round(kern / flips * 1e12, 4)
        sim.close()
    return out


def flips_of(job, sweeps):
    return sweeps * job["L"] ** 3 * job["n_T"] * job["R"] * 2


def bench_batched(B, inputs, torch, sweeps, steps):
    """The uneven job set in one graph-captured launch per step vs the same
    jobs launched one after another (plain path), same sweeps."""
    jobs = inputs.BATCHED_JOBS

    def make():
        return [B.Sim(j["L"], inputs.couplings(j["L"], j["R"], j["seed"]),
                      inputs.geometric_betas(j["n_T"], j["t_min"], j["t_max"]), j["seed"]) for j in jobs]

    flips = sum(flips_of(j, sweeps) for j in jobs) * steps
    # plain: each job alone, back to back
    sims = make()
    for s, j in zip(sims, jobs):
        s.sweep(1, j["swap_every"])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        for s, j in zip(sims, jobs):
            s.sweep(sweeps, j["swap_every"])
    torch.cuda.synchronize()
    plain_s = time.perf_counter() - t0
    for s in sims:
        s.close()
    # batched: one plan, graph replay
    sims = make()
    plan = B.Plan(sims, sweeps, [j["swap_every"] for j in jobs], autotune=True)
    plan.run(1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan.run(steps)
    torch.cuda.synchronize()
    batched_s = time.perf_counter() - t0
    info = plan.info()
    plan.close()
    for s in sims:
        s.close()
    return {"workload": "5 jobs L=8,10,12,16,20 x 128 realizations x 2 copies, 16-40 temperatures, PT every sweep",
            "sweeps_per_step": sweeps, "steps": steps, "flips": flips,
            "batched_ps_per_flip": round(batched_s / flips * 1e12, 4),
            "plain_ps_per_flip": round(plain_s / flips * 1e12, 4),
            "speedup": round(plain_s / batched_s, 3), "block_threads": info["block_threads"],
            "units": info["units"], "uses_graph": info["uses_graph"]}


def bench_serving(B, inputs, n_jobs, rate, quantum, sweep_scale=1.0, max_active=0):
    """Poisson job trace through the continuous-batching server (max_active=1:
    the same server as a plain queue, one job on the GPU at a time)."""
    from paper_1311_5582_amd import serve
    trace = inputs.serving_trace(n_jobs=n_jobs, rate_per_s=rate)
    for j in trace:
        j["sweeps"] = max(1, int(j["sweeps"] * sweep_scale))
    srv = B.Server(quantum_sweeps=quantum, max_active=max_active)
    recs, wall = serve.run_trace(trace, srv)
    st = srv.stats()
    srv.close()
    summ = serve.latency_summary(recs)
    return {"jobs": n_jobs, "rate_per_s": round(rate, 3), "quantum_sweeps": quantum, "sweep_scale": sweep_scale,
            "p50_latency_s": round(summ["p50_s"], 4), "p99_latency_s": round(summ["p99_s"], 4),
            "mean_latency_s": round(summ["mean_s"], 4), "wall_s": round(wall, 3),
            "aggregate_ps_per_flip": round(wall / summ["flips"] * 1e12, 4), "steps": st["steps"],
            "plans_built": st["plans_built"], "launches_replayed": st["launches_replayed"]}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--sweeps-per-step", type=int, default=1000)
    ap.add_argument("--workload", default="L16_R64")
    ap.add_argument("--layout", default="camsc", choices=["camsc", "amsc4", "amsc3", "amsc1"])
    ap.add_argument("--block-threads", type=int, default=0)
    ap.add_argument("--rng", default="words", choices=["words", "planes"],
                    help="flip-draw stream: one Philox word per flip, or bit planes compared MSB first")
    ap.add_argument("--layout-study", action="store_true",
                    help="also time every spin layout on the L=16 job with PT every 10 sweeps")
    ap.add_argument("--no-other-stream", action="store_true",
                    help="skip timing the same workload with the other flip-draw stream")
    ap.add_argument("--no-split", action="store_true",
                    help="one workgroup per ladder even when the job has fewer ladders than compute units")
    ap.add_argument("--swap-every", type=int, default=-1, help="override the workload's PT interval")
    ap.add_argument("--cpu-sweeps", type=int, default=900)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--batched-sweeps", type=int, default=250)
    ap.add_argument("--batched-steps", type=int, default=4)
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--serving-jobs", type=int, default=64)
    ap.add_argument("--serving-quantum", type=int, default=200)
    ap.add_argument("--serving-scale", type=float, default=1.0,
                    help="multiply every job's sweep count (1.0 = the lognormal trace as drawn)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="before timing, run one elementwise kernel that reads and writes this many MiB "
                         "(reference kernel for scaling FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: each realization is an independent Markov chain and this "
              "build measures one GPU's share; run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1311_5582_amd import binding as B
    from paper_1311_5582_amd import inputs

    cfg = dict(inputs.CONFIGS[args.workload])
    L, R, n_T = cfg["L"], cfg["R"], cfg["n_T"]
    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    J = inputs.couplings(L, R, cfg["seed"])
    betas = inputs.geometric_betas(n_T, cfg["t_min"], cfg["t_max"])
    sim = B.Sim(L, J, betas, cfg["seed"], layout=args.layout, block_threads=args.block_threads, stream=stream,
                split=not args.no_split, rng=args.rng)
    launch = sim.info()
    S, se = args.sweeps_per_step, (cfg["swap_every"] if args.swap_every < 0 else args.swap_every)

    def step(events=None):
        if events is not None:
            events[0].record(stream)
        sim.sweep(S, se)
        if events is not None:
            events[1].record(stream)
        return sim.observables()

    if args.copy_probe_mib > 0:
        n = args.copy_probe_mib * (1 << 20)
        src = torch.ones(n, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        # an elementwise kernel (a same-dtype copy_ may go to a DMA engine):
        # reads n bytes, writes n bytes
        torch.bitwise_not(src, out=dst)
        torch.cuda.synchronize()
        del src, dst
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(evs[k])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kernel_ms = [a.elapsed_time(b) for a, b in evs]

    flips_per_step = S * L ** 3 * n_T * R * 2
    total_flips = flips_per_step * args.steps
    ps_per_flip = wall / total_flips * 1e12
    avg_launch_s = float(np.mean(kernel_ms)) / 1e3
    ops_per_flip = ALG_OPS_PER_FLIP if args.rng == "words" else ALG_OPS_PER_FLIP_PLANES
    achieved = ops_per_flip * flips_per_step / avg_launch_s / 1e12
    peak = PEAK_OPS_PER_S / 1e12
    out = {
        "metric": METRIC,
        "value": round(ps_per_flip, 4),
        "unit": "ps/flip",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 4),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": args.workload, "L": L, "spins": L ** 3, "realizations": R, "copies": 2,
                   "temperatures": n_T, "T_range": [cfg["t_min"], cfg["t_max"]], "sweeps_per_step": S,
                   "swap_every": se, "layout": args.layout, "rng": args.rng, "measurement_per_step": True,
                   "block_threads": launch["block_threads"], "workgroups_per_ladder": launch["split_parts"],
                   "kernel_ps_per_flip": round(avg_launch_s / flips_per_step * 1e12, 4),
                   "paper_ps_per_flip_gtx580": 33.5},
        "roofline": {"bound": "alu", "achieved": round(achieved, 3), "peak": round(peak, 3), "unit": "TOP/s",
                     "frac": round(achieved / peak, 4), "traffic": measured_traffic(args.workload, args.layout, args.rng),
                     "ops_per_flip": ops_per_flip, "kernel_sha1": kernel_source_hash(),
                     "kernel": "sweep_kernel<%s, %d>" % (args.layout.upper(), launch["split_parts"])},
    }
    sim.close()
    if not args.no_other_stream and args.layout == "camsc":
        other = "planes" if args.rng == "words" else "words"
        out["other_stream"] = bench_other_stream(B, torch, L, J, betas, cfg["seed"], args.layout, args.block_threads,
                                                 not args.no_split, other, S, se, 3)
    if args.layout_study:
        out["layout_study_kernel_ps_per_flip"] = bench_layout_study(B, torch, inputs, 200, 3)
    if not args.no_batched:
        out["batched"] = bench_batched(B, inputs, torch, args.batched_sweeps, args.batched_steps)
    if not args.no_serving:
        out["serving"] = bench_serving(B, inputs, args.serving_jobs, 20.0, args.serving_quantum, args.serving_scale)
        # the same trace shape at 0.8 x the measured service capacity (jobs/s)
        cap = out["serving"]["jobs"] / max(out["serving"]["wall_s"], 1e-9)
        out["serving_at_0.8_capacity"] = bench_serving(B, inputs, args.serving_jobs, 0.8 * cap,
                                                      args.serving_quantum, args.serving_scale)
        # the first trace through a plain queue: one job on the GPU at a time
        out["serving_queue_only"] = bench_serving(B, inputs, args.serving_jobs, 20.0, args.serving_quantum,
                                                  args.serving_scale, max_active=1)
    if not args.no_cpu_baseline:
        threads = max(1, min(os.cpu_count() or 1, 16))
        out["cpu_baseline"] = cpu_baseline(L, n_T, cfg["t_min"], cfg["t_max"], cfg["seed"], args.cpu_sweeps, threads)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
