"""Benchmark: picoseconds per spin-flip attempt on one MI355X.

Workload (default): 3D +-J EA model, L = 16 (4096 spins), 64 disorder
realizations x 2 copies, 32 temperatures geometric in T in [0.4, 2.0],
parallel tempering after every sweep, CAMSC layout.  One step = one sweep
launch of --sweeps-per-step sweeps plus one measurement (energies and
overlaps); the default 10 steps x 1000 sweeps is the whole 10^4-sweep job.
ps/flip follows Eq. tsf of the paper: wall time / (sweeps x spins x
temperatures x samples), samples = realizations x 2 copies.

Further legs on the same line: the large job (L=24, 256 realizations, 48
temperatures, PT every 10 sweeps) with both draw streams, MC and PT fused in
one launch vs one launch per swap interval, the five uneven jobs batched vs
plain, and the 64-job serving trace through the server vs the plain
single-job path.  The roofline objects price the sweep kernel
against the vector ALU rate of the chip; the cpu_baseline object times the
CPU oracle on a bounded sample of the same workload, on all host cores and
on one.
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

# int32 operations per spin-flip attempt that the method itself needs: a
# quarter of a Philox4x32-10 block (10 rounds x (2 v_mad_u64_u32 + 2
# three-input xors) / 4 = 10), the table column, address, compare and insert
# (4), and the share of the bit-parallel bond energies (2).
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
# MI355X vector ALU peak: 256 CUs x 4 SIMDs x 32 lane-operations per cycle x
# 2.4 GHz = 78.6 T lane-operations/s (the rate behind the published 157.3
# TFLOP/s fp32 vector figure, an FMA being 2 flops).  A wave64 instruction
# occupies a SIMD for 4 cycles at the basic 16 lanes/cycle, but the probe
# (--valu-rate) measures v_bitop3_b32 at 49 T/s with the clock at 1.7 GHz,
# about 28 lanes/cycle, so 16 lanes/cycle is no ceiling; v_xad_u32 and
# two-operand instructions measure ~16 lanes/cycle, v_mad_u64_u32 ~10.5 and
# v_mul_hi_u32 ~8.
PEAK_OPS_PER_S = 256 * 4 * 32 * 2.4e9
KERNEL_SRC = os.path.join(ROOT, "paper_1311_5582_amd", "csrc", "ea_kernels.hip")
PROFILES = os.path.join(ROOT, "profiles")


def progress(msg):
    """One line per finished leg on stderr (stdout carries only the JSON line)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_name(layout, info):
    """The sweep kernel a launch runs: ladders split by lattice halves run
    slab_kernel, every other launch sweep_kernel<layout, workgroups per ladder>."""
    if info.get("split_by_halves"):
        return "slab_kernel"
    return "sweep_kernel<%s, %d>" % (layout.upper(), info["split_parts"])


def kernel_source_hash():
    import hashlib
    return hashlib.sha1(open(KERNEL_SRC, "rb").read()).hexdigest()[:12]


def measured_traffic(workload, layout, rng="words", kernel="sweep_kernel"):
    """HBM bytes per sweep launch from the committed rocprofv3 FETCH_SIZE /
    WRITE_SIZE summary, only if it was taken on the current kernel source."""
    import re
    suffix = "" if rng == "words" else "_" + rng
    path = os.path.join(PROFILES, f"{kernel}_{workload}_{layout}{suffix}.md")
    if not os.path.exists(path):
        return None
    m = re.search(r"traffic_bytes_per_launch:\s*(\d+)\s+kernel_sha1:\s*([0-9a-f]+)", open(path).read())
    if not m or m.group(2) != kernel_source_hash():
        return None
    return int(m.group(1))


def valu_rates(grid=1024, iters=512):
    """Issue rates measured by the probe library: lane-operations per second of
    v_bitop3_b32, v_xor_b32 + v_min_u32, v_xad_u32, v_mad_u64_u32 (each paired
    with a v_mov_b32, counted separately), v_mul_hi_u32 (each with a v_xor_b32),
    and Philox4x32-10 blocks per second; with the shader clock each ran at."""
    import ctypes
    path = os.path.join(ROOT, "paper_1311_5582_amd", "libea_valu_probe.so")
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built; run __graft_entry__.build()")
    lib = ctypes.CDLL(path)
    lib.ea_probe_valu_rates.restype = ctypes.c_int
    rates, ms, ghz = (ctypes.c_double * 6)(), (ctypes.c_double * 6)(), (ctypes.c_double * 6)()
    rc = lib.ea_probe_valu_rates(grid, iters, rates, ms, ghz)
    if rc != 0:
        raise RuntimeError(f"VALU probe failed with HIP error {rc}")
    names = ["v_bitop3_b32", "v_xor_b32+v_min_u32", "v_xad_u32", "v_mad_u64_u32(+v_mov_b32)",
             "v_mul_hi_u32(+v_xor_b32)", "philox4x32_10_blocks"]
    return {"grid": grid, "threads_per_workgroup": 1024, "iters": iters,
            "rates_T_per_s": {n: round(rates[k] / 1e12, 3) for k, n in enumerate(names)},
            "kernel_ms": {n: round(ms[k], 4) for k, n in enumerate(names)},
            "shader_clock_GHz": {n: round(ghz[k], 3) for k, n in enumerate(names)},
            "peak_T_per_s": round(PEAK_OPS_PER_S / 1e12, 3)}


def cpu_model():
    """The host CPU's model name (from /proc/cpuinfo) and its logical CPU count."""
    name = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    name = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return name, os.cpu_count() or 1


def usable_cores():
    try:
        n = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        n = os.cpu_count() or 1
    return max(1, min(n, 16))


def time_oracle(L, n_T, t_min, t_max, seed, sweeps, threads):
    """Wall time of the oracle on `threads` realizations, one per thread."""
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
    return dt, sweeps * L ** 3 * n_T * 2 * threads


def cpu_baseline(L, n_T, t_min, t_max, seed, sweeps, threads, single_sweeps):
    """Time the oracle on all usable host cores (one realization per thread,
    `sweeps` each) and on one core (one realization, `single_sweeps`)."""
    model, logical = cpu_model()
    dt, flips = time_oracle(L, n_T, t_min, t_max, seed, sweeps, threads)
    dt1, flips1 = time_oracle(L, n_T, t_min, t_max, seed, single_sweeps, 1)
    return {"value": dt / flips * 1e12, "unit": "ps/flip", "cores": threads, "kind": "oracle",
            "sample": f"{threads} realizations x 2 copies x {n_T} temps, L={L}, {sweeps} sweeps, "
                      f"PT every sweep, one realization per thread ({flips:.3g} flip attempts, {dt:.1f} s wall)",
            "cpu_model": model, "host_logical_cpus": logical,
            "single_core": {"value": dt1 / flips1 * 1e12, "unit": "ps/flip", "cores": 1,
                            "sample": f"1 realization x 2 copies x {n_T} temps, L={L}, {single_sweeps} sweeps, "
                                      f"PT every sweep ({flips1:.3g} flip attempts, {dt1:.1f} s wall)"}}


def bench_other_stream(B, torch, L, J, betas, seed, layout, block_threads, split, rng, sweeps, swap_every, steps,
                       site_order="natural"):
    """The same workload and launch with the other flip-draw stream (kernel time
    from HIP events on the launch stream, wall time around the steps)."""
    stream = torch.cuda.Stream()
    sim = B.Sim(L, J, betas, seed, layout=layout, block_threads=block_threads, stream=stream, split=split, rng=rng,
                site_order=site_order)
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
    with split ladders (by lattice halves, and by slot groups) and with
    bit-plane draws."""
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
                                     ("camsc_split_slot_groups", "camsc", "slots", "words"),
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


def bench_large(B, inputs, torch, sweeps, steps, rng="words", site_order="natural"):
    """The large production job (L=24, 256 realizations x 2 copies, 48
    temperatures, PT every 10 sweeps): `steps` launches of `sweeps` sweeps,
    each followed by a measurement of energies and overlaps; kernel time from
    HIP events on the launch stream."""
    cfg = inputs.CONFIGS["L24_R256"]
    L, R, n_T = cfg["L"], cfg["R"], cfg["n_T"]
    J = inputs.couplings(L, R, cfg["seed"])
    betas = inputs.geometric_betas(n_T, cfg["t_min"], cfg["t_max"])
    stream = torch.cuda.Stream()
    sim = B.Sim(L, J, betas, cfg["seed"], stream=stream, rng=rng, site_order=site_order)
    info = sim.info()
    sim.sweep(sweeps, cfg["swap_every"])
    sim.observables()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    t0 = time.perf_counter()
    for a, b in evs:
        a.record(stream)
        sim.sweep(sweeps, cfg["swap_every"])
        b.record(stream)
        sim.observables()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    sim.close()
    flips = sweeps * L ** 3 * n_T * R * 2
    kern = float(np.mean([a.elapsed_time(b) for a, b in evs])) / 1e3
    ops = ALG_OPS_PER_FLIP if rng == "words" else ALG_OPS_PER_FLIP_PLANES
    achieved = ops * flips / kern / 1e12
    peak = PEAK_OPS_PER_S / 1e12
    return {"workload": "L24_R256", "L": L, "realizations": R, "copies": 2, "temperatures": n_T,
            "T_range": [cfg["t_min"], cfg["t_max"]], "swap_every": cfg["swap_every"], "rng": rng, "site_order": site_order,
            "sweeps_per_step": sweeps, "steps": steps, "measurement_per_step": True,
            "block_threads": info["block_threads"], "workgroups_per_ladder": info["split_parts"],
            "ps_per_flip": round(wall / (flips * steps) * 1e12, 4), "ms_per_step": round(wall / steps * 1e3, 4),
            "kernel_ps_per_flip": round(kern / flips * 1e12, 4),
            "roofline": {"bound": "alu", "achieved": round(achieved, 3), "peak": round(peak, 3), "unit": "TOP/s",
                         "frac": round(achieved / peak, 4),
                         "traffic": measured_traffic("L24_R256", "camsc", rng, kernel_name("camsc", info).split("<")[0]),
                         "ops_per_flip": ops, "kernel_sha1": kernel_source_hash(),
                         "kernel": kernel_name("camsc", info)}}


def bench_fused_vs_separated(B, inputs, torch, sweeps):
    """MC and PT fused in one persistent launch (this library) against one
    launch per swap interval, the lower bound of the paper's "separated"
    scheme (Sec. 4.1, Fig. korg), which adds a second launch for the swap
    step: the per-interval launches are graph-captured plan steps of
    swap_every sweeps, each loading its ladders into LDS, running the sweeps
    and the fused swap step, and writing them back.  Both runs make the same
    chain, and their energies and overlaps are compared."""
    cfg = inputs.CONFIGS["L16_R64"]
    L, R, n_T = cfg["L"], cfg["R"], cfg["n_T"]
    J = inputs.couplings(L, R, cfg["seed"])
    betas = inputs.geometric_betas(n_T, cfg["t_min"], cfg["t_max"])
    flips = sweeps * L ** 3 * n_T * R * 2
    out = {"workload": "L16_R64", "sweeps": sweeps}
    for se in (1, 10):
        fused = B.Sim(L, J, betas, cfg["seed"])
        fused.sweep(se, se)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fused.sweep(sweeps, se)
        torch.cuda.synchronize()
        t_fused = time.perf_counter() - t0
        sep = B.Sim(L, J, betas, cfg["seed"])
        plan = B.Plan([sep], se, se, autotune=False)
        plan.run(1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan.run(sweeps // se)
        torch.cuda.synchronize()
        t_sep = time.perf_counter() - t0
        parts = plan.info()["split_parts"]
        plan.close()
        same = all(np.array_equal(a, b) for a, b in zip(fused.observables(), sep.observables()))
        fused.close()
        sep.close()
        out[f"swap_every_{se}"] = {"fused_ps_per_flip": round(t_fused / flips * 1e12, 4),
                                   "launch_per_interval_ps_per_flip": round(t_sep / flips * 1e12, 4),
                                   "ratio": round(t_sep / t_fused, 3), "workgroups_per_ladder": parts,
                                   "same_chain": bool(same)}
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


def bench_serving(B, inputs, n_jobs, rate, quantum, sweep_scale=1.0, policy="ratio", fill=0, pack=True):
    """Poisson job trace through the continuous-batching server."""
    from paper_1311_5582_amd import serve
    trace = inputs.serving_trace(n_jobs=n_jobs, rate_per_s=rate)
    for j in trace:
        j["sweeps"] = max(1, int(j["sweeps"] * sweep_scale))
    srv = B.Server(quantum_sweeps=quantum, policy=policy, fill_ladders=fill, pack_rounds=pack)
    recs, wall = serve.run_trace(trace, srv)
    st = srv.stats()
    srv.close()
    summ = serve.latency_summary(recs)
    busy = summ["done_last_s"] - trace[0]["arrival_s"]
    return {"jobs": n_jobs, "rate_per_s": round(rate, 3), "quantum_sweeps": quantum, "sweep_scale": sweep_scale,
            "policy": policy, "fill_ladders": fill, "pack_rounds": pack, "p50_latency_s": round(summ["p50_s"], 4), "p99_latency_s": round(summ["p99_s"], 4),
            "mean_latency_s": round(summ["mean_s"], 4), "wall_s": round(wall, 3),
            "aggregate_ps_per_flip": round(busy / summ["flips"] * 1e12, 4), "steps": st["steps"],
            "plans_built": st["plans_built"], "launches_replayed": st["launches_replayed"], "worst": summ["worst"]}


def bench_queue_plain(B, inputs, torch, n_jobs, rate, sweep_scale=1.0):
    """The same trace through the plain single-job path: jobs in arrival order,
    one at a time, each created and run alone with ea_sweep (split ladders
    where the library picks them), measured and released."""
    from paper_1311_5582_amd import serve
    trace = inputs.serving_trace(n_jobs=n_jobs, rate_per_s=rate)
    for j in trace:
        j["sweeps"] = max(1, int(j["sweeps"] * sweep_scale))
    prepared = [(inputs.couplings(j["L"], j["R"], j["seed"]), inputs.geometric_betas(j["n_T"], j["t_min"], j["t_max"]))
                for j in trace]
    recs = {}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k, (j, (J, betas)) in enumerate(zip(trace, prepared)):
        wait = j["arrival_s"] - (time.perf_counter() - t0)
        if wait > 0:
            time.sleep(wait)
        sim = B.Sim(j["L"], J, betas, j["seed"])
        sim.sweep(j["sweeps"], j["swap_every"])
        sim.observables()
        sim.close()
        now = time.perf_counter() - t0
        recs[k] = dict(job=j, status=B.JOB_DONE, done_s=now, latency_s=now - j["arrival_s"])
    wall = time.perf_counter() - t0
    summ = serve.latency_summary(recs)
    busy = summ["done_last_s"] - trace[0]["arrival_s"]
    return {"jobs": n_jobs, "rate_per_s": round(rate, 3), "sweep_scale": sweep_scale, "path": "ea_sweep per job, FIFO",
            "p50_latency_s": round(summ["p50_s"], 4), "p99_latency_s": round(summ["p99_s"], 4),
            "mean_latency_s": round(summ["mean_s"], 4), "wall_s": round(wall, 3),
            "aggregate_ps_per_flip": round(busy / summ["flips"] * 1e12, 4), "worst": summ["worst"]}


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
    ap.add_argument("--site-order", default="natural", choices=["natural", "by_class"],
                    help="order of the spin words in LDS: natural (unified) or by checkerboard class (separated)")
    ap.add_argument("--split-slots", action="store_true",
                    help="split ladders by slot groups only (not by lattice halves)")
    ap.add_argument("--no-split", action="store_true",
                    help="one workgroup per ladder even when the job has fewer ladders than compute units")
    ap.add_argument("--swap-every", type=int, default=-1, help="override the workload's PT interval")
    ap.add_argument("--cpu-sweeps", type=int, default=900)
    ap.add_argument("--cpu-single-sweeps", type=int, default=700,
                    help="sweeps of the one-core oracle timing (one realization)")
    ap.add_argument("--no-large", action="store_true", help="skip the L=24, 256-realization job")
    ap.add_argument("--large-sweeps", type=int, default=200)
    ap.add_argument("--large-steps", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fused-vs-separated", action="store_true",
                    help="skip the MC/PT fused vs one-launch-per-swap-interval comparison")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--batched-sweeps", type=int, default=250)
    ap.add_argument("--batched-steps", type=int, default=4)
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--serving-jobs", type=int, default=64)
    ap.add_argument("--serving-fill-sweep", default="",
                    help="comma-separated ladder fill targets: only run the served trace at 20 jobs/s and at "
                         "--serving-rate2 for each, with --serving-policy, and print their lines")
    ap.add_argument("--serving-policy", default="ratio", choices=["ratio", "shortest", "fifo"])
    ap.add_argument("--serving-rate2", type=float, default=1.526)
    ap.add_argument("--serving-no-pack", action="store_true",
                    help="fill sweep: every unit of a step equally long (no packing of the last round)")
    ap.add_argument("--serving-policies", action="store_true",
                    help="also run the trace with every waiting job admitted at once (first fit, arrival order), "
                         "shortest remaining work first, and without packing of a step's last round")
    ap.add_argument("--serving-quantum", type=int, default=400)
    ap.add_argument("--serving-scale", type=float, default=1.0,
                    help="multiply every job's sweep count (1.0 = the lognormal trace as drawn)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="before timing, run one elementwise kernel that reads and writes this many MiB "
                         "(reference kernel for scaling FETCH_SIZE / WRITE_SIZE counters)")
    ap.add_argument("--valu-rate", action="store_true",
                    help="only measure the integer issue rates behind the roofline and print them")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: each realization is an independent Markov chain, so more GPUs "
              "would each run their own share of the realizations; it measures one GPU's share: run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    if args.valu_rate:
        print(json.dumps({"valu_rate": valu_rates()}), flush=True)
        return
    if args.serving_fill_sweep:
        from paper_1311_5582_amd import binding as B
        from paper_1311_5582_amd import inputs
        res = {}
        for fill in [int(x) for x in args.serving_fill_sweep.split(",")]:
            for rate in (20.0, args.serving_rate2):
                r = bench_serving(B, inputs, args.serving_jobs, rate, args.serving_quantum, args.serving_scale,
                                  policy=args.serving_policy, fill=fill, pack=not args.serving_no_pack)
                res[f"fill{fill}_rate{rate}"] = r
                progress(f"fill {fill} rate {rate}: p50 {r['p50_latency_s']} p99 {r['p99_latency_s']} "
                         f"{r['aggregate_ps_per_flip']} ps/flip")
        print(json.dumps({"serving_fill_sweep": res}), flush=True)
        return

    import torch
    from paper_1311_5582_amd import binding as B
    from paper_1311_5582_amd import inputs

    cfg = dict(inputs.CONFIGS[args.workload])
    L, R, n_T = cfg["L"], cfg["R"], cfg["n_T"]
    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    J = inputs.couplings(L, R, cfg["seed"])
    betas = inputs.geometric_betas(n_T, cfg["t_min"], cfg["t_max"])
    split = False if args.no_split else ("slots" if args.split_slots else True)
    sim = B.Sim(L, J, betas, cfg["seed"], layout=args.layout, block_threads=args.block_threads, stream=stream,
                split=split, rng=args.rng, site_order=args.site_order)
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
                   "swap_every": se, "layout": args.layout, "rng": args.rng, "site_order": args.site_order,
                   "measurement_per_step": True,
                   "block_threads": launch["block_threads"], "workgroups_per_ladder": launch["split_parts"],
                   "split_by_halves": launch["split_by_halves"],
                   "kernel_ps_per_flip": round(avg_launch_s / flips_per_step * 1e12, 4),
                   "paper_ps_per_flip_gtx580": 33.5},
        "roofline": {"bound": "alu", "achieved": round(achieved, 3), "peak": round(peak, 3), "unit": "TOP/s",
                     "frac": round(achieved / peak, 4),
                     "traffic": measured_traffic(args.workload, args.layout, args.rng,
                                                 kernel_name(args.layout, launch).split("<")[0]),
                     "ops_per_flip": ops_per_flip, "kernel_sha1": kernel_source_hash(),
                     "kernel": kernel_name(args.layout, launch)},
    }
    sim.close()
    progress(f"{args.workload}: {ps_per_flip:.4f} ps/flip")
    if not args.no_other_stream and args.layout == "camsc":
        other = "planes" if args.rng == "words" else "words"
        out["other_stream"] = bench_other_stream(B, torch, L, J, betas, cfg["seed"], args.layout, args.block_threads,
                                                 split, other, S, se, 3, args.site_order)
    if "other_stream" in out:
        progress(f"other stream: {out['other_stream']['ps_per_flip']} ps/flip")
    if args.layout_study:
        out["layout_study_kernel_ps_per_flip"] = bench_layout_study(B, torch, inputs, 200, 3)
        progress("layout study done")
    if not args.no_large:
        out["large"] = bench_large(B, inputs, torch, args.large_sweeps, args.large_steps, site_order=args.site_order)
        out["large_planes"] = bench_large(B, inputs, torch, args.large_sweeps, args.large_steps, rng="planes",
                                          site_order=args.site_order)
        progress(f"L24_R256: {out['large']['ps_per_flip']} / planes {out['large_planes']['ps_per_flip']} ps/flip")
    if not args.no_fused_vs_separated:
        out["mc_pt_fused_vs_separated"] = r = bench_fused_vs_separated(B, inputs, torch, 2000)
        progress(f"fused vs one launch per swap interval: every sweep {r['swap_every_1']['ratio']}x, "
                 f"every 10 {r['swap_every_10']['ratio']}x")
    if not args.no_batched:
        out["batched"] = bench_batched(B, inputs, torch, args.batched_sweeps, args.batched_steps)
        progress(f"batched: {out['batched']['batched_ps_per_flip']} vs plain {out['batched']['plain_ps_per_flip']}")
    if not args.no_serving:
        def leg(name, result):
            out[name] = result
            progress(f"{name}: p50 {result['p50_latency_s']} s p99 {result['p99_latency_s']} s "
                     f"{result['aggregate_ps_per_flip']} ps/flip")

        leg("serving", bench_serving(B, inputs, args.serving_jobs, 20.0, args.serving_quantum, args.serving_scale))
        # the same trace through the plain single-job path, one job at a time
        leg("serving_queue_only", bench_queue_plain(B, inputs, torch, args.serving_jobs, 20.0, args.serving_scale))
        if args.serving_policies:
            # every waiting job admitted at once (processor sharing), and response-ratio admission
            leg("serving_fifo_all", bench_serving(B, inputs, args.serving_jobs, 20.0, args.serving_quantum,
                                                  args.serving_scale, policy="fifo"))
            leg("serving_shortest", bench_serving(B, inputs, args.serving_jobs, 20.0, args.serving_quantum,
                                                  args.serving_scale, policy="shortest"))
            leg("serving_unpacked", bench_serving(B, inputs, args.serving_jobs, 20.0, args.serving_quantum,
                                                  args.serving_scale, pack=False))
        # the same trace shape at 0.8 x the measured service capacity (jobs/s), served and plain
        cap = out["serving"]["jobs"] / max(out["serving"]["wall_s"], 1e-9)
        leg("serving_at_0.8_capacity", bench_serving(B, inputs, args.serving_jobs, 0.8 * cap, args.serving_quantum,
                                                     args.serving_scale))
        leg("serving_queue_only_at_0.8_capacity", bench_queue_plain(B, inputs, torch, args.serving_jobs, 0.8 * cap,
                                                                    args.serving_scale))
        if args.serving_policies:
            leg("serving_shortest_at_0.8_capacity", bench_serving(B, inputs, args.serving_jobs, 0.8 * cap,
                                                                  args.serving_quantum, args.serving_scale,
                                                                  policy="shortest"))
            leg("serving_unpacked_at_0.8_capacity", bench_serving(B, inputs, args.serving_jobs, 0.8 * cap,
                                                                  args.serving_quantum, args.serving_scale,
                                                                  pack=False))
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(L, n_T, cfg["t_min"], cfg["t_max"], cfg["seed"], args.cpu_sweeps,
                                           usable_cores(), args.cpu_single_sweeps)
        progress("cpu baseline done")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
