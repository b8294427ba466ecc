#!/usr/bin/env python
"""Throughput of the deviational phonon Monte Carlo trace on one MI355X.

A step is one pass of the whole hot path over one batch of synthetic particles: zero the
tally buffer, trace the batch (emission inside the persistent kernel: source, position,
frequency, direction, sign, free flights, boundaries, relaxations, detector scores) and
finalize the tallies on the host (kappa and its standard error).  The mode tables are built
once before the timed region (inputs resident in HBM).  Each step uses its own seed.

Default workload: the in-plane thin film (100 nm, diffuse walls, synthetic silicon-like
dispersion of 1400 mode rows at 300 K, 1e6 particles, N_scat^max = 10), FP32 trajectories
with FP64 tables and sums.  One JSON line on stdout.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "particle flights/sec (and κ_eff at fixed 1σ error) per MI355X vs CPU oracle"

# Peak of the bound that limits this path: plain vector ALU issue on 256 CUs x 4 SIMDs x 16 lanes
# at 2.4 GHz (one full-rate 32-bit or 64-bit VALU lane operation per lane per clock).
PEAK_LANE_OPS = 256 * 4 * 16 * 2.4e9

# Algorithmic VALU work of the method's steps, in full-rate lane-operation equivalents
# (quarter-rate instructions -- 32x32->64 integer products, reciprocal, square root, log,
# sin/cos -- count 4).  Derived from the operations the method prescribes, not from the
# compiled code; the derivation is in the design notes.
OPS = {
    "philox_block": 100,      # 10 rounds x (2 products x 4 + 2 three-way XORs)
    "flight_base": 34,        # choice of event, position/time update, one track-length score, particle scores
    "face_axis": 9,           # distance to the face ahead on one bounded axis
    "pore": 24,               # ray-cylinder test
    "tally_comp": 4,          # one scored component (value, conversion, LDS address)
    "free_flight": 7,         # -tau log(1 - u)
    "iso_dir": 21,            # isotropic direction
    "cos_dir": 36,            # cosine-weighted direction about a normal
    "search_step": 5,         # one step of the 64-bit threshold search
    "emit_misc": 20,          # source pick, position, sign, start time
}


def algorithmic_lane_ops(counts: dict, info: dict, geom: dict, ncomp: int, transient: bool) -> float:
    """Lane-operations the method requires for the events of one launch (see OPS)."""
    M = int(info["n_modes"])
    S = int(info["n_sources"])
    steps_M = max(1, math.ceil(math.log2(M + 1)))
    steps_S = max(1, math.ceil(math.log2(S + 1)))
    n_axes = sum(0 if u else 1 for u in geom["unbounded"])
    per_flight = (OPS["flight_base"] + n_axes * OPS["face_axis"] + len(geom["cylinders"]) * OPS["pore"]
                  + ncomp * OPS["tally_comp"])
    relax_draws = counts["relaxations"] - counts["nscat_end"]
    diffuse = counts["diffuse"]
    emit = counts["particles"] * (4 * OPS["philox_block"] + (steps_S + steps_M) * OPS["search_step"]
                                  + OPS["cos_dir"] + OPS["free_flight"] + OPS["emit_misc"])
    return (emit + counts["flights"] * per_flight
            + relax_draws * (2 * OPS["philox_block"] + steps_M * OPS["search_step"] + OPS["iso_dir"]
                             + OPS["free_flight"])
            + diffuse * (OPS["philox_block"] + OPS["cos_dir"])
            + counts["rejections"] * 2 * OPS["philox_block"])


def profiled_traffic(kernel_tag: str):
    """HBM bytes per launch from the committed rocprofv3 FETCH_SIZE / WRITE_SIZE summary of this
    kernel and workload, or None when the kernel source changed since the counters were taken."""
    import hashlib
    src = os.path.join(ROOT, "paper_2104_03573_amd", "csrc")
    h = hashlib.sha256()
    for f in ("mcbte_kernels.hip", "mcbte_dev.h"):
        with open(os.path.join(src, f), "rb") as fh:
            h.update(fh.read())
    path = os.path.join(ROOT, "profiles", f"{kernel_tag}.txt")
    if not os.path.exists(path):
        return None
    kv = dict(l.strip().split("=", 1) for l in open(path) if "=" in l and not l.startswith("#"))
    if kv.get("kernel_source_sha256_16") != h.hexdigest()[:16]:
        return None
    return float(kv["hbm_bytes_per_launch"])


def workload(name: str, scale: float = 1.0):
    import workloads as W
    if name == "film":
        return W.film(N=int(1_000_000 * scale)), "film_d100nm_T300K_1400modes_N1e6_nscat10"
    if name == "gray_slab":
        return W.gray_slab(N=int(100_000 * scale)), "gray_slab_L100nm_Kn1_N1e5_50bins"
    if name == "porous_cell":
        return W.porous_cell(N=int(10_000_000 * scale)), "porous_cell_500nm_phi0.25_N1e7"
    if name == "transient":
        return W.transient_bump(N=int(10_000_000 * scale)), "transient_bump_1um_200times_100bins_N1e7"
    if name == "sweep":
        return W.film_sweep(scale=scale), "film_sweep_16d_x_4T_64instances_N7.2e7"
    raise SystemExit(f"unknown workload {name}")


def cpu_baseline(w: dict, seconds: float, threads: int) -> dict:
    """The oracle as it stands, on the host cores: whole batches of the same workload (a new seed
    per batch, like the GPU steps) until about `seconds` of CPU time have passed; a batch larger
    than that is cut to a prefix of its particles."""
    import oracle
    tb = oracle.Tables(w)
    N = w["problem"]["N"]
    t0 = time.perf_counter()
    probe = oracle.trace(w, n=min(N, 2000), threads=threads, tables=tb)
    rate = probe["counts"][0] / max(time.perf_counter() - t0, 1e-6)
    n = int(min(N, max(2000, rate * seconds)))
    flights = 0
    batches = 0
    t0 = time.perf_counter()
    while True:
        wb = dict(w, seed=int(w["seed"]) + batches)
        res = oracle.trace(wb, n=n, threads=threads, tables=tb)
        flights += int(res["counts"][1])
        batches += 1
        dt = time.perf_counter() - t0
        if dt >= seconds or batches >= 10000:
            break
    what = f"{batches} batches of particles 0..{n - 1}" if n < N else f"{batches} full batches of {N} particles"
    return {"value": flights / dt, "unit": "flights/s", "cores": threads, "kind": "oracle",
            "sample": f"{what} of the same workload, new seed per batch ({flights} flights in {dt:.1f} s, "
                      f"{threads} threads over contiguous particle ranges)"}


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="film")
    ap.add_argument("--scale", type=float, default=1.0)
    ap.add_argument("--precision", type=int, default=32, choices=(32, 64))
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--refill", type=int, default=0)
    ap.add_argument("--grid", type=int, default=0)
    ap.add_argument("--streams", type=int, default=1)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB three times (reference for the "
                         "FETCH_SIZE / WRITE_SIZE counters) and exit")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the tracer runs on a single MI355X here "
              "(multi-GPU sharding is a design note, not a built path); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    if args.copy_calibration:
        nb = args.copy_calibration * 1024 * 1024
        src = torch.ones(nb // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_per_launch": nb, "launches": 3}), flush=True)
        return

    import paper_2104_03573_amd as M

    w, wname = workload(args.workload, args.scale)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if isinstance(w, list):
        return bench_batched(args, w, wname, M, torch)
    t0 = time.perf_counter()
    tabs = M.Tables(w, 0)
    t_tables = time.perf_counter() - t0
    N = w["problem"]["N"]
    ncomp = bin(w["detectors"]["mask"]).count("1")
    S = max(1, args.streams)
    streams = [torch.cuda.current_stream()] + [torch.cuda.Stream() for _ in range(S - 1)]
    tallies = [tabs.new_tally() for _ in range(S)]
    base_seed = int(w["seed"])

    def launch(slot: int, seed: int, ev=None):
        tl = tallies[slot]
        tl.zero_()
        run = M.make_run(seed, args.precision, block=args.block, refill=args.refill, grid=args.grid)
        if ev is not None:
            ev[0].record()
        M.trace(tabs, run, 0, N, None, tl)
        if ev is not None:
            ev[1].record()

    def finish(slot: int):
        return M.tally(tabs, tallies[slot], with_arrays=False)

    def run_steps(n_steps: int, n_streams: int, seed0: int, timed: bool):
        """n_steps batches; batch i on stream i % n_streams; a stream's previous batch is finalized
        before the stream takes its next one."""
        events = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                  for _ in range(n_steps)] if timed else [None] * n_steps
        pending = [False] * n_streams
        results = []
        for i in range(n_steps):
            slot = i % n_streams
            with torch.cuda.stream(streams[slot]):
                if pending[slot]:
                    results.append(finish(slot))
                launch(slot, seed0 + i, events[i])
                pending[slot] = True
        for k in range(n_steps, n_steps + n_streams):
            slot = k % n_streams
            if pending[slot]:
                with torch.cuda.stream(streams[slot]):
                    results.append(finish(slot))
                pending[slot] = False
        return results, events

    # warmup, then the timed steps; the trace kernel of every step is bracketed by HIP events on
    # its stream (the roofline uses their durations; with several streams the kernels overlap)
    run_steps(max(args.warmup, 1), S, base_seed + 100000, False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    results, events = run_steps(args.steps, S, base_seed, True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kernel_ms = [a.elapsed_time(b) for a, b in events]
    ops = sum(algorithmic_lane_ops(r["counts"], tabs.info, w["geometry"], ncomp, w["problem"]["transient"])
              for r in results)
    achieved = ops / (sum(kernel_ms) / 1e3)
    flights = sum(r["counts"]["flights"] for r in results)
    last = results[-1]
    out = {
        "metric": METRIC,
        "value": flights / wall,
        "unit": "flights/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision == 32 else "f64",
        "data": "synthetic",
        "config": {"workload": wname, "particles_per_step": N, "modes": int(tabs.info["n_modes"]),
                   "precision": args.precision, "tallies": "f64", "streams": S,
                   "parallelism": "single GPU" + (", batches overlapped on %d streams" % S if S > 1 else "")},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_LANE_OPS / 1e12,
                     "unit": "T lane-op/s", "frac": achieved / PEAK_LANE_OPS,
                     "traffic": (profiled_traffic("k_trace_solo_film_fp32")
                                 if args.workload == "film" and args.precision == 32 and S == 1 else None),
                     "kernel": "k_trace_solo", "kernel_ms": sum(kernel_ms) / len(kernel_ms),
                     "lane_ops_per_launch": ops / args.steps},
        "kernel_ms_per_step": kernel_ms,
        "flights_per_step": flights / args.steps,
        "particles_per_s": N * args.steps / wall,
        "relaxations_per_s": sum(r["counts"]["relaxations"] for r in results) / wall,
        "table_build_s": t_tables,
    }
    if not w["problem"]["transient"] and last.get("kappa"):
        sig = last["kappa_sigma"] / abs(last["kappa"])
        out["kappa_eff"] = last["kappa"]
        out["kappa_sigma"] = last["kappa_sigma"]
        # time to a 0.5% standard error at this rate: t_step (sigma_rel / 0.005)^2
        out["time_to_sigma_0p5pct_s"] = (wall / args.steps) * (sig / 0.005) ** 2
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds, min(16, os.cpu_count() or 1))
    print(json.dumps(out), flush=True)


def bench_batched(args, ws, wname, M, torch):
    """The batched form: every step traces all instances of the sweep in one persistent launch."""
    t0 = time.perf_counter()
    tabs = [M.Tables(w, 0) for w in ws]
    t_tables = time.perf_counter() - t0
    tallies = [t.new_tally() for t in tabs]
    queue = torch.zeros(M.batch_queue_bytes(len(ws)), dtype=torch.uint8, device="cuda")
    ns = [w["problem"]["N"] for w in ws]
    ids = [w["instance"] for w in ws]
    base_seed = int(ws[0]["seed"])

    def step(seed, ev=None):
        for tl in tallies:
            tl.zero_()
        run = M.make_run(seed, args.precision, block=args.block, refill=args.refill, grid=args.grid)
        if ev is not None:
            ev[0].record()
        M.trace_batch(tabs, ns, ids, tallies, run, queue)
        if ev is not None:
            ev[1].record()
        return [M.tally(t, tl, with_arrays=False) for t, tl in zip(tabs, tallies)]

    for i in range(max(args.warmup, 1)):
        step(base_seed + 100000 + i)
    torch.cuda.synchronize()
    events = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    t0 = time.perf_counter()
    results = [step(base_seed + i, events[i]) for i in range(args.steps)]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kernel_ms = [a.elapsed_time(b) for a, b in events]
    flights = sum(r["counts"]["flights"] for rs in results for r in rs)
    ops = sum(algorithmic_lane_ops(r["counts"], t.info, w["geometry"], bin(w["detectors"]["mask"]).count("1"), False)
              for rs in results for r, t, w in zip(rs, tabs, ws))
    achieved = ops / (sum(kernel_ms) / 1e3)
    last = results[-1]
    worst = max(r["kappa_sigma"] / abs(r["kappa"]) for r in last)
    out = {
        "metric": METRIC, "value": flights / wall, "unit": "flights/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": wall / args.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32" if args.precision == 32 else "f64",
        "data": "synthetic",
        "config": {"workload": wname, "instances": len(ws), "particles_per_step": sum(ns),
                   "precision": args.precision, "tallies": "f64", "parallelism": "single GPU, one batched launch"},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_LANE_OPS / 1e12,
                     "unit": "T lane-op/s", "frac": achieved / PEAK_LANE_OPS, "traffic": None,
                     "kernel": "k_trace_batch", "kernel_ms": sum(kernel_ms) / len(kernel_ms)},
        "kernel_ms_per_step": kernel_ms,
        "kappa_eff_per_instance": [r["kappa"] for r in last],
        "worst_kappa_sigma_rel": worst,
        "table_build_s": t_tables,
    }
    if not args.no_cpu_baseline:
        # the oracle on the most expensive instance alone (particles of every instance cost alike
        # per flight); rate in flights/s
        out["cpu_baseline"] = cpu_baseline(ws[-1], args.cpu_seconds, min(16, os.cpu_count() or 1))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
