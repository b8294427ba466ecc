#!/usr/bin/env python
"""Throughput of the deviational phonon Monte Carlo trace on one MI355X.

A step is one pass of the whole hot path over one batch of synthetic particles: zero the
tally buffer, trace the batch (emission inside the persistent kernel: source, position,
frequency, direction, sign, free flights, boundaries, relaxations, detector scores) and
finalize the tallies on the host (kappa and its standard error).  The mode tables are built
once before the timed region (inputs resident in HBM).  Each step uses its own seed.

Default workload: the 3-D periodic nanostructure -- a 500 nm cubic cell with a centred
cylindrical pore at 25 % porosity, diffuse pore wall, periodic faces, a temperature gradient
along y, the synthetic silicon-like dispersion of 1400 mode rows at 300 K, 1e8 particles,
N_scat^max = 10 -- FP32 trajectories with FP64 tables and sums.  The other configurations (the
thin film, the gray slab, the transient bump, the batched sweep, the sensitivities) are
reported under "forms".  One JSON line on stdout.
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
# sin/cos -- count 4).  Derived from the operations the method prescribes (each entry below
# names them), not from the compiled code.
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
    "snapshot_axis": 9,       # one snapshot: position along a binned axis at t_k, its cell index
}


def exact_snapshots(w: dict, counts: dict) -> int:
    """Snapshot scorings (Eq. sampling) of a transient launch where their number is fixed: every
    particle starts at t = 0 (initial-condition sources only: no heat source, no gradient, no
    isothermal face or line wall) and lives to t_max, so it scores each measurement time below t_max
    once; 0 (not counted) otherwise."""
    import numpy as np
    import workloads as W
    p, g = w["problem"], w["geometry"]
    if not p.get("transient") or p.get("heat") is not None or any(x != 0 for x in g.get("gradT", (0, 0, 0))):
        return 0
    if g.get("walls") or any(f[0] == W.ISOTHERMAL for f in g["faces"].values()):
        return 0
    if counts["timeouts"] != counts["particles"]:
        return 0
    return int(counts["particles"]) * int(np.sum(np.asarray(p["t_meas"]) < p["t_max"]))


def algorithmic_lane_ops(counts: dict, info: dict, geom: dict, ncomp: int, transient: bool,
                         two_clocks: bool = False, snapshots: int = 0, binned_axes: int = 0) -> float:
    """Lane-operations the method requires for the events of one launch (see OPS).  With a
    two-phonon clock every emission and three-phonon relaxation also draws that clock, and a
    two-phonon event draws a direction and the clock again.  A transient launch adds its snapshot
    scorings where their number is known (exact_snapshots): per snapshot the position and cell on
    each binned axis and the scored components."""
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
    clock = OPS["philox_block"] + OPS["free_flight"]       # one draw of the two-phonon clock
    two = (counts.get("two_phonon", 0) * (OPS["philox_block"] + OPS["iso_dir"] + clock)
           + (counts["particles"] + relax_draws) * clock) if two_clocks else 0
    return (emit + counts["flights"] * per_flight
            + relax_draws * (2 * OPS["philox_block"] + steps_M * OPS["search_step"] + OPS["iso_dir"]
                             + OPS["free_flight"])
            + diffuse * (OPS["philox_block"] + OPS["cos_dir"])
            + counts["rejections"] * 2 * OPS["philox_block"] + two
            + snapshots * (binned_axes * OPS["snapshot_axis"] + ncomp * OPS["tally_comp"]))


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
    if kv.get("kernel_source_sha256_16") != h.hexdigest()[:16] or "hbm_bytes_per_launch" not in kv:
        return None
    return float(kv["hbm_bytes_per_launch"])


def workload(name: str, scale: float = 1.0):
    import workloads as W
    if name == "film":
        return W.film(N=int(1_000_000 * scale)), "film_d100nm_T300K_1400modes_N1e6_nscat10"
    if name == "film_two_clocks":
        # the impurity-like A omega^4 term on its own (two-phonon) clock, section 3.3
        return (W.film(N=int(1_000_000 * scale), modes=W.silicon_like_modes(300.0, impurity_clock=True)),
                "film_d100nm_T300K_1400modes_N1e6_nscat10_two_clocks")
    if name == "film_ziman":
        # walls whose specularity follows each row's wavelength (Ziman, roughness 0.2 nm), section 3.5.3
        f = W.film(N=int(1_000_000 * scale))
        return (W.with_spec_table(f, W.ziman_specularity(f["modes"], 0.2e-9)),
                "film_d100nm_T300K_1400modes_N1e6_nscat10_ziman_eta0.2nm")
    if name == "porous_cell_spec2thz":
        # the pore reflects the phonons below 2 THz specularly (the paper's nanomesh variant)
        return (W.porous_cell(N=int(100_000_000 * scale), spec_omega=W.OMEGA_2THZ, n_scat_max=W.C5_NSCAT),
                f"porous_cell_500nm_phi0.25_N1e8_nscat{W.C5_NSCAT}_specular_below_2THz")
    if name == "lone_walker":
        # one phonon of the pore cell with a 10 cm gray free path and N_scat^max 1: a single wave walks
        # ~1e5 pore reflections (the cost of the long-free-path tail of the cell, one reflection at a time)
        w = W.porous_cell(N=max(1, int(scale)), modes=W.gray_modes(6400.0, 0.1 / 6400.0), n_scat_max=1)
        w["problem"]["format"] = 2   # the gray row gives C directly
        return w, "porous_cell_500nm_phi0.25_gray_Lambda10cm_N1_nscat1"
    if name == "gray_slab":
        return W.gray_slab(N=int(100_000 * scale)), "gray_slab_L100nm_Kn1_N1e5_50bins"
    if name == "porous_cell":
        # the relaxation cap at which the cell's kappa has converged (a smaller cap biases it)
        return (W.porous_cell(N=int(100_000_000 * scale), n_scat_max=W.C5_NSCAT),
                f"porous_cell_500nm_phi0.25_N1e8_nscat{W.C5_NSCAT}")
    if name == "transient":
        return W.transient_bump(N=int(10_000_000 * scale)), "transient_bump_1um_200times_100bins_N1e7"
    if name == "heated_slab":
        # time-domain heating: a 5 ps Gaussian pulse into the top 20 nm of a 1 um slab
        return (W.heated_slab(N=int(10_000_000 * scale)),
                "heated_slab_1um_pulse5ps_depth20nm_200times_100bins_N1e7")
    if name == "sweep":
        return W.film_sweep(scale=scale), "film_sweep_16d_x_4T_64instances_N7.2e7"
    raise SystemExit(f"unknown workload {name}")


def is_pore_lattice(w: dict) -> bool:
    """A steady cell periodic in x and y (periodic or unbounded in z) with one pore inside it and no
    line walls: the FP32 trace then walks long free paths from pore to pore with the whole wave."""
    g, p = w["geometry"], w["problem"]
    if p["transient"] or len(g["cylinders"]) != 1 or g.get("walls") or any(w["detectors"]["n"]):
        return False
    if g["unbounded"][0] or g["unbounded"][1]:
        return False
    axis = {1: 1, 2: 0, 3: 1, 4: 0, 5: 2, 6: 2}
    if any(not g["unbounded"][axis[i]] and g["faces"][i][0] != 3 for i in range(1, 7)):
        return False
    cx, cy, r = g["cylinders"][0][:3]
    return cx - r > 0 and cx + r < g["L"][0] and cy - r > 0 and cy + r < g["L"][1]


def host_cores() -> int:
    """Cores this process may run on (its CPU affinity), at most 16: the host share of one GPU on
    the benchmark machines, whatever the machine's total is."""
    try:
        n = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_rate(w, tb, threads: int, seconds: float):
    """flights/s of the oracle on whole batches of w (a new seed per batch), each batch a prefix of
    the particles sized to take a fraction of `seconds`, until `seconds` have passed."""
    import oracle
    N = w["problem"]["N"]
    t0 = time.perf_counter()
    probe = oracle.trace(w, n=min(N, 2000), threads=threads, tables=tb)
    rate = probe["counts"][0] / max(time.perf_counter() - t0, 1e-6)
    n = int(min(N, max(2000, rate * seconds / 4)))
    flights, batches = 0, 0
    t0 = time.perf_counter()
    while True:
        wb = dict(w, seed=int(w["seed"]) + batches)
        res = oracle.trace(wb, n=n, threads=threads, tables=tb)
        flights += int(res["counts"][1])
        batches += 1
        dt = time.perf_counter() - t0
        if dt >= seconds or batches >= 10000:
            break
    return flights / dt, flights, dt, batches, n


def cpu_baseline(w: dict, seconds: float, threads: int) -> dict:
    """The oracle as it stands, on the host cores (threads over contiguous particle ranges): whole
    batches of the same workload, a new seed per batch like the GPU steps, each batch a prefix of
    the particles, until about `seconds` have passed; then the same on one core for a fifth of the
    time (the single-core rate)."""
    import oracle
    tb = oracle.Tables(w)
    N = w["problem"]["N"]
    rate, flights, dt, batches, n = _oracle_rate(w, tb, threads, seconds)
    rate1, flights1, dt1, _, n1 = _oracle_rate(w, tb, 1, max(2.0, seconds / 5))
    what = f"{batches} batches of particles 0..{n - 1}" if n < N else f"{batches} full batches of {N} particles"
    return {"value": rate, "unit": "flights/s", "cores": threads, "kind": "oracle",
            "nproc": os.cpu_count(), "cpu_model": cpu_model(), "single_core_value": rate1,
            "sample": f"{what} of the same workload, new seed per batch ({flights} flights in {dt:.1f} s on "
                      f"{threads} threads over contiguous particle ranges; single core: particles 0..{n1 - 1}, "
                      f"{flights1} flights in {dt1:.1f} s)"}


def launch_config(args, tabs, w, M, precision, probe_cap: int = 4_000_000, reps: int = 3):
    """Block and refill: the caller's, else the autotuner's (outside the timed region)."""
    if args.block or args.refill or args.no_autotune:
        return {"block": args.block or 0, "refill": args.refill or 4, "autotuned": False}
    ws = w if isinstance(w, list) else [w]
    total = sum(x["problem"]["N"] for x in ws)
    t0 = time.perf_counter()
    # the calibration runs the whole batch up to probe_cap particles: a smaller probe shifts the
    # balance between the steady part and the tail of a launch, and with it the best shape
    r = M.tune(w, precision=precision, n_probe=max(1, min(total, probe_cap)), reps=reps, tables=tabs,
               segments=getattr(args, "segments", False))
    return {"block": r["block"], "refill": r["refill"], "autotuned": True,
            "tune_s": round(time.perf_counter() - t0, 3),
            "tune_candidates": M.TUNE_CANDIDATES}


def measure(args, w, M, torch, precision: int, steps: int, warmup: int, streams: int = 1,
            probe_cap: int = 4_000_000, reps: int = 3):
    """Trace `steps` batches of workload w (a new seed per step) after `warmup` untimed ones;
    HIP events bracket each trace launch on its stream."""
    t0 = time.perf_counter()
    tabs = M.Tables(w, 0)
    t_tables = time.perf_counter() - t0
    lc = launch_config(args, tabs, w, M, precision, probe_cap, reps)
    N = w["problem"]["N"]
    ncomp = bin(w["detectors"]["mask"]).count("1")
    S = max(1, streams)
    strm = [torch.cuda.current_stream()] + [torch.cuda.Stream() for _ in range(S - 1)]
    tallies = [tabs.new_tally() for _ in range(S)]
    base_seed = int(w["seed"])

    def launch(slot: int, seed: int, ev=None):
        tl = tallies[slot]
        tl.zero_()
        run = M.make_run(seed, precision, block=lc["block"], refill=lc["refill"], grid=args.grid,
                         segments=args.segments)
        if ev is not None:
            ev[0].record()
        M.trace(tabs, run, 0, N, None, tl)
        if ev is not None:
            ev[1].record()

    def run_steps(n_steps: int, seed0: int, timed: bool):
        """batch i on stream i % S; a stream's previous batch is finalized before its next one."""
        events = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                  for _ in range(n_steps)] if timed else [None] * n_steps
        pending = [False] * S
        results = []
        for i in range(n_steps):
            slot = i % S
            with torch.cuda.stream(strm[slot]):
                if pending[slot]:
                    results.append(M.tally(tabs, tallies[slot], with_arrays=False))
                launch(slot, seed0 + i, events[i])
                pending[slot] = True
        for k in range(n_steps, n_steps + S):
            slot = k % S
            if pending[slot]:
                with torch.cuda.stream(strm[slot]):
                    results.append(M.tally(tabs, tallies[slot], with_arrays=False))
                pending[slot] = False
        return results, events

    run_steps(max(warmup, 1), base_seed + 100000, False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    results, events = run_steps(steps, base_seed, True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kernel_ms = [a.elapsed_time(b) for a, b in events]
    two = bool((w["modes"]["tau_imp"] > 0).any())
    binned = sum(1 for x in w["detectors"]["n"] if x > 0)
    ops = sum(algorithmic_lane_ops(r["counts"], tabs.info, w["geometry"], ncomp, w["problem"]["transient"], two,
                                   exact_snapshots(w, r["counts"]), binned)
              for r in results)
    achieved = ops / (sum(kernel_ms) / 1e3)
    flights = sum(r["counts"]["flights"] for r in results)
    out = {"wall_s": wall, "flights_per_s": flights / wall, "ms_per_step": wall / steps * 1e3,
           "kernel_ms": kernel_ms, "lane_ops_per_launch": ops / steps, "achieved": achieved,
           "frac": achieved / PEAK_LANE_OPS, "flights_per_step": flights / steps,
           "particles_per_s": N * steps / wall,
           "relaxations_per_s": sum(r["counts"]["relaxations"] for r in results) / wall,
           "table_build_s": t_tables, "launch": lc, "tables": tabs, "last": results[-1], "results": results, "N": N,
           "pore_walk": precision == 32 and not args.segments and is_pore_lattice(w)}
    last = results[-1]
    if not w["problem"]["transient"] and last.get("kappa"):
        sig = last["kappa_sigma"] / abs(last["kappa"])
        out["kappa_eff"] = last["kappa"]
        out["kappa_sigma"] = last["kappa_sigma"]
        # time to a 0.5 % standard error at this rate: t_step (sigma_rel / 0.005)^2
        out["time_to_sigma_0p5pct_s"] = (wall / steps) * (sig / 0.005) ** 2
    return out


def measure_batched(args, ws, M, torch, precision: int, steps: int, warmup: int, probe_cap: int = 4_000_000,
                    reps: int = 3):
    """The batched form: every step traces all instances in one persistent launch."""
    t0 = time.perf_counter()
    tabs = [M.Tables(w, 0) for w in ws]
    t_tables = time.perf_counter() - t0
    lc = launch_config(args, tabs, ws, M, precision, probe_cap, reps)
    tallies = [t.new_tally() for t in tabs]
    queue = torch.zeros(M.batch_queue_bytes(len(ws)), dtype=torch.uint8, device="cuda")
    ns = [w["problem"]["N"] for w in ws]
    ids = [w["instance"] for w in ws]
    base_seed = int(ws[0]["seed"])

    def step(seed, ev=None):
        for tl in tallies:
            tl.zero_()
        run = M.make_run(seed, precision, block=lc["block"], refill=lc["refill"], grid=args.grid)
        if ev is not None:
            ev[0].record()
        M.trace_batch(tabs, ns, ids, tallies, run, queue)
        if ev is not None:
            ev[1].record()
        return [M.tally(t, tl, with_arrays=False) for t, tl in zip(tabs, tallies)]

    for i in range(max(warmup, 1)):
        step(base_seed + 100000 + i)
    torch.cuda.synchronize()
    events = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    t0 = time.perf_counter()
    results = [step(base_seed + i, events[i]) for i in range(steps)]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kernel_ms = [a.elapsed_time(b) for a, b in events]
    flights = sum(r["counts"]["flights"] for rs in results for r in rs)
    ops = sum(algorithmic_lane_ops(r["counts"], t.info, w["geometry"], bin(w["detectors"]["mask"]).count("1"), False)
              for rs in results for r, t, w in zip(rs, tabs, ws))
    achieved = ops / (sum(kernel_ms) / 1e3)
    last = results[-1]
    # each instance's cumulative kappa over mean free path from the last step's tallies (a host-side
    # finalize, outside the timed region): the free path below which half of kappa is carried and
    # the share carried by free paths up to the film's thickness
    cum = []
    for t, tl, w in zip(tabs, tallies, ws):
        c = M.kappa_cumulative(t, [tl], "mfp")
        k = c["kappa_cum"][-1]
        d = float(w["geometry"]["L"][2])
        i50 = next(i for i, v in enumerate(c["kappa_cum"]) if v >= 0.5 * k or i == len(c["keys"]) - 1)
        i_d = sum(1 for x in c["keys"] if x <= d) - 1
        cum.append({"instance": int(w["instance"]), "d_m": d, "T_K": float(w["problem"]["T_lin"]),
                    "kappa": float(k), "lambda_half_kappa_m": float(c["keys"][i50]),
                    "kappa_share_lambda_le_d": float(c["kappa_cum"][i_d] / k) if i_d >= 0 else 0.0})
    return {"wall_s": wall, "flights_per_s": flights / wall, "ms_per_step": wall / steps * 1e3,
            "kernel_ms": kernel_ms, "achieved": achieved, "frac": achieved / PEAK_LANE_OPS,
            "lane_ops_per_launch": ops / steps, "flights_per_step": flights / steps, "particles_per_step": sum(ns),
            "kappa_eff_per_instance": [r["kappa"] for r in last], "cumulative_kappa_per_instance": cum,
            "worst_kappa_sigma_rel": max(r["kappa_sigma"] / abs(r["kappa"]) for r in last),
            "table_build_s": t_tables, "launch": lc}


def measure_sensitivity(args, w, M, torch, estimators, steps: int):
    """Forward trace recording each particle's flux score, then the sensitivity replay of each
    estimator (1000 frequency bins), every launch timed with HIP events; the spread of the summed
    sensitivity over the steps is reported per estimator.  A replay re-traces the forward's
    particles event for event, so its algorithmic work is taken as the forward's (the score terms
    it adds are a few operations per relaxation and flight end) and its roofline fraction is that
    work over the replay's time."""
    tabs = M.Tables(w, 0)
    lc = launch_config(args, tabs, w, M, 32)
    N = w["problem"]["N"]
    ncomp = bin(w["detectors"]["mask"]).count("1")
    F = torch.zeros(N, dtype=torch.float64, device="cuda")
    tl = tabs.new_tally()
    adj = torch.zeros(tabs.info["adj_doubles"], dtype=torch.float64, device="cuda")
    fwd, flights, ops = [], 0, []
    rep = {e: [] for e in estimators}
    total = {e: [] for e in estimators}
    for i in range(steps + 1):
        tl.zero_()
        seed = int(w["seed"]) + i
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        M.trace(tabs, M.make_run(seed, 32, block=lc["block"], refill=lc["refill"], particle_F=F), 0, N, None, tl)
        e1.record()
        res = M.tally(tabs, tl, with_arrays=False)
        if i > 0:
            fwd.append(e0.elapsed_time(e1))
            flights += res["counts"]["flights"]
            ops.append(algorithmic_lane_ops(res["counts"], tabs.info, w["geometry"], ncomp, False))
        for est in estimators:
            adj.zero_()
            r0, r1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            r0.record()
            M.adjoint(tabs, M.make_run(seed, 32, block=lc["block"], refill=lc["refill"]), M.ESTIMATORS[est], 0, N, F,
                      adj)
            r1.record()
            d = M.adjoint_finalize(tabs, adj, N)
            if i > 0:                                     # the first step warms up
                rep[est].append(r0.elapsed_time(r1))
                total[est].append(float(d.sum()))
    out = {"forward_ms": fwd, "forward_ms_spread": _spread(fwd), "flights_per_s_forward": flights / (sum(fwd) / 1e3),
           "roofline_frac_forward": sum(ops) / (sum(fwd) / 1e3) / PEAK_LANE_OPS,
           "bins": int(tabs.info["n_bins"]), "launch": lc, "steps": steps}
    for est in estimators:
        tot = total[est]
        mean = sum(tot) / len(tot)
        sd = (sum((x - mean) ** 2 for x in tot) / max(1, len(tot) - 1)) ** 0.5
        out[est] = {"replay_ms": rep[est], "replay_ms_spread": _spread(rep[est]),
                    "roofline_frac_replay": sum(ops) / (sum(rep[est]) / 1e3) / PEAK_LANE_OPS,
                    "sum_dkappa_dlntau_per_step": tot, "sum_dkappa_dlntau_mean": mean, "sum_dkappa_dlntau_sd": sd}
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="porous_cell")
    ap.add_argument("--scale", type=float, default=1.0)
    ap.add_argument("--precision", type=int, default=32, choices=(32, 64))
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--refill", type=int, default=0)
    ap.add_argument("--grid", type=int, default=0)
    ap.add_argument("--streams", type=int, default=1)
    ap.add_argument("--no-autotune", action="store_true", help="default launch shape (block 256, refill 4)")
    ap.add_argument("--segments", action="store_true",
                    help="trace pore lattices one segment at a time in FP32 too (no pore-to-pore wave walk)")
    ap.add_argument("--no-forms", action="store_true",
                    help="skip the other configurations (thin film, gray slab FP64, transient, batched sweep, "
                         "sensitivities) reported under 'forms'")
    ap.add_argument("--only-form", default=None, metavar="KEY",
                    help="run just one of the configurations reported under 'forms' and print it")
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

    if args.only_form:
        torch.cuda.set_device(torch.device("cuda:0"))
        forms = other_forms(args, M, torch, only=args.only_form)
        if not forms:
            raise SystemExit(f"unknown form {args.only_form}")
        print(json.dumps({"form": args.only_form, **forms[args.only_form]}), flush=True)
        return
    w, wname = workload(args.workload, args.scale)
    torch.cuda.set_device(torch.device("cuda:0"))
    dtype = "f32" if args.precision == 32 else "f64"
    common = {"metric": METRIC, "unit": "flights/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
              "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": dtype, "data": "synthetic"}
    if isinstance(w, list):
        m = measure_batched(args, w, M, torch, args.precision, args.steps, args.warmup)
        out = dict(common, value=m["flights_per_s"], ms_per_step=m["ms_per_step"],
                   config={"workload": wname, "instances": len(w), "particles_per_step": m["particles_per_step"],
                           "precision": args.precision, "tallies": "f64", "launch": m["launch"],
                           "parallelism": "single GPU, one batched launch"},
                   roofline={"bound": "alu", "achieved": m["achieved"] / 1e12, "peak": PEAK_LANE_OPS / 1e12,
                             "unit": "T lane-op/s", "frac": m["frac"], "traffic": None, "kernel": "k_trace_batch",
                             "kernel_ms": sum(m["kernel_ms"]) / len(m["kernel_ms"])},
                   kernel_ms_per_step=m["kernel_ms"], kappa_eff_per_instance=m["kappa_eff_per_instance"],
                   cumulative_kappa_per_instance=m["cumulative_kappa_per_instance"],
                   worst_kappa_sigma_rel=m["worst_kappa_sigma_rel"], table_build_s=m["table_build_s"])
        if not args.no_cpu_baseline:
            out["cpu_baseline"] = cpu_baseline(w[-1], args.cpu_seconds, host_cores())
        print(json.dumps(out), flush=True)
        return
    print(f"[bench] main line: {wname}, FP{args.precision}", file=sys.stderr, flush=True)
    m = measure(args, w, M, torch, args.precision, args.steps, args.warmup, args.streams)
    S = max(1, args.streams)
    tag = f"k_trace_solo_{args.workload}_fp{args.precision}"
    out = dict(common, value=m["flights_per_s"], ms_per_step=m["ms_per_step"],
               config={"workload": wname, "particles_per_step": m["N"], "modes": int(m["tables"].info["n_modes"]),
                       "precision": args.precision, "tallies": "f64", "streams": S, "launch": m["launch"],
                       "pore_walk": m["pore_walk"],
                       "parallelism": "single GPU" + (", batches overlapped on %d streams" % S if S > 1 else "")},
               roofline={"bound": "alu", "achieved": m["achieved"] / 1e12, "peak": PEAK_LANE_OPS / 1e12,
                         "unit": "T lane-op/s", "frac": m["frac"],
                         "traffic": profiled_traffic(tag) if S == 1 and not args.segments else None,
                         "kernel": "k_trace_solo", "profile": f"profiles/{tag}.txt",
                         "kernel_ms": sum(m["kernel_ms"]) / len(m["kernel_ms"]),
                         "lane_ops_per_launch": m["lane_ops_per_launch"]},
               kernel_ms_per_step=m["kernel_ms"], kernel_ms_spread=_spread(m["kernel_ms"]),
               flights_per_step=m["flights_per_step"],
               particles_per_s=m["particles_per_s"], relaxations_per_s=m["relaxations_per_s"],
               table_build_s=m["table_build_s"])
    for k in ("kappa_eff", "kappa_sigma", "time_to_sigma_0p5pct_s"):
        if k in m:
            out[k] = m[k]
    if args.workload == "lone_walker" and S == 1:
        # per launch: the walked pore reflections and periodic transfers, and the launch time per reflection
        refl = [r["counts"]["diffuse"] + r["counts"]["specular"] for r in m["results"]]
        out["walk"] = {"reflections": refl, "periodic": [r["counts"]["periodic"] for r in m["results"]],
                       "ns_per_reflection": [t * 1e6 / max(n, 1) for t, n in zip(m["kernel_ms"], refl)]}
    if not args.no_forms and args.workload == "porous_cell" and args.precision == 32 and S == 1:
        out["forms"] = other_forms(args, M, torch)
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds, host_cores())
    print(json.dumps(out), flush=True)


def _spread(xs) -> dict:
    ys = sorted(xs)
    return {"min": ys[0], "median": ys[len(ys) // 2], "max": ys[-1], "n": len(ys)}


def _brief(m: dict, workload: str, precision: int) -> dict:
    r = {"workload": workload, "precision": precision, "flights_per_s": m["flights_per_s"],
         "ms_per_step": m["ms_per_step"], "kernel_ms": sum(m["kernel_ms"]) / len(m["kernel_ms"]),
         "kernel_ms_spread": _spread(m["kernel_ms"]),
         "roofline_frac": m["frac"], "achieved_T_lane_ops": m["achieved"] / 1e12, "launch": m["launch"]}
    for k in ("kappa_eff", "kappa_sigma", "time_to_sigma_0p5pct_s", "kappa_eff_per_instance",
              "cumulative_kappa_per_instance", "worst_kappa_sigma_rel", "particles_per_step"):
        if k in m:
            r[k] = m[k]
    return r


def other_forms(args, M, torch, only: str | None = None) -> dict:
    """The remaining configurations, a few steps each, every one timed like the main line (only:
    just the form of that key).  A form's HBM traffic is the committed rocprofv3 figure of its
    kernel and workload while the kernel source is unchanged since it was taken."""
    forms = {}

    def want(key):
        return only is None or only == key

    plan = [("film_fp32", "film", 32, 20), ("gray_slab_fp64", "gray_slab", 64, 10), ("film_fp64", "film", 64, 5),
            ("transient_fp32", "transient", 32, 3), ("film_two_clocks_fp32", "film_two_clocks", 32, 10),
            ("film_ziman_specularity_fp32", "film_ziman", 32, 10), ("heated_slab_fp32", "heated_slab", 32, 3),
            ("porous_cell_specular_below_2THz_fp32", "porous_cell_spec2thz", 32, 5)]
    # each configuration is tuned on at most 1e6 particles with one timed launch per candidate
    # (the calibration stays outside the timed steps but inside the run's few minutes)
    for key, name, prec, steps in plan:
        if not want(key):
            continue
        w, wname = workload(name, 1.0)
        print(f"[bench] form {key}: {wname}", file=sys.stderr, flush=True)
        forms[key] = _brief(measure(args, w, M, torch, prec, steps, 1, 1, 1_000_000, 1), wname, prec)
        forms[key]["traffic"] = profiled_traffic(f"k_trace_solo_{name}_fp{prec}")
    # the main line's launches each end with a tail (the last particles of every wave, one
    # flight after another) of about half a launch; a job of many batches overlaps one batch's
    # tail with the next batch on a second stream (throughput by wall clock, no roofline figure)
    w, wname = workload("film", 1.0)
    if want("film_fp32_two_streams"):
        print(f"[bench] form film_fp32_two_streams: {wname}", file=sys.stderr, flush=True)
        mf = measure(args, w, M, torch, 32, 20, 3, 2, 1_000_000, 1)
        forms["film_fp32_two_streams"] = {
            "workload": wname, "precision": 32, "streams": 2, "steps": 20, "flights_per_s": mf["flights_per_s"],
            "ms_per_step": mf["ms_per_step"], "launch": mf["launch"], "kappa_eff": mf.get("kappa_eff"),
            "kappa_sigma": mf.get("kappa_sigma")}
    # the same pore cell traced one segment at a time (no pore-to-pore walk by the wave): the
    # step then waits for the few particles of the longest free paths, one lane each
    w, wname = workload("porous_cell", 1.0)
    if want("porous_cell_fp32_segments"):
        print(f"[bench] form porous_cell_fp32_segments: {wname}", file=sys.stderr, flush=True)
        seg_args = argparse.Namespace(**dict(vars(args), segments=True))
        forms["porous_cell_fp32_segments"] = _brief(measure(seg_args, w, M, torch, 32, 4, 1, 1, 1_000_000, 1),
                                                    wname, 32)
    # a job of several batches overlaps each batch's tail (its last particles) with the next
    # batches on other streams (throughput by wall clock; the per-launch event times then include
    # the overlap, so no roofline figure is given for it)
    if want("porous_cell_fp32_four_streams"):
        print(f"[bench] form porous_cell_fp32_four_streams: {wname}", file=sys.stderr, flush=True)
        m2 = measure(args, w, M, torch, 32, 8, 2, 4, 1_000_000, 1)
        forms["porous_cell_fp32_four_streams"] = {
            "workload": wname, "precision": 32, "streams": 4, "steps": 8, "flights_per_s": m2["flights_per_s"],
            "ms_per_step": m2["ms_per_step"], "launch": m2["launch"], "kappa_eff": m2.get("kappa_eff"),
            "kappa_sigma": m2.get("kappa_sigma")}
    if want("batched_sweep_fp32"):
        ws, wname = workload("sweep", 1.0)
        print(f"[bench] form batched_sweep_fp32: {wname}", file=sys.stderr, flush=True)
        forms["batched_sweep_fp32"] = _brief(measure_batched(args, ws, M, torch, 32, 3, 1, 8_000_000, 1), wname, 32)
        forms["batched_sweep_fp32"]["traffic"] = profiled_traffic("k_trace_batch_sweep_fp32")
    if want("porous_cell_sensitivities_fp32"):
        w, wname = workload("porous_cell", 1.0)
        print(f"[bench] form sensitivities: {wname}", file=sys.stderr, flush=True)
        sens = measure_sensitivity(args, w, M, torch, ("score", "local"), 5)
        sens["workload"] = wname
        forms["porous_cell_sensitivities_fp32"] = sens
    return forms


if __name__ == "__main__":
    main()
