"""Parity of the HIP path (through the C ABI) with the CPU oracle.

FP64 form: emitted states, per-particle event sequences and every integer counter are
bit-exact; raw FP64 sums agree to 1e-10 of the largest sum (atomic accumulation order is free).
FP32 form: same random streams; tallies against the FP64 oracle within the stated tolerances.
"""
import math
import os

import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

THREADS = min(16, os.cpu_count() or 1)


def _pkg():
    import paper_2104_03573_amd as M
    return M


def _say(*a):
    print(*a, flush=True)


FP64_CASES = {
    "gray_slab": lambda: W.gray_slab(N=3000),
    "gray_slab_thick": lambda: W.gray_slab(N=2000, Lambda=25e-9),
    "film": lambda: W.film(N=3000),
    "film_partial_specular": lambda: W.film(N=2000, d=30e-9, specularity=0.4),
    "film_zbins": lambda: W.film(N=1500, z_bins=7),
    "transient_bump": lambda: W.transient_bump(N=400),
    # uneven measurement times: log-spaced, a tight cluster, repeats, one at the time horizon
    "transient_uneven_times": lambda: W.with_(W.transient_bump(N=600, n_times=8), **{
        "problem.t_max": 2e-9, "problem.t_meas": np.sort(np.concatenate([np.geomspace(1e-14, 1.5e-9, 40), 7.3e-10 + 1e-15 * np.arange(12),
                                                  [3e-10, 3e-10, 3e-10, 2e-9]]))}),
    "porous_cell": lambda: W.porous_cell(N=2000),
    "porous_cell_specular": lambda: W.porous_cell(N=1000, specularity=0.5),
    # the same lattice driven along x, and with the pore moved off the cell's centre
    "porous_cell_x": lambda: W.with_(W.porous_cell(N=1500), **{"geometry.gradT": (-2.0e6, 0.0, 0.0),
                                                              "problem.score_axis": 0}),
    "porous_cell_moved": lambda: W.with_(W.porous_cell(N=1500), **{"geometry.cylinders": [
        (150e-9, 350e-9) + tuple(W.porous_cell(N=1)["geometry"]["cylinders"][0][2:])]}),
    "ballistic_transient": lambda: W.ballistic_transient(N=3000),
    "bulk_dispersive": lambda: W.bulk_gradient(N=2000, n_scat_max=3, modes=W.silicon_like_modes(300.0)),
    "grid3d": lambda: W.with_(W.gray_slab(N=1500), **{"detectors.lo": (0.0, 0.0, 0.0),
                                                      "detectors.hi": (3e-8, 2e-8, 1e-7),
                                                      "detectors.n": (3, 2, 5)}),
    # separate two-phonon and three-phonon clocks
    "film_two_clocks": lambda: W.film(N=3000, modes=W.silicon_like_modes(300.0, impurity_clock=True)),
    "gray_slab_two_clocks": lambda: W.with_(W.gray_slab(N=2000),
                                            modes=W.gray_modes(6400.0, 3e-11, tau_imp=1.5e-11)),
    "bulk_two_clocks": lambda: W.bulk_gradient(N=2000, n_scat_max=3,
                                               modes=W.silicon_like_modes(300.0, impurity_clock=True)),
    "transient_two_clocks": lambda: W.transient_bump(N=300, modes=W.silicon_like_modes(300.0, impurity_clock=True)),
    "porous_two_clocks": lambda: W.porous_cell(N=1000, modes=W.silicon_like_modes(300.0, impurity_clock=True)),
    # frequency-dependent specularity: phonons below the cutoff reflect specularly
    "film_spec_cutoff": lambda: W.film(N=3000, spec_omega=2.5 * W.OMEGA_2THZ),
    "film_partial_spec_cutoff": lambda: W.film(N=2000, d=30e-9, specularity=0.4, spec_omega=2.5 * W.OMEGA_2THZ),
    "porous_spec_cutoff": lambda: W.porous_cell(N=1000, spec_omega=W.OMEGA_2THZ),
    # specularity per material row from a table (random in [0, 1), or 0 / 1 at random: the film's
    # cooperative bouncing then runs the diffuse rows, the cell's lone-lane walk the others)
    "film_spec_table": lambda: W.with_spec_table(W.film(N=2000, d=30e-9), W.random_specularity(1400, 3)),
    "film_spec_table_binary": lambda: W.with_spec_table(W.film(N=3000), W.random_specularity(1400, 4, binary=True)),
    "porous_spec_table": lambda: W.with_spec_table(W.porous_cell(N=1000), W.random_specularity(1400, 5)),
    "porous_spec_table_binary": lambda: W.with_spec_table(W.porous_cell(N=1500),
                                                          W.random_specularity(1400, 6, binary=True)),
    "walled_spec_table": lambda: W.with_spec_table(W.walled_film(N=1500), W.random_specularity(1400, 7)),
    # the external heat source: a Gaussian pulse in the top layer of a slab; heating then cooling
    # in a strip of the porous cell beside its pore (with the gradient source of the cell)
    "heated_slab": lambda: W.heated_slab(N=1500, t_max=100e-12, n_times=20, n_cells=20),
    "porous_heat": lambda: W.with_(W.porous_cell(N=1200), **{
        "problem.transient": True, "problem.t_max": 60e-12, "problem.t_meas": np.array([10e-12, 30e-12, 59e-12]),
        "detectors.lo": (0.0, 0.0, 0.0), "detectors.hi": (500e-9, 0.0, 0.0), "detectors.n": (5, 0, 0),
        "problem.heat": {"lo": (0.0, 0.0, 0.0), "hi": (80e-9, 500e-9, 500e-9), "t": np.array([0.0, 5e-12, 20e-12]),
                         "P": np.array([2e17, -5e16])}}),
    # heat-source regions built from tetrahedra: one in a corner of a closed box (specular and
    # diffuse walls), and a cuboid as six tetrahedra next to a seventh (silicon-like rows)
    "heated_box_tet": lambda: W.heated_box(N=1500),
    "heated_box_tets_diffuse": lambda: W.heated_box(
        N=1200, specularity=0.0, modes=W.silicon_like_modes(300.0),
        tets=np.concatenate([W.cube_tets((50e-9, 40e-9, 30e-9), (350e-9, 240e-9, 130e-9)),
                             [[[20e-9, 260e-9, 20e-9], [390e-9, 280e-9, 30e-9], [60e-9, 295e-9, 40e-9],
                               [80e-9, 270e-9, 190e-9]]]])),
    # internal line walls: the paper's square pore of four walls, a channel between two walls
    "square_pore_walls": lambda: W.square_pore_cell(N=1000),
    "square_pore_walls_partial": lambda: W.square_pore_cell(N=800, specularity=0.5),
    "walled_film": lambda: W.walled_film(N=2000),
    "walled_slab": lambda: W.walled_slab(N=2000),     # isothermal line walls: emission and absorption
    # the extended physics together: walls with a cutoff and partial specularity, two clocks
    "square_pore_all": lambda: W.with_(W.square_pore_cell(N=800, modes=W.silicon_like_modes(300.0, impurity_clock=True)),
                                       **{"geometry.walls": [c[:8] + (0.5, W.OMEGA_2THZ) for c in
                                                             W.square_pore_cell(N=1)["geometry"]["walls"]]}),
    # isothermal line walls switched on at t = 0, measured at a few times
    "walled_slab_transient": lambda: W.with_(W.walled_slab(N=1500, Lambda=50e-9),
                                             **{"problem.transient": True, "problem.t_max": 40e-12,
                                                "problem.t_meas": np.array([5e-12, 10e-12, 20e-12, 39e-12]),
                                                "detectors.lo": (0.0, 100e-9, 0.0), "detectors.hi": (200e-9, 200e-9, 0.0),
                                                "detectors.n": (0, 5, 0)}),
}


def _first_log_mismatch(a, b):
    for i in range(len(a)):
        if not np.array_equal(a[i], b[i]):
            n = int(max(a[i][0], b[i][0]))
            ea = [(int(e) >> 28, (int(e) >> 20) & 255, int(e) & 0xFFFFF) for e in a[i][1:1 + min(n, len(a[i]) - 1)]]
            eb = [(int(e) >> 28, (int(e) >> 20) & 255, int(e) & 0xFFFFF) for e in b[i][1:1 + min(n, len(b[i]) - 1)]]
            k = next((j for j in range(min(len(ea), len(eb))) if ea[j] != eb[j]), None)
            return i, k, ea[max(0, (k or 0) - 2):(k or 0) + 3], eb[max(0, (k or 0) - 2):(k or 0) + 3]
    return None


@pytest.mark.parametrize("name", list(FP64_CASES))
def test_fp64_event_sequences_bit_exact(name):
    M = _pkg()
    w = FP64_CASES[name]()
    n = w["problem"]["N"]
    stride = 96
    _say(f"[fp64 parity] {name} N={n}")
    got = M.run(w, precision=64, n_log=n, log_stride=stride)
    ref = oracle.trace(w, n_log=n, log_stride=stride, threads=THREADS)
    mism = _first_log_mismatch(got["log"], ref["log"])
    assert mism is None, f"first differing particle / event: {mism}"
    assert np.array_equal(got["counts_raw"], ref["counts"]), (got["counts_raw"], ref["counts"])
    r_ref = ref["raw"].reshape(got["raw"].shape)
    scale = np.abs(r_ref).max()
    err = np.abs(got["raw"] - r_ref).max() / scale
    _say(f"   counts {got['counts']}  max raw err / max = {err:.2e}")
    assert err <= 1e-10
    if not w["problem"]["transient"]:
        assert np.allclose(got["moments"], ref["moments"], rtol=1e-10, atol=1e-10 * np.abs(ref["moments"]).max())


def _read_state(M, buf, precision, cap):
    b = buf.cpu().numpy()
    rb = precision // 8
    fb = (cap * rb + 255) // 256 * 256
    ib = (cap * 4 + 255) // 256 * 256
    rt = np.float64 if precision == 64 else np.float32
    f = [np.frombuffer(b[q * fb:q * fb + cap * rb].tobytes(), dtype=rt) for q in range(8)]
    i = [np.frombuffer(b[8 * fb + q * ib:8 * fb + q * ib + cap * 4].tobytes(), dtype=np.int32) for q in range(7)]
    return np.stack(f, 1), np.stack(i, 1)


@pytest.mark.parametrize("name", ["heated_box_tets_diffuse", "heated_slab", "gray_slab", "film", "transient_bump", "porous_cell", "ballistic_transient",
                                  "square_pore_walls", "walled_slab", "film_two_clocks"])
def test_emission_matches_oracle(name):
    import torch
    M = _pkg()
    w = FP64_CASES[name]()
    n = 1500
    t = M.Tables(w)
    o = oracle.Tables(w)
    for prec in (64, 32):
        buf = torch.zeros(M.state_bytes(prec, n), dtype=torch.uint8, device="cuda")
        run = M.make_run(int(w["seed"]), prec)
        M.emit(t, run, 100, n, buf, n)
        torch.cuda.synchronize()
        f, i = _read_state(M, buf, prec, n)
        ref_f = np.zeros((n, 8))
        ref_i = np.zeros((n, 4), dtype=np.int32)
        for k in range(n):
            ref_f[k], ref_i[k] = o.emit_state(100 + k)
        assert np.array_equal(i[:, 0], ref_i[:, 0]) and np.array_equal(i[:, 1], ref_i[:, 1])   # mode, sign
        assert np.array_equal(i[:, 5], ref_i[:, 2]) and np.array_equal(i[:, 6], ref_i[:, 3])   # source, rejections
        if prec == 64:
            # positions and times: products of exactly rounded values -> identical
            assert np.array_equal(f[:, [0, 1, 2, 6]], ref_f[:, [0, 1, 2, 6]])
            # directions (sin, cos) and free flights (log): libm vs device math within 2 ulp
            ulp = np.spacing(np.maximum(np.abs(ref_f[:, [3, 4, 5, 7]]), 1e-300))
            assert np.all(np.abs(f[:, [3, 4, 5, 7]] - ref_f[:, [3, 4, 5, 7]]) <= 2 * ulp + 1e-300)
        else:
            # FP32 form: 24-bit uniforms (common random numbers), single-precision arithmetic
            f64 = f.astype(np.float64)
            ext = np.array([max(abs(x), 1.0) if u else x for x, u in zip(w["geometry"]["L"],
                                                                       w["geometry"]["unbounded"])])
            assert np.all(np.abs(f64[:, :3] - ref_f[:, :3]) <= 2e-6 * ext[None, :])         # positions
            assert np.all(np.abs(f64[:, 3:6] - ref_f[:, 3:6]) <= 4e-6)                      # directions
            t_scale = max(w["problem"]["t_max"], 1e-30)
            assert np.all(np.abs(f64[:, 6] - ref_f[:, 6]) <= 2e-6 * t_scale)               # start times
            rel = np.abs(f64[:, 7] - ref_f[:, 7]) / ref_f[:, 7]                            # free flights
            assert np.median(rel) < 2e-6 and rel.max() < 1e-2, (np.median(rel), rel.max())


def _oracle_full(w, n=None):
    return oracle.run(w, n=n, threads=THREADS)


@pytest.mark.parametrize("name", ["film", "porous_cell"])
def test_fp32_tallies_against_fp64_oracle(name):
    """FP32 trajectories, FP64 tables and sums, same random streams as the oracle.  Film: kappa
    and the flux total within 2e-4 relative (a particle whose FP32 decisions flip at a near-tie
    diverges; its share of a 1e5-particle total is ~1e-5).  Porous cell: long ballistic
    trajectories through the periodic channels between pores accumulate FP32 position error
    over many transfers and flip later decisions, so the FP32 estimate is an independent-looking
    sample for those heavy particles: kappa agrees within 3 oracle standard errors."""
    M = _pkg()
    w = {"film": lambda: W.film(N=100000), "porous_cell": lambda: W.porous_cell(N=60000)}[name]()
    got = M.run(w, precision=32)
    ref = _oracle_full(w)
    rel_k = abs(got["kappa"] - ref["kappa"]) / abs(ref["kappa"])
    flights_rel = abs(got["counts"]["flights"] - ref["counts"]["flights"]) / ref["counts"]["flights"]
    q = got["q"][..., 1].sum(), ref["q"][..., 1].sum()
    per_mode = np.abs(got["q"][0, :, 1] - ref["q"][0, :, 1]).max() / np.abs(ref["q"][0, :, 1]).max()
    _say(f"[fp32 vs oracle] {name}: kappa {got['kappa']:.6g} vs {ref['kappa']:.6g} (rel {rel_k:.2e}, "
         f"sigma {ref['kappa_sigma'] / abs(ref['kappa']):.2e}), flights rel {flights_rel:.2e}, "
         f"q_y tot rel {abs(q[0] - q[1]) / abs(q[1]):.2e}, per-mode q_y max err/max {per_mode:.2e}")
    assert got["counts"]["particles"] == ref["counts"]["particles"]
    if name == "film":
        assert rel_k < 2e-4
        assert flights_rel < 1e-3
        assert abs(q[0] - q[1]) / abs(q[1]) < 2e-4
        assert per_mode < 2e-2
    else:
        assert abs(got["kappa"] - ref["kappa"]) < 3.0 * ref["kappa_sigma"]
        assert flights_rel < 1e-2


def test_fp64_launch_shape_invariance():
    """Block size, refill period and grid change only the order of FP64 atomics."""
    M = _pkg()
    w = W.film(N=20000, d=40e-9)
    base = M.run(w, precision=64)
    for block, refill, grid in ((64, 1, 7), (128, 16, 300), (256, 3, 0), (192, 32, 1)):
        r = M.run(w, precision=64, block=block, refill=refill, grid=grid)
        assert np.array_equal(r["counts_raw"], base["counts_raw"]), (block, refill, grid)
        scale = np.abs(base["raw"]).max()
        assert np.abs(r["raw"] - base["raw"]).max() <= 1e-12 * scale


@pytest.mark.parametrize("precision", [64, 32])
def test_grid_pieces_scored_by_the_wave_match_per_lane_scoring(precision):
    """Gray slab with 50 detector cells: in sparse waves the whole wave scores the pending
    segments' grid pieces, in dense waves each lane walks its own; launch shapes that mix the two
    differently give the same counters and the same sums up to summation order."""
    M = _pkg()
    w = W.gray_slab(N=4000)
    base = M.run(w, precision=precision)
    for block, refill, grid in ((64, 1, 1), (64, 4, 0), (256, 64, 2)):
        r = M.run(w, precision=precision, block=block, refill=refill, grid=grid)
        assert np.array_equal(r["counts_raw"], base["counts_raw"]), (block, refill, grid)
        scale = np.abs(base["raw"]).max()
        assert np.abs(r["raw"] - base["raw"]).max() <= 1e-12 * scale, (block, refill, grid)


def test_emit_then_trace_equals_fused():
    M = _pkg()
    for w, prec in ((W.film(N=5000), 64), (W.transient_bump(N=300), 64), (W.film(N=5000), 32),
                    (W.square_pore_cell(N=2000), 64), (W.walled_slab(N=3000), 64),
                    (W.porous_cell(N=2000, spec_omega=W.OMEGA_2THZ), 32)):
        fused = M.run(w, precision=prec, n_log=200, log_stride=64)
        staged = M.run(w, precision=prec, n_log=200, log_stride=64, emit_first=True)
        assert np.array_equal(fused["counts_raw"], staged["counts_raw"])
        assert np.array_equal(fused["log"], staged["log"])
        scale = np.abs(fused["raw"]).max()
        assert np.abs(fused["raw"] - staged["raw"]).max() <= 1e-12 * scale


def test_partition_of_particle_ranges_accumulates():
    import torch
    M = _pkg()
    w = W.film(N=9000)
    t = M.Tables(w)
    one = t.new_tally()
    two = t.new_tally()
    run = M.make_run(int(w["seed"]), 64)
    M.trace(t, run, 0, 9000, None, one)
    M.trace(t, run, 0, 4000, None, two)
    M.trace(t, run, 4000, 5000, None, two)
    a, b = M.tally(t, one), M.tally(t, two)
    assert np.array_equal(a["counts_raw"], b["counts_raw"])
    assert np.abs(t.raw(one) - t.raw(two)).max() <= 1e-12 * np.abs(t.raw(one)).max()
    torch.cuda.synchronize()


def test_batched_launch_equals_solo_runs():
    import torch
    M = _pkg()
    ws = [W.film(N=n, d=d, T=T) for n, d, T in ((12000, 2e-8, 300.0), (3000, 1e-7, 100.0), (20000, 5e-7, 400.0),
                                                 (1, 1e-8, 200.0))]
    for i, w in enumerate(ws):
        w["instance"] = 5 + i
    for prec in (64, 32):
        tabs = [M.Tables(w) for w in ws]
        tallies = [t.new_tally() for t in tabs]
        queue = torch.zeros(M.batch_queue_bytes(len(ws)), dtype=torch.uint8, device="cuda")
        run = M.make_run(int(ws[0]["seed"]), prec)
        M.trace_batch(tabs, [w["problem"]["N"] for w in ws], [w["instance"] for w in ws], tallies, run, queue)
        for w, t, tl in zip(ws, tabs, tallies):
            b = M.tally(t, tl)
            s = M.run(w, precision=prec, tables=t)
            assert np.array_equal(b["counts_raw"], s["counts_raw"]), (w["name"], b["counts"], s["counts"])
            assert np.abs(t.raw(tl) - s["raw"]).max() <= 1e-12 * np.abs(s["raw"]).max()


@pytest.mark.parametrize("name", ["film", "film_two_clocks"])
def test_fp32_trace_from_emitted_states_equals_the_inline_trace(name):
    """FP32 steady traces from states written by mcbte_emit run a kernel without the event log; the
    particles and every counter are those of the trace that emits inline (FP64 sums to rounding)."""
    import torch
    M = _pkg()
    w = W.film(N=50_000) if name == "film" else W.film(N=50_000, modes=W.silicon_like_modes(300.0, impurity_clock=True))
    t = M.Tables(w)
    n = w["problem"]["N"]
    for block, refill in ((0, 0), (64, 1)):
        run = M.make_run(int(w["seed"]), 32, block=block, refill=refill)
        st = torch.zeros(M.state_bytes(32, n), dtype=torch.uint8, device="cuda")
        M.emit(t, run, 0, n, st, n)
        a_tl, b_tl = t.new_tally(), t.new_tally()
        M.trace(t, run, 0, n, st, a_tl)
        M.trace(t, run, 0, n, None, b_tl)
        a, b = M.tally(t, a_tl), M.tally(t, b_tl)
        assert np.array_equal(a["counts_raw"], b["counts_raw"]), (block, refill, a["counts"], b["counts"])
        assert np.abs(t.raw(a_tl) - t.raw(b_tl)).max() <= 1e-6 * np.abs(t.raw(b_tl)).max()


def test_batched_transient_launch_equals_solo_runs():
    """Transient instances (a bump with uneven measurement times, a pulse-heated slab, the bump
    on its regular grid) in one batched launch: the batched kernel's snapshot scoring gives each
    instance the solo run's counters exactly and its sums to rounding (FP64), and the same counters
    in FP32 (the solo FP32 launch sums snapshots in FP32 per workgroup, the batched one in FP64)."""
    import torch
    M = _pkg()
    ws = [FP64_CASES["transient_uneven_times"](), W.heated_slab(N=700, t_max=100e-12, n_times=20, n_cells=10),
          W.transient_bump(N=900, n_times=40)]
    for i, w in enumerate(ws):
        w["instance"] = 11 + i
        w["seed"] = ws[0]["seed"]            # one launch, one key: instances differ by their ids
    for prec in (64, 32):
        tabs = [M.Tables(w) for w in ws]
        tallies = [t.new_tally() for t in tabs]
        queue = torch.zeros(M.batch_queue_bytes(len(ws)), dtype=torch.uint8, device="cuda")
        run = M.make_run(int(ws[0]["seed"]), prec)
        M.trace_batch(tabs, [w["problem"]["N"] for w in ws], [w["instance"] for w in ws], tallies, run, queue)
        for w, t, tl in zip(ws, tabs, tallies):
            b = M.tally(t, tl)
            s = M.run(w, precision=prec, tables=t)
            assert np.array_equal(b["counts_raw"], s["counts_raw"]), (prec, w["name"], b["counts"], s["counts"])
            scale = np.abs(s["raw"]).max()
            assert np.abs(t.raw(tl) - s["raw"]).max() <= (1e-12 if prec == 64 else 1e-5) * scale, (prec, w["name"])


def test_full_size_film_fp32_against_oracle():
    """The benchmark workload at full size (1e6 particles, FP32, default launch shape) against
    the FP64 oracle on the same particles."""
    M = _pkg()
    w = W.film(N=1_000_000)
    got = M.run(w, precision=32)
    ref = _oracle_full(w)
    rel_k = abs(got["kappa"] - ref["kappa"]) / abs(ref["kappa"])
    _say(f"[full film] kappa gpu {got['kappa']:.6f} oracle {ref['kappa']:.6f} rel {rel_k:.2e} "
         f"sigma_rel {ref['kappa_sigma'] / ref['kappa']:.2e} counts gpu {got['counts']} oracle {ref['counts']}")
    assert got["counts"]["particles"] == 1_000_000
    assert rel_k < 1e-4
    assert abs(got["counts"]["flights"] - ref["counts"]["flights"]) <= 1e-3 * ref["counts"]["flights"]


@pytest.mark.parametrize("lam,spec", [(20e-6, 0.0), (20e-6, 1.0), (2e-6, 0.5)])
def test_fp32_long_flights_in_pore_lattice_against_fp64_oracle(lam, spec):
    """Gray medium in the porous cell with mean free paths of 2-20 um (4-40 cells per free
    path on average, thousands for the long ones; diffuse, specular and partly specular pore):
    every event count of the FP32 trajectories agrees with the FP64 oracle's on the same
    particles within 1 %, and kappa within 3 oracle standard errors."""
    M = _pkg()
    gray = W.gray_modes(6400.0, lam / 6400.0)
    w = W.with_(W.porous_cell(N=20000, modes=gray, specularity=spec, n_scat_max=4), **{"problem.format": 2})
    got = M.run(w, precision=32)
    ref = _oracle_full(w)
    c, r = got["counts"], ref["counts"]
    _say(f"[pore lattice] lam {lam:g} spec {spec}: kappa {got['kappa']:.5g} vs {ref['kappa']:.5g} "
         f"(sigma {ref['kappa_sigma']:.3g}); periodic {c['periodic']} vs {r['periodic']}, "
         f"pore hits {c['diffuse'] + c['specular']} vs {r['diffuse'] + r['specular']}")
    for k in ("particles", "relaxations", "nscat_end", "rejections"):
        assert c[k] == r[k], k
    for k in ("flights", "periodic"):
        assert abs(c[k] - r[k]) <= 0.01 * r[k], k
    hits = c["diffuse"] + c["specular"], r["diffuse"] + r["specular"]
    assert abs(hits[0] - hits[1]) <= 0.01 * hits[1] + 5
    assert c["escaped"] == 0 and c["cap_end"] == 0
    assert abs(got["kappa"] - ref["kappa"]) < 3.0 * ref["kappa_sigma"]


def test_fp64_long_pore_lattice_walks_independent_of_launch_shape():
    """Free paths of 20 um (40 cells) in the pore cell: the FP64 event sequences, counters and
    particle scores do not depend on the launch shape, which decides when a lane is the last one
    of its wave and follows its chains of periodic transfers within one call.  (Against the oracle
    such walks agree only up to the tens of pore reflections after which the lattice's dispersion
    of neighbouring rays has grown the last-place differences of the device and host sin, cos and
    log into different events; the FP32 counts are compared with the oracle's statistically.)"""
    M = _pkg()
    w = W.with_(W.porous_cell(N=300, modes=W.gray_modes(6400.0, 20e-6 / 6400.0), n_scat_max=3),
                **{"problem.format": 2})
    n, stride = 300, 2048
    runs = [M.run(w, precision=64, n_log=n, log_stride=stride, **shape)
            for shape in ({}, {"block": 64, "refill": 1}, {"block": 256, "refill": 64, "grid": 2})]
    base = runs[0]
    assert int(base["log"][:, 0].max()) + 1 < stride
    for r in runs[1:]:
        assert np.array_equal(r["log"], base["log"])
        assert np.array_equal(r["counts_raw"], base["counts_raw"])
        scale = np.abs(base["raw"]).max()
        assert np.abs(r["raw"] - base["raw"]).max() <= 1e-12 * scale
    _say(f"[long walks] counts {base['counts']}")
    assert base["counts"]["periodic"] > 20 * n


@pytest.mark.parametrize("spec", [0.0, 1.0, 0.5])
@pytest.mark.parametrize("precision", [64, 32])
def test_lone_lane_walk_matches_one_segment_steps(precision, spec):
    """Free paths of 20 um in the pore cell, 300 particles (few per wave): the last live lane of
    a wave runs its periodic transfers and diffuse or specular pore reflections in the lone-lane
    loop (a partly specular pore stops it), the event-logging launch takes one segment per step.
    Both give the same counters and the same particle scores; the tally sums agree to rounding.
    (FP32 runs step one segment at a time here, MCBTE_RUN_SEGMENTS: the wave's pore-to-pore walk
    of long free paths rounds differently and has tests of its own.)"""
    M = _pkg()
    w = W.with_(W.porous_cell(N=300, modes=W.gray_modes(6400.0, 20e-6 / 6400.0), n_scat_max=3,
                              specularity=spec), **{"problem.format": 2})
    seg = {"segments": True} if precision == 32 else {}
    plain = M.run(w, precision=precision, **seg)
    other = M.run(w, precision=precision, block=64, refill=1, **seg)
    logged = M.run(w, precision=precision, n_log=300, log_stride=16)
    for r in (other, logged):
        assert np.array_equal(r["counts_raw"], plain["counts_raw"])
        scale = np.abs(plain["raw"]).max()
        assert np.abs(r["raw"] - plain["raw"]).max() <= 1e-12 * scale
        assert np.allclose(r["moments"], plain["moments"], rtol=1e-12, atol=1e-12 * np.abs(plain["moments"]).max())
    assert plain["counts"]["periodic"] > 20 * 300


@pytest.mark.parametrize("cap", [1, 7, 20])
def test_event_cap_fp64_bit_exact_and_in_the_lone_lane_walk(cap):
    """The per-particle segment cap ends a walk where the oracle ends it: FP64 event sequences and
    counters bit-exact (pore cell with long free paths, film), and the lone-lane walk, which
    checks the cap before every segment, gives the one-segment step's counters."""
    M = _pkg()
    long_pores = W.with_(W.porous_cell(N=300, modes=W.gray_modes(6400.0, 20e-6 / 6400.0), n_scat_max=3),
                         **{"problem.format": 2, "problem.max_events": cap})
    film = W.with_(W.film(N=500), **{"problem.max_events": cap})
    for w in (long_pores, film):
        n = w["problem"]["N"]
        got = M.run(w, precision=64, n_log=n, log_stride=64)
        ref = oracle.trace(w, n_log=n, log_stride=64, threads=THREADS)
        assert _first_log_mismatch(got["log"], ref["log"]) is None
        assert np.array_equal(got["counts_raw"], ref["counts"])
        assert got["counts"]["cap_end"] > 0
        assert got["counts"]["flights"] <= cap * n
    plain = M.run(long_pores, precision=64)
    logged = M.run(long_pores, precision=64, n_log=300, log_stride=16)
    assert np.array_equal(plain["counts_raw"], logged["counts_raw"])


@pytest.mark.parametrize("name", ["transient_bump", "transient_uneven_times"])
def test_fp32_transient_wide_kernel_against_fp64_oracle(name):
    """The transient bump with its full snapshot detector (100 bins x 200 times, too large for a
    per-workgroup FP64 copy): the FP32 kernel sums it per workgroup in FP32 in LDS.  Each particle
    adds its sign once per measurement time, so the total of every snapshot equals the oracle's
    exactly, and every cell agrees within two particles moved to a neighbouring bin by FP32
    rounding (a particle adds s to T and s v Omega_z to q_z of one bin per time).  Also on uneven
    measurement times (clusters, repeats, log spacing), where a segment's snapshot range comes
    from the guided search of the times."""
    M = _pkg()
    w = W.transient_bump(N=20000) if name == "transient_bump" else W.with_(FP64_CASES[name](), **{"problem.N": 20000})
    got = M.run(w, precision=32)
    ref = _oracle_full(w)
    rg = np.asarray(got["raw"])
    rr = np.asarray(ref["raw"]).reshape(rg.shape)          # (bins, times, components)
    Tg, Tr = rg[..., 0], rr[..., 0]
    qg, qr = rg[..., 3], rr[..., 3]
    _say(f"[transient fp32] max |dT| {np.abs(Tg - Tr).max():.3g} of {np.abs(Tr).max():.3g}; "
         f"max |dq| {np.abs(qg - qr).max():.3g} of {np.abs(qr).max():.3g}")
    assert got["counts"]["particles"] == ref["counts"]["particles"]
    assert np.array_equal(Tg.sum(axis=0), Tr.sum(axis=0))
    vmax = float(np.max(w["modes"]["v"]))
    assert np.abs(Tg - Tr).max() <= 4.0
    assert np.abs(qg - qr).max() <= 4.0 * vmax


def test_fp64_parity_across_the_2_32_particle_id():
    """Particle ids past 2^32 use the second counter word of every Philox draw: a range crossing
    that boundary gives the oracle's event sequences bit for bit."""
    M = _pkg()
    first = (1 << 32) - 100
    for w in (W.film(N=200), W.porous_cell(N=200)):
        got = M.run(w, n=200, first_pid=first, precision=64, n_log=200, log_stride=96)
        ref = oracle.trace(w, n=200, first_pid=first, n_log=200, log_stride=96, threads=THREADS)
        assert _first_log_mismatch(got["log"], ref["log"]) is None
        assert np.array_equal(got["counts_raw"], ref["counts"])
        # and the two halves are different particles: ids below and above 2^32 do not repeat
        low = M.run(w, n=100, first_pid=first, precision=64)
        high = M.run(w, n=100, first_pid=first + 100, precision=64)
        assert not np.array_equal(low["raw"], high["raw"])


@pytest.mark.parametrize("n", [0, 1, 63, 65, 257])
def test_fp64_ragged_and_empty_ranges(n):
    """Empty, single-particle and wave-ragged launches: counts equal the oracle's exactly (an
    empty launch leaves the tally untouched)."""
    M = _pkg()
    w = W.film(N=max(n, 1))
    got = M.run(w, n=n, precision=64, block=64, refill=1)
    if n == 0:
        assert got["counts"]["particles"] == 0 and not np.any(got["raw"])
        return
    ref = oracle.trace(w, n=n, threads=1)
    assert np.array_equal(got["counts_raw"], ref["counts"])
    assert np.abs(got["raw"] - ref["raw"].reshape(got["raw"].shape)).max() <= 1e-10 * np.abs(ref["raw"]).max()


def test_batched_launch_with_an_empty_instance():
    """An instance with no particles inside a batch contributes nothing and disturbs no other."""
    import torch
    M = _pkg()
    counts = (5000, 0, 7000)
    ws = [W.film(N=max(n, 1), d=d) for n, d in zip(counts, (2e-8, 1e-7, 5e-7))]
    for i, w in enumerate(ws):
        w["instance"] = 11 + i
    tabs = [M.Tables(w) for w in ws]
    tallies = [t.new_tally() for t in tabs]
    queue = torch.zeros(M.batch_queue_bytes(len(ws)), dtype=torch.uint8, device="cuda")
    M.trace_batch(tabs, list(counts), [w["instance"] for w in ws], tallies, M.make_run(int(ws[0]["seed"]), 64), queue)
    for n, w, t, tl in zip(counts, ws, tabs, tallies):
        b = M.tally(t, tl)
        if n == 0:
            assert b["counts"]["particles"] == 0 and not np.any(t.raw(tl))
            continue
        s = M.run(w, precision=64, tables=t)
        assert np.array_equal(b["counts_raw"], s["counts_raw"])
