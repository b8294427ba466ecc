"""The extended physics on the HIP path, through the C ABI: separate two-phonon and
three-phonon clocks (section 3.3), frequency-dependent specularity (section 3.5.3) and internal
line walls (section 4.2).

The FP64 event sequences of such workloads are compared bit-exactly with the oracle in
test_gpu_parity.py (FP64_CASES); this file covers the emitted clocks, the state-buffer path,
the batched kernel, launch shapes that route walks through the lone-lane and wave-cooperative
paths, and the FP32 form against the FP64 oracle.
"""
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


def _two_film(N, **kw):
    return W.film(N=N, modes=W.silicon_like_modes(300.0, impurity_clock=True), **kw)


def _lead(buf, precision, cap):
    """The clocks' lead array of a state buffer (after the real and integer arrays)."""
    b = buf.cpu().numpy()
    rb = precision // 8
    fb = (cap * rb + 255) // 256 * 256
    ib = (cap * 4 + 255) // 256 * 256
    off = 8 * fb + 7 * ib
    return np.frombuffer(b[off:off + cap * rb].tobytes(), dtype=np.float64 if precision == 64 else np.float32)


@pytest.mark.parametrize("precision", [64, 32])
def test_emitted_clocks_match_oracle(precision):
    """Which clock fires first agrees exactly; the lead agrees to the rounding of two logarithms
    (FP64) or of the FP32 form."""
    import torch
    M = _pkg()
    w = _two_film(2000)
    n = 2000
    t = M.Tables(w)
    o = oracle.Tables(w)
    buf = torch.zeros(M.state_bytes(precision, n), dtype=torch.uint8, device="cuda")
    M.emit(t, M.make_run(int(w["seed"]), precision), 0, n, buf, n)
    torch.cuda.synchronize()
    lead = _lead(buf, precision, n).astype(np.float64)
    ref = np.array([o.emit_clocks(k) for k in range(n)])
    first = np.array([o.emit_state(k)[0][7] for k in range(n)])     # the earlier clock
    nx2 = np.signbit(lead).astype(int)
    assert np.array_equal(nx2, ref[:, 1].astype(int))
    assert 0 < nx2.sum() < n
    assert np.all(np.isfinite(ref[:, 0])) and np.all(np.isfinite(lead))
    # the lead is a difference of the two times: its error is bounded by theirs, i.e. by the
    # later time's rounding (FP64: device and host logarithms within 2 ulp each)
    later = first + ref[:, 0]
    err = np.abs(np.abs(lead) - ref[:, 0])
    if precision == 64:
        assert np.all(err <= 4 * np.spacing(later)), (err / later).max()
    else:
        # FP32 form: single-precision logarithm, whose relative error grows for arguments
        # near 1 (short times), as for the free flights of the emission test
        rel = err / later
        assert np.median(rel) < 2e-6 and rel.max() < 1e-2, (np.median(rel), rel.max())


@pytest.mark.parametrize("precision", [64, 32])
def test_emit_then_trace_equals_fused(precision):
    M = _pkg()
    w = _two_film(4000)
    fused = M.run(w, precision=precision, n_log=300, log_stride=64)
    staged = M.run(w, precision=precision, n_log=300, log_stride=64, emit_first=True)
    assert np.array_equal(fused["counts_raw"], staged["counts_raw"])
    assert fused["counts"]["two_phonon"] > 0
    assert np.array_equal(fused["log"], staged["log"])
    scale = np.abs(fused["raw"]).max()
    assert np.abs(fused["raw"] - staged["raw"]).max() <= 1e-12 * scale


def test_batched_launch_with_two_clock_instances_equals_solo_runs():
    """The batched kernel with the two-clock code (some instance has a two-phonon process) next
    to a single-clock instance."""
    import torch
    M = _pkg()
    ws = [_two_film(6000, d=2e-8), W.film(N=3000, d=1e-7, T=100.0), _two_film(9000, d=5e-7, T=400.0)]
    for i, w in enumerate(ws):
        w["instance"] = 3 + i
    for prec in (64, 32):
        tabs = [M.Tables(w) for w in ws]
        tallies = [t.new_tally() for t in tabs]
        queue = torch.zeros(M.batch_queue_bytes(len(ws)), dtype=torch.uint8, device="cuda")
        run = M.make_run(int(ws[0]["seed"]), prec)
        M.trace_batch(tabs, [w["problem"]["N"] for w in ws], [w["instance"] for w in ws], tallies, run, queue)
        for w, t, tl in zip(ws, tabs, tallies):
            b = M.tally(t, tl)
            s = M.run(w, precision=prec, tables=t)
            assert np.array_equal(b["counts_raw"], s["counts_raw"]), (prec, b["counts"], s["counts"])
            assert np.abs(t.raw(tl) - s["raw"]).max() <= 1e-12 * np.abs(s["raw"]).max()


@pytest.mark.parametrize("name", ["film", "porous"])
def test_launch_shapes_route_two_clock_walks_through_every_path(name):
    """One-wave grids leave lanes walking alone (lone-lane walk) and the film's long flights go
    to the wave-cooperative bouncing; every shape gives the same FP64 counters and sums."""
    M = _pkg()
    w = _two_film(6000, d=40e-9) if name == "film" else \
        W.porous_cell(N=1500, modes=W.silicon_like_modes(300.0, impurity_clock=True))
    base = M.run(w, precision=64)
    assert base["counts"]["two_phonon"] > 0
    for block, refill, grid in ((64, 1, 1), (64, 8, 3), (256, 32, 0)):
        r = M.run(w, precision=64, block=block, refill=refill, grid=grid)
        assert np.array_equal(r["counts_raw"], base["counts_raw"]), (block, refill, grid)
        assert np.abs(r["raw"] - base["raw"]).max() <= 1e-12 * np.abs(base["raw"]).max()


def test_fp32_two_clock_film_against_fp64_oracle():
    """FP32 trajectories with both clocks against the FP64 oracle on the same particles: kappa
    and the flux within 2e-4 relative, event counts within 1e-3."""
    M = _pkg()
    w = _two_film(100000)
    got = M.run(w, precision=32)
    ref = oracle.run(w, threads=THREADS)
    rel_k = abs(got["kappa"] - ref["kappa"]) / abs(ref["kappa"])
    c, rc = got["counts"], ref["counts"]
    _say(f"[fp32 two clocks] kappa {got['kappa']:.6g} vs {ref['kappa']:.6g} (rel {rel_k:.2e}); "
         f"two-phonon {c['two_phonon']} vs {rc['two_phonon']}, relaxations {c['relaxations']} vs {rc['relaxations']}")
    assert c["particles"] == rc["particles"]
    assert rel_k < 2e-4
    for k in ("flights", "two_phonon", "relaxations", "diffuse"):
        assert abs(c[k] - rc[k]) <= 1e-3 * rc[k], k


def test_specular_cutoff_launch_shapes_batched_kernel_and_fp32():
    """Pore cell with the phonons below 2 THz specular: launch shapes that leave lanes walking
    alone (whose pore reflections then take each phonon's own class) give the same FP64 counters
    and sums; the batched kernel with the extended code equals solo runs; the FP32 film with a
    cutoff agrees with the FP64 oracle."""
    import torch
    M = _pkg()
    w = W.porous_cell(N=1500, spec_omega=W.OMEGA_2THZ)
    base = M.run(w, precision=64)
    assert base["counts"]["specular"] > 0 and base["counts"]["diffuse"] > 0
    for block, refill, grid in ((64, 1, 1), (64, 8, 3)):
        r = M.run(w, precision=64, block=block, refill=refill, grid=grid)
        assert np.array_equal(r["counts_raw"], base["counts_raw"]), (block, refill, grid)
        assert np.abs(r["raw"] - base["raw"]).max() <= 1e-12 * np.abs(base["raw"]).max()
    ws = [W.film(N=5000, d=3e-8, spec_omega=2.5 * W.OMEGA_2THZ), W.film(N=4000, d=1e-7)]
    for i, wi in enumerate(ws):
        wi["instance"] = 11 + i
    tabs = [M.Tables(wi) for wi in ws]
    tallies = [t.new_tally() for t in tabs]
    queue = torch.zeros(M.batch_queue_bytes(len(ws)), dtype=torch.uint8, device="cuda")
    run = M.make_run(int(ws[0]["seed"]), 64)
    M.trace_batch(tabs, [wi["problem"]["N"] for wi in ws], [wi["instance"] for wi in ws], tallies, run, queue)
    for wi, t, tl in zip(ws, tabs, tallies):
        b = M.tally(t, tl)
        s = M.run(wi, precision=64, tables=t)
        assert np.array_equal(b["counts_raw"], s["counts_raw"])
    wf = W.film(N=100000, spec_omega=2.5 * W.OMEGA_2THZ)
    got = M.run(wf, precision=32)
    ref = oracle.run(wf, threads=THREADS)
    rel_k = abs(got["kappa"] - ref["kappa"]) / abs(ref["kappa"])
    _say(f"[fp32 cutoff film] kappa {got['kappa']:.6g} vs {ref['kappa']:.6g} (rel {rel_k:.2e})")
    assert rel_k < 2e-4
    for k in ("flights", "specular", "diffuse"):
        assert abs(got["counts"][k] - ref["counts"][k]) <= 1e-3 * ref["counts"][k], k


def test_line_walls_launch_shapes_batched_kernel_and_fp32():
    """Square pore of four walls: launch shapes (one-wave grids included) give the same FP64
    counters and sums; a batch mixing a walled and a plain instance equals solo runs; the FP32
    channel between two walls agrees with the FP64 oracle."""
    import torch
    M = _pkg()
    w = W.square_pore_cell(N=1500)
    base = M.run(w, precision=64)
    assert base["counts"]["diffuse"] > 0 and base["counts"]["rejections"] > 0
    for block, refill, grid in ((64, 1, 1), (64, 8, 3), (256, 32, 0)):
        r = M.run(w, precision=64, block=block, refill=refill, grid=grid)
        assert np.array_equal(r["counts_raw"], base["counts_raw"]), (block, refill, grid)
        assert np.abs(r["raw"] - base["raw"]).max() <= 1e-12 * np.abs(base["raw"]).max()
    ws = [W.square_pore_cell(N=3000), W.porous_cell(N=3000)]
    for i, wi in enumerate(ws):
        wi["instance"] = 21 + i
        wi["seed"] = ws[0]["seed"]          # one launch, one key
    tabs = [M.Tables(wi) for wi in ws]
    tallies = [t.new_tally() for t in tabs]
    queue = torch.zeros(M.batch_queue_bytes(len(ws)), dtype=torch.uint8, device="cuda")
    run = M.make_run(int(ws[0]["seed"]), 64)
    M.trace_batch(tabs, [wi["problem"]["N"] for wi in ws], [wi["instance"] for wi in ws], tallies, run, queue)
    for wi, t, tl in zip(ws, tabs, tallies):
        b = M.tally(t, tl)
        s = M.run(wi, precision=64, tables=t)
        assert np.array_equal(b["counts_raw"], s["counts_raw"])
    wf = W.walled_film(N=100000)
    got = M.run(wf, precision=32)
    ref = oracle.run(wf, threads=THREADS)
    rel_k = abs(got["kappa"] - ref["kappa"]) / abs(ref["kappa"])
    _say(f"[fp32 walled film] kappa {got['kappa']:.6g} vs {ref['kappa']:.6g} (rel {rel_k:.2e})")
    assert rel_k < 2e-4
    for k in ("flights", "diffuse", "periodic"):
        assert abs(got["counts"][k] - ref["counts"][k]) <= 1e-3 * ref["counts"][k], k


def test_paper_format_case_runs_through_the_library(tmp_path):
    """The paper's nanomesh example files (a 34-nm cell, 22 nm thick, an 11-nm square pore of
    four line walls) traced on the GPU through the file front end: the output files hold the
    library's result for the case, and the FP64 counters equal the oracle's."""
    from paper_2104_03573_amd import paper_io as P
    (tmp_path / "Out_bnd.txt").write_text("34e-9 34e-9 22e-9\n")
    (tmp_path / "In_bnd.txt").write_text("11.5e-9 11.5e-9 22.5e-9 11.5e-9 0 -1 0\n"
                                         "22.5e-9 11.5e-9 22.5e-9 22.5e-9 1 0 0\n"
                                         "22.5e-9 22.5e-9 11.5e-9 22.5e-9 0 1 0\n"
                                         "11.5e-9 22.5e-9 11.5e-9 11.5e-9 -1 0 0\n")
    (tmp_path / "Boundary_prop.txt").write_text(
        "1 3 0 34e-9 0\n2 3 -34e-9 0 0\n3 3 0 -34e-9 0\n4 3 34e-9 0 0\n5 2 0 0 0\n6 2 0 0 0\n"
        "7 2 0 0 0\n8 2 0 0 0\n9 2 0 0 0\n10 2 0 0 0\n")
    (tmp_path / "Thermal_gradient.txt").write_text("1 3 0 -2.94e6 0\n")
    (tmp_path / "Sim_param.txt").write_text("2000 10 2.28e-23 300\n")
    (tmp_path / "mat_data.txt").write_text("1e13 6400 1.5625e-11 1e6\n")
    (tmp_path / "Measure_region.txt").write_text("0 34e-9 0 34e-9 0 22e-9 1\n")
    res = P.run_case(str(tmp_path), fmt=2, precision=64)
    qy = np.loadtxt(tmp_path / "Qy300.txt")
    assert qy.shape == (8,) and np.allclose(qy, res["q"][:, 0, 1])
    w = P.read_case(str(tmp_path), fmt=2)
    ref = oracle.trace(w, threads=THREADS)
    assert np.array_equal(res["counts_raw"], ref["counts"])
