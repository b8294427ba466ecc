"""The FP32 form's error per detector, measured against FP64.

The transient bump's snapshot detector (100 bins x 200 times x T, q_z) is too large for a
per-workgroup FP64 copy in LDS.  The default FP32 launch keeps an FP32 copy per workgroup and folds
it into the FP64 sums once; a launch with a state buffer sums every snapshot straight into the FP64
buffer with FP64 atomics.  Both trace the same FP32 trajectories, so their difference is the error
of the FP32 partial sums alone.  Against the FP64 oracle the error also holds FP32 trajectory
rounding (a particle near a bin edge lands in the neighbour).  Both are measured at full size and
stated relative to the largest bin and to the bins' statistical standard errors.
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


def test_fp32_partial_sums_of_the_transient_detector_against_fp64_accumulation():
    """1e7 particles: the same FP32 trajectories summed through FP32 workgroup copies and through
    FP64 atomics.  Counters equal; T is a sum of signs, exact in both; q_z differs by the FP32
    partial sums' rounding only (measured bound below, far under the bins' statistical error)."""
    M = _pkg()
    w = W.transient_bump(N=10_000_000)
    wide = M.run(w, precision=32)
    full = M.run(w, precision=32, emit_first=True)
    assert np.array_equal(wide["counts_raw"], full["counts_raw"])
    rw, rf = np.asarray(wide["raw"]), np.asarray(full["raw"])
    assert np.array_equal(rw[..., 0], rf[..., 0])
    dq = np.abs(rw[..., 3] - rf[..., 3])
    scale = np.abs(rf[..., 3]).max()
    vmax = float(np.max(w["modes"]["v"]))
    # a bin's statistical standard error of sum s v Omega_z: about v_rms sqrt(particles in the bin)
    n_bin = np.abs(rf[..., 0]) + 1.0
    rel_sigma = (dq / (vmax * np.sqrt(n_bin))).max()
    _say(f"[FP32 partial sums, transient 1e7] q_z: max |d| {dq.max():.3g} = {dq.max() / scale:.2e} of the "
         f"largest bin, {rel_sigma:.2e} of a bin's statistical error (v_max sqrt(n))")
    assert dq.max() <= 1e-6 * scale
    assert rel_sigma <= 1e-5


@pytest.mark.parametrize("name", ["transient_bump", "heated_slab", "heated_box"])
def test_fp32_transient_per_detector_error_against_the_oracle(name):
    """A 1e6-particle prefix in 8 groups: per bin and time, the FP32 launch against the FP64 oracle
    on the same particles, T and q_z, stated relative to the largest bin and to each bin's batch
    standard error.  Every snapshot's total over the bins is exact (a particle's sign counts once
    per time) and the bins agree far inside their statistical errors.  The transient bump starts
    from its initial condition; the heated slab is heated by a 5 ps pulse in its top 20 nm; the
    heated box by a 10 ps pulse in a tetrahedron."""
    M = _pkg()
    w = {"transient_bump": W.transient_bump, "heated_slab": W.heated_slab,
         "heated_box": W.heated_box}[name](N=1_000_000)
    t = M.Tables(w)
    n, G = w["problem"]["N"], 8
    bounds = [(n * i) // G for i in range(G + 1)]
    tallies = []
    for lo, hi in zip(bounds[:-1], bounds[1:]):
        tl = t.new_tally()
        M.trace(t, M.make_run(int(w["seed"]), 32), lo, hi - lo, None, tl)
        tallies.append(tl)
    got = M.tally_batches(t, tallies)
    ref = oracle.batch_statistics(oracle.run_batches(w, G, threads=THREADS))
    Tg, Tr, Ts = got["T"], ref["mean"][..., 0], ref["sigma"][..., 0]
    qg, qr, qs = got["q"][..., 2], ref["mean"][..., 3], ref["sigma"][..., 3]
    out = {}
    for comp, g, r, s in (("T", Tg, Tr, Ts), ("q_z", qg, qr, qs)):
        d = np.abs(g - r)
        ok = s > 0
        out[comp] = (d.max() / np.abs(r).max(), np.median(d[ok] / s[ok]), (d[ok] / s[ok]).max())
        _say(f"[FP32 vs oracle, {name} 1e6] {comp}: max |d| {out[comp][0]:.2e} of the largest bin; "
             f"|d| / batch sigma median {out[comp][1]:.2e}, max {out[comp][2]:.2e}")
    assert np.allclose(Tg.sum(axis=0), Tr.sum(axis=0), rtol=1e-12, atol=1e-12 * np.abs(Tr).max())
    assert out["T"][0] <= 1e-3 and out["q_z"][0] <= 1e-2
    assert out["T"][1] <= 0.05 and out["q_z"][1] <= 0.05
