"""Parity of the launches that earlier tests compared only with other launches of the HIP path,
now against the CPU oracle directly, through the C ABI:

  - the batched persistent launch (one launch over many instances) against the oracle's trace of
    every instance: integer counters bit-exact and FP64 sums to rounding (FP64), kappa per
    instance (FP32);
  - the plain FP64 trace kernel (no event log, the one that is timed) against the oracle's counts
    at the default launch and at a two-workgroup grid of 64-lane blocks, where every lane refills
    many times;
  - the FP32 pore cell on a 1e6-particle prefix against the oracle, at the measured bound;
  - the sensitivity estimators against common-random-number finite differences per frequency bin
    at dtau / tau = 1e-3 and 0.05 (section 3.3, Eq. time_to_scat).
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


def _sweep(scale):
    """The batched sweep's 16 thicknesses x 4 temperatures with particle counts scaled down."""
    return W.film_sweep(scale=scale)


def _batch(M, ws, precision):
    import torch
    tabs = [M.Tables(w) for w in ws]
    tallies = [t.new_tally() for t in tabs]
    queue = torch.zeros(M.batch_queue_bytes(len(ws)), dtype=torch.uint8, device="cuda")
    run = M.make_run(int(ws[0]["seed"]), precision)
    M.trace_batch(tabs, [w["problem"]["N"] for w in ws], [w["instance"] for w in ws], tallies, run, queue)
    return [(M.tally(t, tl), t.raw(tl)) for t, tl in zip(tabs, tallies)]


def test_batched_sweep_fp64_against_oracle_per_instance():
    """All 64 instances of the sweep (16 thicknesses 10 nm - 10 um x 4 temperatures) with 1e-3 of
    their particle counts (100 - 4000, uneven) in one FP64 batched launch: every instance's integer
    counters equal the oracle's trace of that instance (its own tables and Philox instance word),
    raw sums to 1e-10 of the largest."""
    M = _pkg()
    ws = _sweep(1e-3)
    got = _batch(M, ws, 64)
    worst = 0.0
    for w, (r, raw) in zip(ws, got):
        ref = oracle.trace(w, threads=THREADS)
        assert np.array_equal(r["counts_raw"], ref["counts"]), (w["name"], r["counts"])
        rr = ref["raw"].reshape(raw.shape)
        err = np.abs(raw - rr).max() / np.abs(rr).max()
        worst = max(worst, err)
        assert err <= 1e-10, (w["name"], err)
    _say(f"[batched vs oracle] 64 instances, {sum(w['problem']['N'] for w in ws)} particles, worst raw err {worst:.2e}")


def test_batched_fp32_kappa_per_instance_against_oracle():
    """FP32 batched launch over 16 instances of 1e5 - 2e5 particles (10 nm - 10 um films at 100 -
    400 K): each instance's kappa against the FP64 oracle on the same particles within 1e-4, except
    the thinnest, coldest films, whose long free paths make hundreds of wall bounces per flight (the
    FP32 sum of the bounces' chords then ends a flight on another bounce than the FP64 recursion for
    a few particles): there within a tenth of the statistical error (measured: 3.5e-3 at 10 nm,
    100 K, where sigma is 5.7e-2; 1.5e-4 at 10 nm, 200 K; the rest 2e-7 - 9e-5)."""
    M = _pkg()
    ws = [w for w in _sweep(1.0) if w["instance"] % 16 in (0, 5, 10, 15)]
    for w in ws:
        w["problem"]["N"] = min(w["problem"]["N"], 200_000)
    got = _batch(M, ws, 32)
    for w, (r, _) in zip(ws, got):
        ref = oracle.run(w, threads=THREADS)
        rel = abs(r["kappa"] - ref["kappa"]) / abs(ref["kappa"])
        srel = ref["kappa_sigma"] / abs(ref["kappa"])
        _say(f"[batched fp32] {w['name']}: kappa {r['kappa']:.6g} vs {ref['kappa']:.6g} rel {rel:.2e} "
             f"(sigma_rel {srel:.1e})")
        assert r["counts"]["particles"] == w["problem"]["N"]
        thin_cold = w["geometry"]["L"][2] < 2e-8 and w["problem"]["T_lin"] <= 200.0
        assert rel < (0.1 * srel if thin_cold else 1e-4), w["name"]


def _fp64_cases():
    from test_gpu_parity import FP64_CASES
    return FP64_CASES


@pytest.mark.parametrize("shape", [{}, {"block": 64, "grid": 2, "refill": 1}], ids=["default", "grid2_block64"])
@pytest.mark.parametrize("name", list(_fp64_cases()))
def test_plain_fp64_kernel_counts_equal_oracle(name, shape):
    """The FP64 trace kernel without the event log (the timed one: lone-lane walks, cooperative
    film bouncing, wave-wide grid scoring compiled in) against the oracle: every integer counter
    equal, raw sums to 1e-10 of the largest, at the default launch and at two workgroups of 64
    lanes (each lane then takes dozens of particles, refilling after every flight)."""
    M = _pkg()
    w = _fp64_cases()[name]()
    got = M.run(w, precision=64, **shape)
    ref = oracle.trace(w, threads=THREADS)
    assert np.array_equal(got["counts_raw"], ref["counts"]), (got["counts"], ref["counts"])
    rr = ref["raw"].reshape(got["raw"].shape)
    assert np.abs(got["raw"] - rr).max() <= 1e-10 * np.abs(rr).max()


def test_porous_cell_fp32_prefix_against_oracle():
    """The pore cell's first 1e6 particles, FP32 (the pore-to-pore walk on), against the FP64 oracle
    on the same particles.  The lattice is a dispersing billiard: a flight's FP32 rounding grows by
    about its length over the pore radius at each reflection, so the long-free-path particles, which
    carry much of kappa, take other paths than the oracle's after some reflections and the FP32
    estimate is, for them, another sample.  Measured: kappa 2.7e-3 - 4.2e-3 (standard error 4.6e-3);
    event counts 1e-5 - 1.6e-4; the flux of the modes with mean free paths below 1 um (89 % of
    kappa) within 1.3e-4 of the total, of those between 1 and 10 um (10 %) within 3.1e-3, longer ones
    5e-4; a single mode's flux up to half the largest mode's (a mode carried by a few particles of
    long channel flights).  Bounds at those values with some room."""
    M = _pkg()
    w = W.porous_cell(N=1_000_000)
    got = M.run(w, precision=32)
    ref = oracle.run(w, threads=THREADS)
    c, r = got["counts"], ref["counts"]
    rel_k = abs(got["kappa"] - ref["kappa"]) / abs(ref["kappa"])
    qg, qr = got["q"][0, :, 1], ref["q"][0, :, 1]
    per_mode = np.abs(qg - qr).max() / np.abs(qr).max()
    t_rel = abs(got["T"].sum() - ref["T"].sum()) / abs(ref["T"].sum())
    _say(f"[pore cell fp32 1e6] kappa {got['kappa']:.6f} vs {ref['kappa']:.6f} rel {rel_k:.2e} (sigma_rel "
         f"{ref['kappa_sigma'] / abs(ref['kappa']):.2e}); per-mode q_y {per_mode:.2e}; T sum {t_rel:.2e}; "
         f"flights {c['flights']} / {r['flights']}, periodic {c['periodic']} / {r['periodic']}")
    for k in ("particles", "rejections"):
        assert c[k] == r[k], k
    for k in ("flights", "periodic", "diffuse", "relaxations"):
        assert abs(c[k] - r[k]) <= 1e-3 * r[k], k
    assert rel_k < 6e-3
    assert t_rel < 1.5e-2
    lam = w["modes"]["v"] * w["modes"]["tau"]
    tot = qr.sum()
    for lo, hi, bound in ((0.0, 1e-6, 5e-4), (1e-6, 1e-5, 6e-3), (1e-5, 1.0, 2e-3)):
        sel = (lam >= lo) & (lam < hi)
        err = abs(qg[sel].sum() - qr[sel].sum()) / abs(tot)
        _say(f"   modes with mean free path in [{lo:.0e}, {hi:.0e}): flux share {qr[sel].sum() / tot:.3f}, "
             f"error {err:.2e} of the total")
        assert err < bound, (lo, hi)
    assert per_mode < 1.0


def _bins_spread_over_mfp(w, t, n_pick):
    """n_pick frequency bins spread over the mean free path: of the bins that carry 95 % of the bulk
    kappa (sum over the bin's rows of C v^2 tau / 3), evenly spaced in the order of their LA row's
    mean free path."""
    M = _pkg()
    C = M.table_export(t, "C")
    m = w["modes"]
    nb = int(m["bin"].max()) + 1
    kb = np.zeros(nb)
    lam = np.zeros(nb)
    np.add.at(kb, m["bin"], C * m["v"] ** 2 * m["tau"] / 3.0)
    for i in range(len(m)):
        if m["branch"][i] == 0:
            lam[m["bin"][i]] = m["v"][i] * m["tau"][i]
    order = np.argsort(-kb)
    keep = order[: int(np.searchsorted(np.cumsum(kb[order]) / kb.sum(), 0.95)) + 1]
    keep = keep[np.argsort(lam[keep])]
    return [int(keep[int(round(k * (len(keep) - 1) / (n_pick - 1)))]) for k in range(n_pick)]


@pytest.mark.parametrize("d,n_per", [(1e-3, 1_000_000), (0.05, 10_000_000)])
def test_crn_finite_differences_per_bin(d, n_per):
    """The pore cell: for 16 single frequency bins spread over the mean free path, central
    differences (kappa(tau_i (1 + d)) - kappa(tau_i (1 - d))) / 2d with common random numbers,
    against the sensitivity estimates dkappa/dln tau_i (local pathwise and score function) on the
    same particles, 16 batches.  The error of an estimate minus the difference is
    taken from their paired per-batch values (both come from the same particles, so they are
    correlated); each bin must agree within 4.5 of those standard errors (Student t, 15 degrees of
    freedom).
    At d = 1e-3 the differences do not resolve single bins: changing a flight by 1e-3 of its length
    moves its next pore hit, and in the lattice (a dispersing billiard) the trajectory after it parts
    from the unperturbed one, so each affected particle contributes its whole score difference
    divided by 2d (measured with 1e6 particles per batch: standard errors 0.02 - 1.8 W/m/K against
    sensitivities 0.02 - 0.12).  At d = 0.05 that noise is some 20 times smaller; with 1e7 particles
    per batch the differences must resolve at least a quarter of the bins (the central difference's
    O(d^2) bias stays far below the error)."""
    M = _pkg()
    base = W.porous_cell(N=n_per)
    t0 = M.Tables(base)
    bins = _bins_spread_over_mfp(base, t0, 16)
    B = 16
    pert = []
    for i in bins:
        sel = base["modes"]["bin"] == i
        wp, wm = W.with_(base), W.with_(base)
        wp["modes"]["tau"][sel] *= 1.0 + d
        wm["modes"]["tau"][sel] *= 1.0 - d
        pert.append((M.Tables(wp), M.Tables(wm)))
    ests = {"local": np.zeros((B, len(bins))), "score": np.zeros((B, len(bins)))}
    fd = np.zeros((B, len(bins)))
    for b in range(B):
        w = W.with_(base, **{"seed": int(base["seed"]) + 7919 * (b + 1)})
        for e in ests:
            ests[e][b] = M.sensitivities(w, precision=32, tables=t0, estimator=e)["dkappa_dlntau"][bins]
        for k, (tp, tm) in enumerate(pert):
            fd[b, k] = (M.run(w, precision=32, tables=tp)["kappa"] - M.run(w, precision=32, tables=tm)["kappa"]) / (2 * d)
    se_fd = fd.std(0, ddof=1) / math.sqrt(B)
    resolved = int(np.sum(np.abs(fd.mean(0)) > 3.0 * se_fd))
    _say(f"[CRN FD d={d:g}] bins {bins}; FD resolves {resolved} of {len(bins)} bins")
    _say(f"   FD       {np.round(fd.mean(0), 4)}  (se {np.round(se_fd, 4)})")
    for e, est in ests.items():
        diff = est - fd
        se = diff.std(0, ddof=1) / math.sqrt(B)
        z = diff.mean(0) / np.where(se > 0, se, 1.0)
        _say(f"   {e:6s} {np.round(est.mean(0), 4)}  paired se {np.round(se, 4)}  z {np.round(z, 2)}")
        assert np.all(np.abs(z) < 4.5), e
    if d >= 0.01:
        assert resolved >= len(bins) // 4
