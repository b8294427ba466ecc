"""Pins of the oracle's cumulative thermal conductivity (the per-row steady flux output of section
4.5, accumulated over mean free path or frequency as in section 5.6) and of its batch-mean
standard errors.

The in-plane film with diffuse walls has a closed form per row: Fuchs-Sondheimer's suppression
S(d / Lambda_i) of the row's bulk conductivity C_i v_i^2 tau_i / 3, independent of the other rows
(rows couple only through relaxation, which the deviational gradient source leaves at
equilibrium).  Prefix sums of those closed forms in ascending Lambda (or frequency) are the
cumulative curves; the oracle's must lie within a few batch standard errors of them at every
decile.  A wrong order key, a transposed flux component or a dropped row moves the curve by many
standard errors.  The standard error itself is pinned by an identity: groups of one particle each
give the batch-mean error of the particle scores, which the oracle also accumulates as moments.
"""
import math
import os

import numpy as np

import closed_forms as cf
import oracle
import workloads as W

THREADS = min(8, os.cpu_count() or 1)


def _fs_rows(w, tb, d):
    C = tb.get("C")
    m = w["modes"]
    lam = m["v"] * m["tau"]
    return lam, np.array([C[i] * m["v"][i] ** 2 * m["tau"][i] / 3.0 * cf.fs_suppression(d / lam[i])
                          for i in range(len(m))])


def _check_deciles(cum, sig, ref, n_sigma=3.5):
    worst = 0.0
    for q in (0.1, 0.2, 0.3, 0.4, 0.5, 0.6, 0.7, 0.8, 0.9):
        k = min(int(np.searchsorted(ref, q * ref[-1])), len(ref) - 1)
        z = (cum[k] - ref[k]) / sig[k]
        worst = max(worst, abs(z))
        assert abs(z) < n_sigma, (q, k, cum[k], ref[k], sig[k])
    return worst


def test_film_cumulative_kappa_over_mean_free_path_matches_fuchs_sondheimer_prefix_sums():
    """100 nm film of the silicon-like crystal, 2e6 particles in 16 groups: the cumulative curve
    in ascending v tau equals the prefix sums of the rows' Fuchs-Sondheimer conductivities at
    every decile (3.5 batch standard errors); the keys ascend; the last entry is kappa."""
    d = 100e-9
    w = W.film(N=2_000_000, d=d, n_scat_max=10)
    b = oracle.run_batches(w, 16, threads=THREADS)
    c = oracle.kappa_cumulative(b, "mfp")
    lam, k_fs = _fs_rows(w, b[0]["tables"], d)
    idx = np.argsort(lam, kind="stable")
    ref = np.cumsum(k_fs[idx])
    assert np.all(np.diff(c["keys"]) >= 0.0)
    assert np.array_equal(c["keys"], lam[idx])
    _check_deciles(c["kappa_cum"], c["kappa_cum_sigma"], ref)
    whole = oracle.run(w, threads=THREADS)
    assert abs(c["kappa_cum"][-1] - whole["kappa"]) <= 1e-12 * abs(whole["kappa"])
    # the batch error of the total and the moment error of kappa estimate the same quantity
    assert 0.5 < c["kappa_cum_sigma"][-1] / whole["kappa_sigma"] < 1.6


def test_film_cumulative_kappa_over_frequency_matches_fuchs_sondheimer_prefix_sums():
    """The same film summed per frequency bin (an LA and a TA row share a bin below the TA edge)
    in ascending frequency."""
    d = 100e-9
    w = W.film(N=2_000_000, d=d, n_scat_max=10)
    b = oracle.run_batches(w, 16, threads=THREADS)
    c = oracle.kappa_cumulative(b, "omega")
    lam, k_fs = _fs_rows(w, b[0]["tables"], d)
    m = w["modes"]
    nb = int(m["bin"].max()) + 1
    per_bin = np.zeros(nb)
    np.add.at(per_bin, m["bin"], k_fs)
    centres = (np.arange(nb) + 0.5) * (W.OMEGA_MAX_LA / nb)
    assert np.allclose(c["keys"], centres, rtol=1e-12)
    ref = np.cumsum(per_bin)
    _check_deciles(c["kappa_cum"], c["kappa_cum_sigma"], ref)


def test_two_clock_rows_are_ordered_by_their_combined_relaxation_time():
    """With the impurity-like term as a separate clock, a row's free path is v / (1/tau + 1/tau_imp)
    (Matthiessen's rule): the order of the keys and the curve equal those of the one-clock rows."""
    w1 = W.film(N=200_000, n_scat_max=4)
    w2 = W.with_(w1, modes=W.silicon_like_modes(300.0, impurity_clock=True))
    c1 = oracle.kappa_cumulative(oracle.run_batches(w1, 4, threads=THREADS), "mfp")
    c2 = oracle.kappa_cumulative(oracle.run_batches(w2, 4, threads=THREADS), "mfp")
    assert np.allclose(c2["keys"], c1["keys"], rtol=1e-12)


def test_batches_of_one_particle_give_the_moment_standard_error():
    """Groups of one particle each: the batch-mean error of the last cumulative entry is the
    sample standard error of the particles' flux scores, which the oracle's tracer accumulates
    separately as moments (sum F, sum F^2), and their mean is kappa (1e-12)."""
    w = W.film(N=3000, d=50e-9, n_scat_max=6)
    b = oracle.run_batches(w, 3000, threads=THREADS)
    c = oracle.kappa_cumulative(b, "mfp")
    whole = oracle.run(w, threads=THREADS)
    assert abs(c["kappa_cum"][-1] - whole["kappa"]) <= 1e-12 * abs(whole["kappa"])
    assert abs(c["kappa_cum_sigma"][-1] - whole["kappa_sigma"]) <= 1e-9 * whole["kappa_sigma"]
    s = oracle.batch_statistics(b)
    assert abs(s["mean"][0, :, 2].sum() - whole["q"][0, :, 1].sum()) <= 1e-12 * abs(whole["q"][0, :, 1].sum())


def test_binned_batch_errors_follow_their_definition_on_unequal_groups():
    """Gray slab, 50 bins, groups of 1000, 3000 and 6000 particles: the mean is the finalized sum of
    all particles (bin by bin, 1e-12) and the error is the weighted spread written out per bin; one
    group gives NaN."""
    w = W.gray_slab(N=10_000)
    tb = oracle.Tables(w)
    bounds = [0, 1000, 4000, 10_000]
    groups = []
    for lo, hi in zip(bounds[:-1], bounds[1:]):
        raw, counts, mom, _ = tb.trace_range(int(w["seed"]), 0, lo, hi - lo)
        g = {"raw": raw, "counts": counts, "moments": mom, "tables": tb}
        g.update(oracle.finalize(g))
        groups.append(g)
    whole = oracle.run(w, threads=THREADS)
    s = oracle.batch_statistics(groups)
    scale = np.abs(whole["T"]).max()
    assert np.abs(s["mean"][..., 0] - whole["T"]).max() <= 1e-12 * scale
    n = np.array([1000.0, 3000.0, 6000.0])
    T = np.stack([g["T"] for g in groups])
    for cell in (0, 17, 49):
        x = T[:, cell, 0]
        m = float(np.dot(n, x) / n.sum())
        want = math.sqrt(float(np.dot(n, (x - m) ** 2)) / (2 * n.sum()))
        assert abs(s["sigma"][cell, 0, 0] - want) <= 1e-12 * want
    assert np.isnan(oracle.batch_statistics(groups[:1])["sigma"]).all()
