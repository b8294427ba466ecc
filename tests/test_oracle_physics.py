"""Whole-run pins of the CPU oracle against closed forms and exact invariants (no GPU).

Statistical pins use 3-sigma bounds (sigma from per-particle moments or from batch means
over contiguous particle ranges) plus, where a deterministic reference carries its own
discretisation error, that error stated next to the bound.
"""
import math

import numpy as np
import pytest

import closed_forms as cf
import oracle
import workloads as W

THREADS = 8
NB = 64          # batch means for binned tallies


def assert_bins_agree(batches_vals, ref, sys_err=0.0, family_alpha=1e-3):
    """Batch-mean check of binned tallies against a reference.

    z = |mean - ref| / (se + sys_err) follows Student-t with NB - 1 degrees of freedom; every
    bin must lie below the two-sided quantile at family-wise level family_alpha, and the mean of
    z^2 below its expectation nu/(nu-2) plus 4 standard errors.  Bins where no batch saw any
    particle (se = 0) must match the reference to rounding."""
    from scipy import stats
    vals = np.asarray(batches_vals)
    nb = vals.shape[0]
    mean = vals.mean(0)
    se = vals.std(0, ddof=1) / math.sqrt(nb)
    ref = np.broadcast_to(ref, mean.shape)
    ok = (se > 0)
    assert np.all(np.abs(mean[~ok] - ref[~ok]) <= 1e-12 + sys_err), "empty bins disagree"
    z = np.abs(mean - ref)[ok] / (se[ok] + sys_err)
    nu = nb - 1
    thr = stats.t.ppf(1.0 - family_alpha / (2.0 * max(z.size, 1)), nu)
    assert np.all(z < thr), (z.max(), thr)
    ez2 = nu / (nu - 2.0)
    var_z2 = 2.0 * ez2 ** 2 * (nu - 1.0) / (nu - 4.0)
    assert np.mean(z ** 2) < ez2 + 4.0 * math.sqrt(var_z2 / z.size), np.mean(z ** 2)


def test_ballistic_slab_flux_is_deterministic():
    """tau -> infinity: every wall particle crosses the slab once and contributes exactly L to
    sum s l_z, so q_z = (|dT_hot| + |dT_cold|) C v / 4 to rounding (walls at 301 / 299 K)."""
    w = W.gray_slab(N=20000)
    w["modes"]["tau"][0] = 1.0
    r = oracle.run(w, threads=THREADS)
    C, v = 1e6, 6400.0
    assert r["counts"]["relaxations"] == 0
    assert r["counts"]["absorbed"] == 20000
    assert r["q_score"] == pytest.approx(2.0 * C * v / 4.0, rel=1e-12)
    assert r["q_score_sigma"] < 1e-10 * r["q_score"]
    # per-bin: both walls superpose; the binned flux equals the same constant in every bin
    qz = r["q"][:, 0, 2]
    assert np.allclose(qz, 2.0 * C * v / 4.0, rtol=1e-11)


def test_ballistic_single_wall_temperature_is_half():
    """One emitting wall (the other held at T_lin): the ballistic steady temperature is dT/2
    everywhere (linearised ballistic limit)."""
    w = W.gray_slab(N=40000)
    w["modes"]["tau"][0] = 1.0
    w["geometry"]["faces"][6] = (W.ISOTHERMAL, 300.0, 0, 0)
    batches = oracle.run_batches(w, NB, threads=THREADS)
    assert_bins_agree([b["T"][:, 0] for b in batches], 0.5)


@pytest.mark.parametrize("tau_L", [1.0, 0.25])
def test_gray_slab_matches_integral_equation(tau_L):
    """Gray slab between black walls (301 / 299 K): flux Psi and the temperature profile against
    the product-integration solution of the E1-kernel integral equation."""
    L = 100e-9
    N = 100000
    w = W.gray_slab(N=N, Lambda=L / tau_L)
    t, phi, Psi = cf.gray_slab_integral_equation(tau_L, 2000)
    _, _, Psi2 = cf.gray_slab_integral_equation(tau_L, 1000)
    disc = abs(Psi - Psi2)                          # discretisation error of the reference
    r = oracle.run(w, threads=THREADS)
    q_ref = Psi * 1e6 * 6400.0 * 2.0 / 4.0
    assert abs(r["q_score"] - q_ref) < 3.0 * r["q_score_sigma"] + disc * q_ref
    # profile: T(z) = 2 phi(z / Lambda) - 1, averaged over the 50 detector bins
    nb = w["detectors"]["n"][2]
    ref = (2.0 * phi - 1.0).reshape(nb, -1).mean(1)
    batches = oracle.run_batches(w, NB, n=N, threads=THREADS)
    assert_bins_agree([b["T"][:, 0] for b in batches], ref, sys_err=1e-4)


def test_gradient_source_gives_kinetic_bulk_kappa_gray():
    """Unbounded gray bulk under the spatially varying control: kappa = C v^2 tau / 3 (this
    pins the factor 1/2 of the gradient source and the sign convention of its particles)."""
    for nsm in (1, 5):
        w = W.bulk_gradient(N=200000, n_scat_max=nsm)
        r = oracle.run(w, threads=THREADS)
        k_ref = 1e6 * 6400.0 ** 2 * (100e-9 / 6400.0) / 3.0
        assert abs(r["kappa"] - k_ref) < 3.0 * r["kappa_sigma"], (nsm, r["kappa"], r["kappa_sigma"])
        # single flight: per-particle score c = l mu with l ~ Exp(Lambda), mu ~ 2 mu dmu
        # -> coefficient of variation sqrt(5)/2
        if nsm == 1:
            cv = r["kappa_sigma"] * math.sqrt(200000) / r["kappa"]
            assert cv == pytest.approx(math.sqrt(5) / 2, rel=0.03)


def test_gradient_source_gives_kinetic_bulk_kappa_dispersive():
    """Frequency-dependent bulk: kappa = (1/3) sum_m C_m v_m^2 tau_m."""
    w = W.bulk_gradient(N=300000, n_scat_max=1, modes=W.silicon_like_modes(300.0))
    r = oracle.run(w, threads=THREADS)
    k_ref = r["tables"].kappa_bulk
    assert abs(r["kappa"] - k_ref) < 3.0 * r["kappa_sigma"], (r["kappa"], r["kappa_sigma"], k_ref)


def test_thin_film_matches_fuchs_sondheimer():
    """Diffuse-walled film, in-plane gradient: kappa = sum_m kappa_m S(d / Lambda_m)."""
    for d in (100e-9, 20e-9):
        w = W.film(N=150000, d=d)
        r = oracle.run(w, threads=THREADS)
        tb = r["tables"]
        C = tb.get("C")
        m = w["modes"]
        lam = m["v"] * m["tau"]
        k_fs = sum(C[i] * m["v"][i] ** 2 * m["tau"][i] / 3.0 * cf.fs_suppression(d / lam[i]) for i in range(len(m)))
        assert abs(r["kappa"] - k_fs) < 3.0 * r["kappa_sigma"], (d, r["kappa"], r["kappa_sigma"], k_fs)


def test_partially_specular_film_matches_fuchs():
    """Specularity p = 0.6 (drawn per hit against a 64-bit threshold): Fuchs' partially
    specular suppression, gray medium at Kn = 1 and Kn = 4."""
    for d in (100e-9, 25e-9):
        w = W.film(N=200000, d=d, specularity=0.6, n_scat_max=2)
        w["modes"] = W.gray_modes(6400.0, 100e-9 / 6400.0)
        w["problem"]["format"] = 2
        r = oracle.run(w, threads=THREADS)
        k_ref = 1e6 * 6400.0 ** 2 * (100e-9 / 6400.0) / 3.0 * cf.fs_suppression(d / 100e-9, 0.6)
        assert abs(r["kappa"] - k_ref) < 3.0 * r["kappa_sigma"], (d, r["kappa"], r["kappa_sigma"], k_ref)
        c = r["counts"]
        frac = c["specular"] / (c["specular"] + c["diffuse"])
        assert abs(frac - 0.6) < 4 * math.sqrt(0.24 / (c["specular"] + c["diffuse"]))


def test_specular_film_recovers_bulk():
    """Fully specular walls do not resist in-plane flow: kappa -> kappa_bulk."""
    w = W.film(N=100000, specularity=1.0, n_scat_max=1)
    w["modes"] = W.gray_modes(6400.0, 100e-9 / 6400.0)
    w["problem"]["format"] = 2
    r = oracle.run(w, threads=THREADS)
    k_ref = 1e6 * 6400.0 ** 2 * (100e-9 / 6400.0) / 3.0
    assert abs(r["kappa"] - k_ref) < 3.0 * r["kappa_sigma"]
    assert r["counts"]["specular"] > 0 and r["counts"]["diffuse"] == 0


def test_ballistic_transient_matches_closed_form():
    """The paper's ballistic benchmark (Eq. Analytical_T) on its own setup, per bin and time."""
    w = W.ballistic_transient(N=240000)
    p, det = w["problem"], w["detectors"]
    L, v = w["geometry"]["L"][2], 12360.0
    batches = oracle.run_batches(w, NB, threads=THREADS)
    ref = np.stack([cf.bin_average(lambda z: cf.ballistic_transient_dT(z, tk, L, v, 3.0, -3.0), 0.0, L,
                                   det["n"][2]) for tk in p["t_meas"]], axis=1)          # cell x time
    assert_bins_agree([b["T"] for b in batches], ref)


def test_transient_energy_is_conserved_exactly():
    """Specular walls, positive initial bump, nothing absorbed: the detector energy
    sum_c T_c C V_c equals the emitted energy at every measurement time."""
    w = W.transient_bump(N=20000, n_times=40, dt_meas=50e-12)
    r = oracle.run(w, threads=THREADS)
    tb = r["tables"]
    E = (r["T"] * tb.C_tot * r["V_cell"]).sum(0)
    assert np.allclose(E, tb.E_tot, rtol=1e-12)
    assert r["counts"]["timeouts"] == 20000
    assert r["counts"]["absorbed"] == 0 and r["counts"]["escaped"] == 0
    # the initial-condition energy is C A sum_c dT_c dz_c = C A sigma sqrt(2 pi) (1 K peak)
    assert tb.E_tot == pytest.approx(tb.C_tot * 50e-9 * math.sqrt(2 * math.pi), rel=1e-9)


def test_transient_first_snapshot_is_the_initial_condition():
    w = W.transient_bump(N=200000, n_times=2, dt_meas=10e-12)
    batches = oracle.run_batches(w, NB, threads=THREADS)
    dT = w["problem"]["ic_dT"]
    ref = (dT.reshape(100, 10)).mean(1)                       # 1 nm cells into 10 nm detector bins
    # bins far in the tails see no particle; there the reference is below 1e-3 K
    vals = np.array([b["T"][:, 0] for b in batches])
    seen = vals.std(0) > 0
    assert np.all(ref[~seen] < 1e-3)
    assert_bins_agree(vals[:, seen], ref[seen])


def test_gray_diffusive_bump_follows_fourier():
    """Short mean free path (10 nm) in a 1 um slab: at ~1000 relaxation times the bump spreads
    as the heat equation with D = v Lambda / 3 (insulated ends).  Bound: 3.5 sigma plus the
    O(Kn^2) ~ 1e-3 relative non-Fourier correction."""
    w = W.gray_diffusive_bump(N=64000, n_times=4)
    p, det = w["problem"], w["detectors"]
    L = 1e-6
    D = 6400.0 * 10e-9 / 3.0
    batches = oracle.run_batches(w, NB, threads=THREADS)
    for k, tk in enumerate(p["t_meas"]):
        if tk < 0.5e-9:
            continue
        ref = cf.bin_average(lambda z: cf.fourier_neumann_piecewise(z, tk, D, L, p["ic_edges"], p["ic_dT"]),
                             0.0, L, det["n"][2], per_bin=8)
        assert_bins_agree([b["T"][:, k] for b in batches], ref, sys_err=1e-3 * ref.max())


def test_swapping_wall_temperatures_negates_tallies_exactly():
    w = W.gray_slab(N=4000)
    a = oracle.run(w)
    w2 = W.with_(w, **{"geometry.faces": {5: (W.ISOTHERMAL, 299.0, 0, 0), 6: (W.ISOTHERMAL, 301.0, 0, 0)}})
    b = oracle.run(w2)
    assert np.array_equal(a["raw"], -b["raw"])
    assert np.array_equal(a["counts"], b["counts"])


def test_doubling_the_drive_doubles_results_exactly():
    w = W.gray_slab(N=4000)
    a = oracle.run(w)
    w2 = W.with_(w, **{"geometry.faces": {5: (W.ISOTHERMAL, 302.0, 0, 0), 6: (W.ISOTHERMAL, 298.0, 0, 0)}})
    b = oracle.run(w2)
    assert np.array_equal(a["raw"], b["raw"])
    assert np.array_equal(2.0 * a["T"], b["T"]) and np.array_equal(2.0 * a["q"], b["q"])


def test_particle_range_partition_is_invisible():
    """Particles are independent: [0, a) + [a, N) equals [0, N) (counts exact, sums to rounding)."""
    w = W.film(N=6000, d=50e-9)
    whole = oracle.trace(w)
    parts = [oracle.trace(w, first_pid=lo, n=hi - lo) for lo, hi in ((0, 1234), (1234, 4000), (4000, 6000))]
    assert np.array_equal(whole["counts"], sum(p["counts"] for p in parts))
    raw = sum(p["raw"] for p in parts)
    assert np.allclose(raw, whole["raw"], rtol=0, atol=1e-12 * np.abs(whole["raw"]).max())


def test_periodic_faces_are_transparent():
    """Linearised periodic condition (Eq. periodic_lin_final): reinsertion leaves the particle
    unchanged, so a periodic box reproduces unbounded bulk trajectory by trajectory."""
    w = W.bulk_gradient(N=20000, n_scat_max=6)
    faces = {1: (W.PERIODIC, 0, 3e-8, 0), 3: (W.PERIODIC, 0, -3e-8, 0), 2: (W.PERIODIC, -2e-8, 0, 0),
             4: (W.PERIODIC, 2e-8, 0, 0), 5: (W.PERIODIC, 0, 0, 5e-8), 6: (W.PERIODIC, 0, 0, -5e-8)}
    wp = W.with_(w, **{"geometry.unbounded": (False, False, False), "geometry.L": (2e-8, 3e-8, 5e-8),
                       "geometry.faces": faces, "geometry.volume": 1.0})
    a = oracle.trace(w, n_log=200)
    b = oracle.trace(wp, n_log=200)
    assert b["counts"][5] > 10 * 20000               # many periodic transfers happened
    for i in (0, 2, 8):                               # particles, relaxations, N_scat terminations
        assert a["counts"][i] == b["counts"][i]
    assert np.allclose(a["moments"], b["moments"], rtol=1e-11)
    # the event logs agree once periodic transfers are removed
    for ra, rb in zip(a["log"], b["log"]):
        ea = [e for e in ra[1:1 + ra[0]] if (e >> 28) != 4]
        eb = [e for e in rb[1:1 + min(rb[0], 63)] if (e >> 28) != 4]
        n = min(len(ea), len(eb))
        assert ea[:n] == eb[:n]


def test_dispersive_diffusion_uses_post_scattering_distribution():
    """Three short-mean-free-path modes: the late-time spreading of a bump follows Fourier with
    D = sum_m C_m v_m^2 tau_m / (3 sum_m C_m), which holds only if relaxations redraw modes with
    probability C_m / tau_m (Eq. norm_post_coll) -- a redraw proportional to C_m would give the
    D of time-fractions C_m tau_m instead."""
    modes = np.array([(1e13, 0.0, 6000.0, 0.0, 1.0e-12, 5.0e5, 0.0, 0, 1),
                      (2e13, 0.0, 1000.0, 0.0, 1.0e-11, 5.0e5, 0.0, 1, 1),
                      (3e13, 0.0, 3000.0, 0.0, 3.0e-12, 2.0e5, 0.0, 2, 2)], dtype=W.MODE_DTYPE)
    L = 3e-6
    w = W.transient_bump(N=48000, L=L, sigma=50e-9, n_cells=300, n_times=3, dt_meas=0.4e-9, bins=60,
                         modes=modes, fmt=2)
    w["problem"]["t_meas"] = np.array([0.4e-9, 0.8e-9, 1.19e-9])
    C, v, tau = modes["C"], modes["v"], modes["tau"]
    D = np.sum(C * v * v * tau) / (3 * C.sum())
    D_wrong = np.sum(C * tau * v * v * tau) / (3 * np.sum(C * tau))
    assert abs(D_wrong / D - 1) > 0.3
    batches = oracle.run_batches(w, NB, threads=THREADS)
    p = w["problem"]
    for k, tk in enumerate(p["t_meas"]):
        ref = cf.bin_average(lambda z: cf.fourier_neumann_piecewise(z, tk, D, L, p["ic_edges"], p["ic_dT"]),
                             0.0, L, 60, per_bin=8)
        assert_bins_agree([b["T"][:, k] for b in batches], ref, sys_err=3e-3 * ref.max())


def test_adjoint_gray_bulk_is_kappa():
    """kappa = C v^2 tau / 3 for the gray bulk, so dkappa / dln tau = kappa."""
    for nsm in (1, 4):
        w = W.bulk_gradient(N=200000, n_scat_max=nsm)
        a = oracle.adjoint(w, threads=THREADS, n_batches=NB)
        k_ref = 1e6 * 6400.0 ** 2 * (100e-9 / 6400.0) / 3.0
        assert_bins_agree(a["per_batch"], np.array([k_ref]))
        # the flux itself comes out of the same replayed particles
        assert abs(a["kappa"] - k_ref) < 4 * a["dkappa_dlntau_sigma"][0]


def test_pathwise_gray_bulk_equals_kappa_per_particle():
    """Gray bulk, periodic cell: stretching every flight by (1 + e) stretches the whole
    trajectory, so each particle's pathwise term equals its own flux score F (the draw terms of a
    single mode cancel: -1 + P = 0) and the estimate equals the kappa of the same particles."""
    for nsm in (1, 4):
        w = W.bulk_gradient(N=20000, n_scat_max=nsm)
        a = oracle.adjoint(w, threads=THREADS, estimator="pathwise", per_particle=True)
        assert np.allclose(a["per_particle"][:, 0], a["F"], rtol=1e-9, atol=1e-12 * np.abs(a["F"]).max())
        assert a["dkappa_dlntau"][0] == pytest.approx(a["kappa"], rel=1e-10)


def _tau_scaled(w, xi, eps):
    w2 = W.with_(w)
    w2["modes"]["tau"] = w2["modes"]["tau"] * (1.0 + eps * xi[w2["modes"]["bin"]])
    return w2


_GRAY = W.gray_modes(6400.0, 100e-9 / 6400.0)


@pytest.mark.parametrize("name,make", [
    ("gray_pore_diffuse", lambda: W.with_(W.porous_cell(N=300, modes=_GRAY), **{"problem.format": 2})),
    ("gray_pore_specular", lambda: W.with_(W.porous_cell(N=300, modes=_GRAY, specularity=1.0),
                                           **{"problem.format": 2})),
    ("gray_pore_partial", lambda: W.with_(W.porous_cell(N=300, modes=_GRAY, specularity=0.5),
                                          **{"problem.format": 2})),
    ("film_partial", lambda: W.film(N=300, specularity=0.4)),
    ("dispersive_pore", lambda: W.porous_cell(N=200)),
    ("dispersive_film", lambda: W.film(N=300)),
])
def test_pathwise_tangents_match_per_particle_finite_differences(name, make):
    """Brute force on single trajectories: scale tau_i by (1 +- e xi_i) with random signs xi over
    all bins (e = 1e-7, same random numbers).  Wherever neither run changes the particle's event
    sequence, the central difference of its flux score F is the pathwise part of its derivative,
    sum_i xi_i (tangent terms)_i -- a check of the tangent transport through boundary hits, specular
    and diffuse reflections off planes and the cylinder, periodic transfers and relaxations that
    does not use that transport."""
    w = make()
    n = w["problem"]["N"]
    tb = oracle.Tables(w)
    xi = np.random.default_rng(11).choice([-1.0, 1.0], size=tb.n_bins)
    eps = 1e-7
    a = oracle.adjoint(w, threads=THREADS, estimator="pathwise", per_particle=True)
    pred = a["per_particle"] @ xi
    wp, wm = _tau_scaled(w, xi, eps), _tau_scaled(w, xi, -eps)
    fp = oracle.adjoint(wp, threads=THREADS, estimator="pathwise")["F"]
    fm = oracle.adjoint(wm, threads=THREADS, estimator="pathwise")["F"]
    logs = [oracle.trace(x, n, n_log=n, log_stride=4096, threads=THREADS)["log"] for x in (w, wp, wm)]
    same = np.all(logs[1] == logs[0], axis=1) & np.all(logs[2] == logs[0], axis=1)
    assert same.mean() > 0.95
    fd = (fp - fm) / (2 * eps)
    scale = np.abs(pred[same]).max()
    assert scale > 0
    assert np.abs(fd - pred)[same].max() < 1e-7 * scale


@pytest.mark.parametrize("estimator", ["score", "pathwise", "local"])
def test_adjoint_dispersive_bulk_per_bin(estimator):
    """Dispersive bulk: after a relaxation the new direction is isotropic, so only the first
    flight carries mean flux and dkappa / dln tau_i = sum over the rows of bin i of
    C v^2 tau / 3 (groups of 25 bins and the total).  The relaxation times are capped at 1 ns
    (mean free paths up to 10 um): with the uncapped 2e-5 s of the lowest bins a few particles
    carry most of their sum and batch errors are unreliable; the relation holds for any table."""
    modes = W.silicon_like_modes(300.0)
    modes["tau"] = np.minimum(modes["tau"], 1e-9)
    n = 300000
    w = W.bulk_gradient(N=n, n_scat_max=3, modes=modes)
    a = oracle.adjoint(w, threads=THREADS, n_batches=NB, estimator=estimator)
    tb = a["tables"]
    C = tb.get("C")
    m = w["modes"]
    bins = tb.get("bin")
    ref = np.zeros(tb.n_bins)
    np.add.at(ref, bins, C * m["v"] ** 2 * m["tau"] / 3.0)
    # bins are grouped until each group expects >= 2000 emitted particles (emission ~ C v):
    # bins that are hardly ever emitted have skewed batch means whose spread underestimates
    # their error
    p_emit = np.zeros(tb.n_bins)
    np.add.at(p_emit, bins, C * m["v"])
    group = _groups_by_count(n * p_emit / p_emit.sum(), 2000.0)
    pb = a["per_batch"]
    G = group.max() + 1
    gb = np.zeros((NB, G))
    for k in range(NB):
        np.add.at(gb[k], group, pb[k])
    gr = np.zeros(G)
    np.add.at(gr, group, ref)
    assert G >= 20
    assert_bins_agree(gb, gr)
    assert_bins_agree(pb.sum(1)[:, None], np.array([ref.sum()]))


def _groups_by_count(expected, least):
    """Consecutive bins merged into groups with at least `least` expected events each (the last
    group absorbs a short remainder)."""
    g = np.zeros(len(expected), dtype=np.int64)
    k, acc = 0, 0.0
    for i, e in enumerate(expected):
        g[i] = k
        acc += e
        if acc >= least:
            k, acc = k + 1, 0.0
    if acc > 0.0 and k > 0:
        g[g == k] = k - 1
    return g


@pytest.mark.parametrize("estimator", ["score", "pathwise", "local"])
def test_adjoint_film_matches_fuchs_sondheimer_derivative(estimator):
    """Diffuse film: only the first flight carries mean flux, so dkappa/dln tau_i is the
    derivative of sum_{m in bin i} kappa_m S(d / Lambda_m) (closed form differentiated); compared
    in groups of 10 frequency bins (single low-frequency bins are too rarely emitted for a batch
    error) and in total."""
    d0 = 100e-9
    w = W.film(N=400000, d=d0)
    a = oracle.adjoint(w, threads=THREADS, n_batches=NB, estimator=estimator)
    tb = a["tables"]
    C = tb.get("C")
    m = w["modes"]
    bins = tb.get("bin")
    lam = m["v"] * m["tau"]
    ref = np.zeros(tb.n_bins)
    for i in range(len(m)):
        k = C[i] * m["v"][i] ** 2 * m["tau"][i] / 3.0
        delta = d0 / lam[i]
        e = 1e-5
        dS = (cf.fs_suppression(delta * math.exp(-e)) - cf.fs_suppression(delta * math.exp(e))) / (2 * e)
        ref[bins[i]] += k * cf.fs_suppression(delta) + k * dS
    pb = a["per_batch"]
    assert_bins_agree(pb.reshape(NB, -1, 10).sum(2), ref.reshape(-1, 10).sum(1))
    assert_bins_agree(pb.sum(1)[:, None], np.array([ref.sum()]))


def test_local_pathwise_at_absorbing_walls_against_crn_finite_difference():
    """Gray slab between isothermal (absorbing) walls with a gradient source: a flight that would
    end just past a wall is absorbed instead, which changes what follows, so carrying the stretch
    along the trajectory (the propagated pathwise form) is biased there; the local form keeps
    only the flight's own flux pathwise and scores what follows.  Both it and the score function
    must agree with central differences of kappa at tau (1 +- 0.05) on the same particles
    (16 batches, 3 combined standard errors)."""
    base = W.with_(W.gray_slab(N=1), **{"geometry.gradT": (0.0, 0.0, -2e7)})
    nb, n, eps = 16, 40000, 0.05
    est = {"score": [], "local": []}
    fd = []
    for b in range(nb):
        w = W.with_(base, **{"problem.N": n, "seed": int(base["seed"]) + 7 * b + 1})
        for e in est:
            est[e].append(oracle.adjoint(w, threads=THREADS, estimator=e)["dkappa_dlntau"][0])
        wp, wm = W.with_(w), W.with_(w)
        wp["modes"]["tau"] = w["modes"]["tau"] * (1 + eps)
        wm["modes"]["tau"] = w["modes"]["tau"] * (1 - eps)
        fd.append((oracle.run(wp, threads=THREADS)["kappa"] - oracle.run(wm, threads=THREADS)["kappa"]) / (2 * eps))
    fd = np.array(fd)
    for e, v in est.items():
        v = np.array(v)
        se = math.sqrt(v.var(ddof=1) / nb + fd.var(ddof=1) / nb)
        assert abs(v.mean() - fd.mean()) < 3.0 * se, (e, v.mean(), fd.mean(), se)
        assert se < 0.1 * abs(fd.mean())


# --------------------------------------------------------------------------------------------
# Separate two-phonon and three-phonon clocks (section 3.3): each process draws its own time to
# scattering from Eq. time_to_scat, the earlier one fires; a two-phonon event redraws only the
# direction (section 3.5.1), a three-phonon event redraws the phonon and both clocks.
# --------------------------------------------------------------------------------------------

def test_two_clock_gray_slab_matches_integral_equation_at_the_combined_free_path():
    """Gray medium: both events send the phonon off isotropically, so the race of two
    exponential clocks (rates 1/tau3 + 1/tau2) is one process with tau_eff = 1 / (1/tau3 +
    1/tau2); the slab must reproduce the E1 integral equation at Kn = v tau_eff / L = 1 and
    the share of two-phonon events must be tau3 / (tau2 + tau3)."""
    L, v, N = 100e-9, 6400.0, 100000
    tau_eff = L / v
    tau3, tau2 = 1.5 * tau_eff, 3.0 * tau_eff          # 1/1.5 + 1/3 = 1
    w = W.gray_slab(N=N, Lambda=L)
    w["modes"] = W.gray_modes(v, tau3, tau_imp=tau2)
    t, phi, Psi = cf.gray_slab_integral_equation(1.0, 2000)
    _, _, Psi2 = cf.gray_slab_integral_equation(1.0, 1000)
    disc = abs(Psi - Psi2)
    r = oracle.run(w, threads=THREADS)
    q_ref = Psi * 1e6 * v * 2.0 / 4.0
    assert abs(r["q_score"] - q_ref) < 3.0 * r["q_score_sigma"] + disc * q_ref
    n2, n3 = r["counts"]["two_phonon"], r["counts"]["relaxations"]
    p = tau3 / (tau2 + tau3)
    n = n2 + n3
    assert n > 10000
    assert abs(n2 / n - p) < 4.0 * math.sqrt(p * (1 - p) / n), (n2, n3)
    nb = w["detectors"]["n"][2]
    ref = (2.0 * phi - 1.0).reshape(nb, -1).mean(1)
    batches = oracle.run_batches(w, NB, n=N, threads=THREADS)
    assert_bins_agree([b["T"][:, 0] for b in batches], ref, sys_err=1e-4)


def test_two_clock_race_and_scattering_cap_counts_three_phonon_events_only():
    """Gray bulk, N_scat^max = 1: a walk ends at its first three-phonon event, and the two-phonon
    events before it are geometric with mean tau3 / tau2 (rate ratio); kappa = C v^2 tau_eff / 3."""
    v, N = 6400.0, 200000
    tau3, tau2 = 60e-12, 20e-12
    w = W.bulk_gradient(N=N, n_scat_max=1, modes=W.gray_modes(v, tau3, tau_imp=tau2))
    w["problem"]["format"] = 2                      # the gray row gives C directly
    r = oracle.run(w, threads=THREADS)
    c = r["counts"]
    assert c["relaxations"] == N and c["nscat_end"] == N
    mean2 = c["two_phonon"] / N
    ratio = tau3 / tau2
    p = ratio / (1.0 + ratio)
    sd = math.sqrt(p / (1.0 - p) ** 2 / N)          # geometric count on {0, 1, ...}
    assert abs(mean2 - ratio) < 4.0 * sd, (mean2, ratio, sd)
    tau_eff = 1.0 / (1.0 / tau3 + 1.0 / tau2)
    k_ref = 1e6 * v ** 2 * tau_eff / 3.0
    assert abs(r["kappa"] - k_ref) < 3.0 * r["kappa_sigma"], (r["kappa"], r["kappa_sigma"], k_ref)


def test_two_clock_dispersive_bulk_equals_the_summed_rate_kappa():
    """Silicon-like rows with the A omega^4 term on its own (two-phonon) clock: in bulk both
    processes relax the part of the deviation that carries heat, so kappa is
    (1/3) sum_m C_m v_m^2 / (1/tau3 + 1/tau2) -- the same number as the single clock with the
    rates summed."""
    w = W.bulk_gradient(N=300000, n_scat_max=1, modes=W.silicon_like_modes(300.0, impurity_clock=True))
    r = oracle.run(w, threads=THREADS)
    C = r["tables"].get("C")
    m = w["modes"]
    k_ref = float(np.sum(C * m["v"] ** 2 / (1.0 / m["tau"] + 1.0 / m["tau_imp"])) / 3.0)
    single = W.silicon_like_modes(300.0)
    k_single = float(np.sum(C * single["v"] ** 2 * single["tau"]) / 3.0)
    assert k_ref == pytest.approx(k_single, rel=1e-12)
    assert abs(r["kappa"] - k_ref) < 3.0 * r["kappa_sigma"], (r["kappa"], r["kappa_sigma"], k_ref)
    assert r["counts"]["two_phonon"] > 0


def test_two_clock_film_matches_fuchs_sondheimer_at_the_combined_free_path():
    """Diffuse film with the impurity term on the two-phonon clock: the deviation that carries
    the in-plane flux is odd in Omega_y, so the direction-only redraw removes it like a
    relaxation and kappa = sum_m kappa_m S(d / (v_m tau_eff,m))."""
    d = 100e-9
    w = W.film(N=150000, d=d, modes=W.silicon_like_modes(300.0, impurity_clock=True))
    r = oracle.run(w, threads=THREADS)
    C = r["tables"].get("C")
    m = w["modes"]
    tau_eff = 1.0 / (1.0 / m["tau"] + 1.0 / m["tau_imp"])
    lam = m["v"] * tau_eff
    k_fs = sum(C[i] * m["v"][i] ** 2 * tau_eff[i] / 3.0 * cf.fs_suppression(d / lam[i]) for i in range(len(m)))
    assert abs(r["kappa"] - k_fs) < 3.0 * r["kappa_sigma"], (r["kappa"], r["kappa_sigma"], k_fs)
    assert r["counts"]["two_phonon"] > 0


def test_two_phonon_draws_use_their_own_records():
    """A two-phonon clock that never fires (tau2 = 1e300 s) still draws its times, from records of
    its own: every count, tally and logged event equals the single-clock run's."""
    w1 = W.film(N=3000, modes=W.silicon_like_modes(300.0))
    w2 = W.film(N=3000, modes=W.silicon_like_modes(300.0))
    w2["modes"]["tau_imp"] = 1e300
    o1, o2 = oracle.Tables(w1), oracle.Tables(w2)
    sd = int(w1["seed"])
    raw1, c1, m1, log1 = o1.trace_range(sd, 0, 0, 3000, n_log=3000, log_stride=64)
    raw2, c2, m2, log2 = o2.trace_range(sd, 0, 0, 3000, n_log=3000, log_stride=64)
    assert np.array_equal(c1, c2) and c2[12] == 0
    assert np.array_equal(raw1, raw2) and np.array_equal(m1, m2) and np.array_equal(log1, log2)


# --------------------------------------------------------------------------------------------
# Frequency-dependent specularity (section 3.5.3: the specularity depends on the phonon; the
# paper's nanomesh reflects the phonons below 2 THz specularly): a boundary's cutoff frequency
# makes every phonon below it reflect specularly, the others with the boundary's d.
# --------------------------------------------------------------------------------------------

def test_film_with_a_specular_cutoff_matches_fuchs_sondheimer_per_mode():
    """Diffuse walls above the cutoff, specular below: kappa = sum_m kappa_m S(d / Lambda_m, p_m)
    with p_m = 1 below the cutoff and 0 above."""
    d = 100e-9
    wc = W.OMEGA_2THZ * 2.5                         # 5 THz: a sizeable share of the flux is specular
    w = W.film(N=150000, d=d, spec_omega=wc)
    r = oracle.run(w, threads=THREADS)
    C = r["tables"].get("C")
    m = w["modes"]
    lam = m["v"] * m["tau"]
    p = (m["omega"] < wc).astype(float)
    k_ref = sum(C[i] * m["v"][i] ** 2 * m["tau"][i] / 3.0 * cf.fs_suppression(d / lam[i], p[i])
                for i in range(len(m)))
    k_diffuse = sum(C[i] * m["v"][i] ** 2 * m["tau"][i] / 3.0 * cf.fs_suppression(d / lam[i])
                    for i in range(len(m)))
    assert k_ref > k_diffuse + 6.0 * r["kappa_sigma"]     # the pin separates the two readings
    assert abs(r["kappa"] - k_ref) < 3.0 * r["kappa_sigma"], (r["kappa"], r["kappa_sigma"], k_ref)
    assert r["counts"]["specular"] > 0 and r["counts"]["diffuse"] > 0


def test_specular_cutoff_extremes_reduce_to_constant_specularity():
    """A cutoff above every phonon is a specular wall, one below every phonon leaves d in force:
    counts, tallies and event logs bit-identical to those runs (no draw is added or moved)."""
    def trace(w):
        o = oracle.Tables(w)
        return o.trace_range(int(w["seed"]), 0, 0, 2000, n_log=2000, log_stride=64)
    for d_wall in (0.0, 0.4):
        base = W.film(N=2000, d=30e-9, specularity=d_wall)
        low = W.film(N=2000, d=30e-9, specularity=d_wall, spec_omega=1.0)       # below every row
        for a, b in zip(trace(base), trace(low)):
            assert np.array_equal(a, b)
    spec = W.film(N=2000, d=30e-9, specularity=1.0)
    high = W.film(N=2000, d=30e-9, specularity=0.4, spec_omega=1e15)             # above every row
    for a, b in zip(trace(spec), trace(high)):
        assert np.array_equal(a, b)
    pore = W.porous_cell(N=500, specularity=0.0)
    pore_hi = W.porous_cell(N=500, specularity=0.0, spec_omega=1e15)
    pore_sp = W.porous_cell(N=500, specularity=1.0)
    for a, b in zip(trace(pore_sp), trace(pore_hi)):
        assert np.array_equal(a, b)
    assert not np.array_equal(trace(pore)[1], trace(pore_hi)[1])


# --------------------------------------------------------------------------------------------
# Internal line walls (the paper's In_bnd rows: segments in the x-y plane through the thickness,
# normal into the domain)
# --------------------------------------------------------------------------------------------

def test_walled_film_matches_fuchs_sondheimer():
    """A channel between two diffuse line walls, periodic along the gradient: the thin film of
    thickness d, so kappa = sum_m kappa_m S(d / Lambda_m); the positions behind the walls are
    redrawn (emission with rejection), so about (H - d)/H of the first draws are rejected."""
    d = 100e-9
    w = W.walled_film(N=150000, d=d)
    r = oracle.run(w, threads=THREADS)
    C = r["tables"].get("C")
    m = w["modes"]
    lam = m["v"] * m["tau"]
    k_fs = sum(C[i] * m["v"][i] ** 2 * m["tau"][i] / 3.0 * cf.fs_suppression(d / lam[i]) for i in range(len(m)))
    assert abs(r["kappa"] - k_fs) < 3.0 * r["kappa_sigma"], (r["kappa"], r["kappa_sigma"], k_fs)
    H = w["geometry"]["L"][1]
    c = r["counts"]
    p_rej = (H - d) / H                   # rejections per emitted particle: geometric, mean p/(1-p)
    mean = c["rejections"] / c["particles"]
    sd = math.sqrt(p_rej / (1 - p_rej) ** 2 / c["particles"])
    assert abs(mean - p_rej / (1 - p_rej)) < 4 * sd, (mean, p_rej / (1 - p_rej))


def test_square_pore_of_line_walls_rejects_its_area_and_conserves_the_flux_sign():
    """The square pore of four walls: emission rejects positions inside it at the pore's area
    fraction; the pore lowers kappa below the bulk value but keeps it positive."""
    w = W.square_pore_cell(N=40000)
    r = oracle.run(w, threads=THREADS)
    c = r["counts"]
    p_rej = (250e-9 / 500e-9) ** 2
    mean = c["rejections"] / c["particles"]
    sd = math.sqrt(p_rej / (1 - p_rej) ** 2 / c["particles"])
    assert abs(mean - p_rej / (1 - p_rej)) < 4 * sd, (mean, p_rej / (1 - p_rej))
    assert c["diffuse"] > 0 and 0 < r["kappa"] < r["tables"].kappa_bulk


def test_isothermal_line_walls_ballistic_flux_is_deterministic():
    """tau -> infinity between two isothermal line walls: every particle goes from its wall to the
    other one and contributes exactly the gap to sum s l_y, so q = (|dT_hot| + |dT_cold|) C v / 4
    to rounding -- the walls' emission (area = segment length x thickness), direction about the
    normal and absorption."""
    w = W.walled_slab(N=20000)
    w["modes"]["tau"][0] = 1.0
    r = oracle.run(w, threads=THREADS)
    C, v = 1e6, 6400.0
    assert r["counts"]["relaxations"] == 0 and r["counts"]["absorbed"] == 20000
    assert r["q_score"] == pytest.approx(2.0 * C * v / 4.0, rel=1e-12)
    assert r["q_score_sigma"] < 1e-9 * r["q_score"]


def test_isothermal_line_walls_gray_slab_matches_integral_equation():
    """The gray slab at Kn = 1 between isothermal line walls: flux against the E1 integral equation."""
    w = W.walled_slab(N=100000)
    _, _, Psi = cf.gray_slab_integral_equation(1.0, 2000)
    _, _, Psi2 = cf.gray_slab_integral_equation(1.0, 1000)
    r = oracle.run(w, threads=THREADS)
    q_ref = Psi * 1e6 * 6400.0 * 2.0 / 4.0
    assert abs(r["q_score"] - q_ref) < 3.0 * r["q_score_sigma"] + abs(Psi - Psi2) * q_ref


def test_pore_lattice_kappa_is_isotropic_in_plane_and_translation_invariant():
    """The cell with a z-axis pore tiles a square lattice of pores: its in-plane conductivity
    tensor is isotropic (a 90-degree rotation maps the lattice onto itself), and moving the pore
    inside the cell only moves the lattice's origin.  Gray phonons, Lambda = 100 nm against a
    500 nm pitch and a 141 nm pore radius, so the pores cut kappa well below its bulk value."""
    base = W.porous_cell(N=400000, modes=W.gray_modes(6400.0, 1.5625e-11), n_scat_max=10)
    base["problem"]["format"] = 2
    Wc = base["geometry"]["L"][0]
    cyl = base["geometry"]["cylinders"][0]
    g = base["geometry"]["gradT"][1]
    runs = {
        "y": base,
        "x": W.with_(base, **{"geometry.gradT": (g, 0.0, 0.0), "problem.score_axis": 0}),
        "moved": W.with_(base, **{"geometry.cylinders": [(0.3 * Wc, 0.7 * Wc) + tuple(cyl[2:])]}),
    }
    res = {k: oracle.run(w, threads=THREADS) for k, w in runs.items()}
    k_bulk = res["y"]["tables"].kappa_bulk
    for k, r in res.items():
        assert r["kappa"] < 0.9 * k_bulk - 10.0 * r["kappa_sigma"], (k, r["kappa"], k_bulk)
    for a, b in (("y", "x"), ("y", "moved"), ("x", "moved")):
        ra, rb = res[a], res[b]
        assert abs(ra["kappa"] - rb["kappa"]) < 3.5 * math.hypot(ra["kappa_sigma"], rb["kappa_sigma"]), \
            (a, b, ra["kappa"], rb["kappa"], ra["kappa_sigma"], rb["kappa_sigma"])
