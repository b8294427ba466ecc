"""Sensitivities dkappa / dln tau_i through the C ABI (forward trace + replay) against the oracle's
likelihood-ratio estimator, and against common-random-number finite differences."""
import math
import os

import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

THREADS = min(16, os.cpu_count() or 1)


def _say(*a):
    print(*a, flush=True)


CASES = {
    "bulk_gray": lambda: W.bulk_gradient(N=5000, n_scat_max=3),
    "bulk_dispersive": lambda: W.bulk_gradient(N=4000, n_scat_max=4, modes=W.silicon_like_modes(300.0)),
    "film": lambda: W.film(N=4000),
    "film_partial": lambda: W.film(N=3000, d=40e-9, specularity=0.3),
    "porous_cell": lambda: W.porous_cell(N=2000),
    "porous_partial": lambda: W.porous_cell(N=2000, specularity=0.5),
    "gray_slab": lambda: W.with_(W.gray_slab(N=3000), **{"geometry.gradT": (0.0, 0.0, -2e7)}),
}
# the pathwise form needs a bounded number of flights per particle (1 <= n_scat_max <= 16)
PATHWISE_CASES = [k for k in CASES if k != "gray_slab"]


@pytest.mark.parametrize("name,estimator", [(k, "score") for k in CASES] + [(k, "pathwise") for k in PATHWISE_CASES]
                         + [(k, "local") for k in CASES])
def test_fp64_sensitivities_match_oracle(name, estimator):
    """Same particles, same events: the per-particle flux scores agree to rounding (the device
    logarithm and trigonometric functions may differ from the host's in the last place) and the
    summed sensitivity terms agree to rounding (the GPU also sums them in another order, and the
    pathwise form composes each flight's response before applying it)."""
    import paper_2104_03573_amd as M
    w = CASES[name]()
    _say(f"[adjoint fp64] {name} {estimator}")
    got = M.sensitivities(w, precision=64, estimator=estimator)
    ref = oracle.adjoint(w, threads=THREADS, estimator=estimator)
    _say(f"[adjoint fp64] {name} {estimator}: kappa {got['kappa']:.6g} / {ref['kappa']:.6g}")
    assert np.abs(got["F"] - ref["F"]).max() <= 1e-11 * np.abs(ref["F"]).max()
    nb = got["tables"].info["n_bins"]
    scale_s = max(np.abs(ref["sparse"]).max(), 1e-300)
    assert np.abs(got["adj_raw"][:nb] - ref["sparse"]).max() <= 1e-10 * scale_s
    assert abs(got["adj_raw"][nb] - ref["dense"]) <= 1e-10 * max(abs(ref["dense"]), scale_s)
    d_ref = ref["dkappa_dlntau"]
    assert np.abs(got["dkappa_dlntau"] - d_ref).max() <= 1e-9 * np.abs(d_ref).max()
    assert got["kappa"] == pytest.approx(ref["kappa"], rel=1e-12)


def test_pathwise_rejects_unbounded_flights():
    """A table with n_scat_max = 0 (unbounded flights per particle) has no pathwise form."""
    import paper_2104_03573_amd as M
    w = W.with_(W.gray_slab(N=100), **{"geometry.gradT": (0.0, 0.0, -2e7)})
    with pytest.raises(M.MCBTEError):
        M.sensitivities(w, precision=64, estimator="pathwise")


@pytest.mark.parametrize("estimator", ["score", "pathwise", "local"])
def test_fp32_sensitivities_match_oracle_statistically(estimator):
    """FP32 trajectories: the sensitivities of the film agree with the FP64 oracle's on the same
    particles within the oracle's batch errors (groups of 10 bins and the total).  The score form
    is far tighter than that (the same random numbers drive both).  The pathwise terms of long
    flights, s L Omega_y with L up to ~0.1 m, hinge on the last direction of the flight, which FP32
    rounding of a long bounce chain can change, so there only the batch errors bound it."""
    import paper_2104_03573_amd as M
    w = W.film(N=200000)
    got = M.sensitivities(w, precision=32, estimator=estimator)
    ref = oracle.adjoint(w, threads=THREADS, n_batches=32, estimator=estimator)
    g = got["dkappa_dlntau"].reshape(-1, 10).sum(1)
    pb = ref["per_batch"].reshape(32, -1, 10).sum(2)
    r = pb.mean(0)
    se = pb.std(0, ddof=1) / math.sqrt(32)
    ok = se > 0
    z = np.abs(g - r)[ok] / se[ok]
    se_tot = pb.sum(1).std(ddof=1) / math.sqrt(32)
    _say(f"[adjoint fp32] film {estimator}: total {g.sum():.4f} / {r.sum():.4f} (se {se_tot:.4f}), "
         f"max |z| over groups {z.max():.3f}")
    if estimator != "pathwise":
        assert z.max() < 1.0
        assert abs(g.sum() - r.sum()) < 0.1 * se_tot + 1e-12
    else:
        assert z.max() < 4.0
        assert abs(g.sum() - r.sum()) < 3.0 * se_tot


def _scaled(w, bins_set, factor):
    w2 = W.with_(w)
    sel = np.isin(w2["modes"]["bin"], list(bins_set))
    w2["modes"]["tau"][sel] *= factor
    return w2


@pytest.mark.parametrize("estimator", ["score", "local"])
def test_sensitivities_against_crn_finite_differences(estimator):
    """The porous cell (25 % pore, diffuse pore wall, periodic cell): for groups of frequency
    bins, the estimate (likelihood ratio, or local pathwise) agrees with central differences of kappa at
    tau (1 +- 0.05) computed with the same random numbers, within 3.5 standard errors
    (from the 16 paired batch differences: both come from the same particles). The central difference
    is biased by O(eps^2) of the second derivative, well below the tolerance; the test is only
    meaningful if the difference resolves the sensitivity, which it also checks for the groups
    that carry most of kappa."""
    import paper_2104_03573_amd as M
    base = W.porous_cell(N=1)
    nb_batches = 16
    n_per = 250000
    groups = [range(40, 80), range(80, 160), range(160, 320), range(320, 500)]
    eps = 0.05
    sf = np.zeros((nb_batches, len(groups)))
    fd = np.zeros((nb_batches, len(groups)))
    t0 = M.Tables(W.with_(base, **{"problem.N": n_per}))
    for b in range(nb_batches):
        w = W.with_(base, **{"problem.N": n_per, "seed": int(base["seed"]) + 7919 * b})
        s = M.sensitivities(w, precision=32, tables=t0, estimator=estimator)
        for gi, grp in enumerate(groups):
            sf[b, gi] = s["dkappa_dlntau"][list(grp)].sum()
            kp = M.run(_scaled(w, grp, 1.0 + eps), precision=32)["kappa"]
            km = M.run(_scaled(w, grp, 1.0 - eps), precision=32)["kappa"]
            fd[b, gi] = (kp - km) / (2.0 * eps)
    m_sf, m_fd = sf.mean(0), fd.mean(0)
    # both from the same particles: the error of their difference from the paired batch differences
    se = (sf - fd).std(0, ddof=1) / math.sqrt(nb_batches)
    se_fd = fd.std(0, ddof=1) / math.sqrt(nb_batches)
    _say(f"[adjoint vs CRN FD] {estimator}: estimate {np.round(m_sf, 4)} FD {np.round(m_fd, 4)} "
         f"paired se {np.round(se, 4)} (estimate alone {np.round(sf.std(0, ddof=1) / 4, 4)}, FD alone "
         f"{np.round(se_fd, 4)})")
    assert np.all(np.abs(m_sf - m_fd) < 3.5 * se)
    # the low-frequency group carries little of kappa: agreement only; the others must be resolved
    assert np.all(se_fd[1:] < 0.25 * np.abs(m_fd[1:]))


def _gray_pore(lam, N, specularity=0.0):
    return W.with_(W.porous_cell(N=N, modes=W.gray_modes(6400.0, lam / 6400.0), specularity=specularity),
                   **{"problem.format": 2})


@pytest.mark.parametrize("estimator", ["score", "pathwise", "local"])
def test_short_mean_free_path_pore_against_crn_finite_difference(estimator):
    """Gray medium with a 50 nm mean free path in the porous cell (pore radius 141 nm), where the
    pathwise form is well behaved: both estimates of dkappa / dln tau agree with the central
    difference at tau (1 +- 0.05) on the same particles within 3.5 standard errors of their paired
    batch differences, and the difference resolves the value."""
    import paper_2104_03573_amd as M
    nb_batches = 16
    n_per = 200000
    eps = 0.05
    est = np.zeros(nb_batches)
    fd = np.zeros(nb_batches)
    for b in range(nb_batches):
        w = W.with_(_gray_pore(50e-9, n_per), **{"seed": 0x5EED0 + 7919 * b})
        est[b] = M.sensitivities(w, precision=32, estimator=estimator)["dkappa_dlntau"][0]
        wp, wm = W.with_(w), W.with_(w)
        wp["modes"]["tau"] = w["modes"]["tau"] * (1.0 + eps)
        wm["modes"]["tau"] = w["modes"]["tau"] * (1.0 - eps)
        fd[b] = (M.run(wp, precision=32)["kappa"] - M.run(wm, precision=32)["kappa"]) / (2.0 * eps)
    # both from the same particles: the error of their difference from the paired batch differences
    se = (est - fd).std(ddof=1) / math.sqrt(nb_batches)
    _say(f"[short-mfp pore] {estimator}: {est.mean():.4f} +- {est.std(ddof=1) / 4:.4f}, "
         f"FD {fd.mean():.4f} +- {fd.std(ddof=1) / 4:.4f}, paired se {se:.4f}")
    assert abs(est.mean() - fd.mean()) < 3.5 * se
    assert fd.std(ddof=1) / math.sqrt(nb_batches) < 0.1 * abs(fd.mean())


def test_pathwise_overflow_is_reported():
    """Specular pore, 1 mm mean free path: every flight crosses thousands of cells and reflects
    off the convex pore again and again; the pathwise shifts grow geometrically until they are
    not finite in FP32.  The library must say so rather than return a number."""
    import paper_2104_03573_amd as M
    w = _gray_pore(1e-3, 2000, specularity=1.0)
    with pytest.raises(M.MCBTEError) as e:
        M.sensitivities(w, precision=32, estimator="pathwise")
    assert e.value.status == M.mcbte.ERANGE


@pytest.mark.parametrize("case,estimator", [("porous_cell", "score"), ("porous_cell", "local"),
                                            ("film_capped", "score"), ("film_capped", "pathwise")])
def test_rademacher_projection_against_crn_finite_difference(case, estimator):
    """One +- pair over all bins at once: tau_i -> tau_i (1 +- e xi_i) with random signs xi_i gives
    (kappa+ - kappa-) / 2e = sum_i xi_i dkappa / dln tau_i + O(e^2), compared with the estimate on
    the same particles (16 batches, e = 0.02).  Film with relaxation times capped at 1 ns (mean
    free paths up to 10 um) for the pathwise form, whose terms scale with the mean free path."""
    import paper_2104_03573_amd as M
    if case == "porous_cell":
        base = W.porous_cell(N=1)
    else:
        modes = W.silicon_like_modes(300.0)
        modes["tau"] = np.minimum(modes["tau"], 1e-9)
        base = W.film(N=1, modes=modes)
    nb_batches = 16
    n_per = 250000
    eps = 0.02
    t0 = M.Tables(W.with_(base, **{"problem.N": n_per}))
    xi = np.random.default_rng(5).choice([-1.0, 1.0], size=t0.info["n_bins"])
    est = np.zeros(nb_batches)
    fd = np.zeros(nb_batches)
    for b in range(nb_batches):
        w = W.with_(base, **{"problem.N": n_per, "seed": int(base["seed"]) + 104729 * b})
        est[b] = M.sensitivities(w, precision=32, tables=t0, estimator=estimator)["dkappa_dlntau"] @ xi
        wp, wm = W.with_(w), W.with_(w)
        wp["modes"]["tau"] = w["modes"]["tau"] * (1.0 + eps * xi[w["modes"]["bin"]])
        wm["modes"]["tau"] = w["modes"]["tau"] * (1.0 - eps * xi[w["modes"]["bin"]])
        fd[b] = (M.run(wp, precision=32)["kappa"] - M.run(wm, precision=32)["kappa"]) / (2.0 * eps)
    # both from the same particles: the error of their difference from the paired batch differences
    se = (est - fd).std(ddof=1) / math.sqrt(nb_batches)
    _say(f"[projection] {case} {estimator}: {est.mean():.4f} +- {est.std(ddof=1) / 4:.4f}, FD {fd.mean():.4f} +- "
         f"{fd.std(ddof=1) / 4:.4f}, paired se {se:.4f}")
    assert abs(est.mean() - fd.mean()) < 3.5 * se


def test_autograd_function_backward_is_the_replay():
    """kappa_of_tau: the forward value is the traced kappa, the gradient is the replay's
    dkappa / dln tau_i divided by tau_i, and it composes with other torch operations."""
    import torch
    import paper_2104_03573_amd as M
    w = W.film(N=20000)
    t0 = M.tau_bins(w)
    tau = torch.tensor(t0, dtype=torch.float64, requires_grad=True)
    k = M.kappa_of_tau(tau, w, precision=64)
    loss = (k - 40.0) ** 2
    loss.backward()
    ref = M.sensitivities(w, precision=64)
    assert k.item() == pytest.approx(ref["kappa"], rel=1e-12)
    expect = 2.0 * (ref["kappa"] - 40.0) * ref["dkappa_dlntau"] / t0
    assert np.allclose(tau.grad.numpy(), expect, rtol=1e-9, atol=1e-12 * np.abs(expect).max())


@pytest.mark.parametrize("precision", [64, 32])
def test_autograd_gray_bulk_matches_finite_difference_exactly(precision):
    """Gray unbounded bulk: scaling tau by (1 + e) scales every flight and so every particle's
    flux score by (1 + e) with the same random numbers, so kappa(tau) is linear in tau along the
    ray; the pathwise gradient through the Function must equal the central difference to rounding."""
    import torch
    import paper_2104_03573_amd as M
    w = W.bulk_gradient(N=20000, n_scat_max=3)
    t0 = M.tau_bins(w)
    tau = torch.tensor(t0, dtype=torch.float64, requires_grad=True)
    k = M.kappa_of_tau(tau, w, precision=precision, estimator="pathwise")
    k.backward()
    e = 1e-3
    kp = M.kappa_of_tau(torch.tensor(t0 * (1 + e)), w, precision=precision).item()
    km = M.kappa_of_tau(torch.tensor(t0 * (1 - e)), w, precision=precision).item()
    fd = (kp - km) / (2 * e)
    got = float(tau.grad.numpy() @ t0)
    tol = 1e-9 if precision == 64 else 2e-4
    assert got == pytest.approx(fd, rel=tol)
    assert got == pytest.approx(k.item(), rel=tol)
