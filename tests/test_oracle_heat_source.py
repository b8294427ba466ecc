"""Pins of the oracle's external heat source (the phonon generation by an external source that the
paper's summary names for time-domain thermoreflectance): deviational power density P_k over time
intervals in a cuboid; particles start at a time uniform in their interval, a position uniform in
the cuboid, a row drawn by heat capacity and an isotropic direction.

* Energy: in a slab with adiabatic walls nothing leaves, so after the pulse every particle is in
  some bin at every measurement time (the snapshot total equals the particle count exactly), and
  before it the count of particles already started follows the pulse's cumulative energy.
* A source filling the whole slab heats it uniformly: T(t) = int_0^t P dt' / C_tot in every bin,
  with a heating and a cooling interval.
* Ballistic spreading (tau -> infinity) of a thin heated layer: the closed-form density of
  z_e + v (t - t_e) mu with z_e, t_e and mu uniform, per bin.
* The rows drawn: each row's share of the emitted particles is C_m / C_tot.
"""
import math
import os

import numpy as np

import closed_forms as cf
import oracle
import workloads as W
from test_oracle_physics import assert_bins_agree

THREADS = min(8, os.cpu_count() or 1)
NB = 32


def test_heated_slab_conserves_the_energy_of_the_pulse():
    w = W.heated_slab(N=40_000, t_max=100e-12, n_times=40, n_cells=20)
    r = oracle.run(w, threads=THREADS)
    raw = r["raw"].reshape(20, 40, 4)
    count = raw[..., 0].sum(axis=0)                      # signs summed over the bins, per time
    heat = w["problem"]["heat"]
    edges, P = heat["t"], heat["P"]
    t_meas = w["problem"]["t_meas"]
    cum = np.concatenate([[0.0], np.cumsum(P * np.diff(edges))])
    N = w["problem"]["N"]
    for k, t in enumerate(t_meas):
        if t >= edges[-1]:
            assert count[k] == N                          # every particle started and none left
        else:
            f = np.interp(t, edges, cum) / cum[-1]       # share of the pulse's energy before t
            assert abs(count[k] - N * f) <= 5.0 * math.sqrt(N * f * (1 - f)) + 1, (t, count[k], N * f)
    # the finalized deviational energy after the pulse: C_tot V_cell sum_cells T = E_tot
    tb = r["tables"]
    E = tb.C_tot * r["V_cell"] * r["T"][:, -1].sum()
    assert abs(E - tb.E_tot) <= 1e-12 * tb.E_tot
    assert r["counts"]["particles"] == N and r["counts"]["timeouts"] == N


def test_source_filling_the_slab_heats_it_uniformly():
    """Heating at P over [0, 20 ps), cooling at -P/2 over [20, 60 ps); specular walls, 80 ps:
    T = int_0^t P dt' / C_tot in all 10 bins at every time (batch means of 32 groups)."""
    L, Pw = 200e-9, 5e16
    w = W.heated_slab(N=200_000, L=L, t_max=80e-12, n_times=8, n_cells=10, specularity=1.0)
    w["problem"]["heat"] = {"lo": (0.0, 0.0, 0.0), "hi": (1.0, 1.0, L), "t": np.array([0.0, 20e-12, 60e-12]),
                            "P": np.array([Pw, -0.5 * Pw])}
    batches = oracle.run_batches(w, NB, threads=THREADS)
    C_tot = batches[0]["tables"].C_tot
    t = w["problem"]["t_meas"]
    Q = Pw * np.minimum(t, 20e-12) - 0.5 * Pw * np.clip(t - 20e-12, 0.0, 40e-12)
    assert_bins_agree([b["T"] for b in batches], (Q / C_tot)[None, :])


def test_ballistic_spreading_of_a_heated_layer():
    """Gray medium with tau -> infinity, a 100 nm layer in the middle of a 3 um slab heated over
    [0, 2 ps); at 20, 60 and 120 ps the layer has spread to z_e + v (t - t_e) mu (no particle has
    reached a wall): T per bin against the bin average of that density."""
    L, v, a, b, dt = 3e-6, 6400.0, 1.45e-6, 1.55e-6, 2e-12
    t_meas = np.array([20e-12, 60e-12, 120e-12])
    w = W.heated_slab(N=300_000, L=L, modes=W.gray_modes(v, 1.0), t_max=150e-12, n_cells=60)
    w["problem"].update(format=2, t_meas=t_meas)
    w["problem"]["heat"] = {"lo": (0.0, 0.0, a), "hi": (1.0, 1.0, b), "t": np.array([0.0, dt]),
                            "P": np.array([1e17])}
    batches = oracle.run_batches(w, NB, threads=THREADS)
    tb = batches[0]["tables"]
    xg, wg = np.polynomial.legendre.leggauss(16)
    ref = np.zeros((60, 3))
    for k, t in enumerate(t_meas):
        for x, wq in zip(xg, wg):
            te = 0.5 * dt * (x + 1.0)
            rr = v * (t - te)

            def dens(z):
                lo = np.maximum(z - rr, a)
                hi = np.minimum(z + rr, b)
                return np.maximum(hi - lo, 0.0) / (2.0 * rr * (b - a))
            ref[:, k] += 0.5 * wq * cf.bin_average(dens, 0.0, L, 60)
    # bin average of the density times the energy, over the bin's heat capacity
    ref *= tb.E_tot / tb.C_tot
    assert abs(ref[:, 0].sum() * (L / 60) - tb.E_tot / tb.C_tot) < 1e-6 * tb.E_tot / tb.C_tot
    assert_bins_agree([bt["T"] for bt in batches], ref)


def test_heat_source_rows_are_drawn_by_heat_capacity():
    """The silicon-like crystal: the emitted rows, grouped into 20 bands of rows, against C_m / C_tot
    (binomial, 5 standard errors per band)."""
    w = W.heated_slab(N=60_000, t_max=40e-12, n_times=4, n_cells=4)
    r = oracle.trace(w, n_log=60_000, log_stride=4, threads=THREADS)
    rows = np.array([int(row[1]) & 0xFFFFF for row in r["log"]])
    C = r["tables"].get("C")
    p = C / C.sum()
    groups = np.array_split(np.arange(len(C)), 20)
    n = len(rows)
    for g in groups:
        want = p[g].sum()
        got = np.isin(rows, g).sum()
        assert abs(got - n * want) <= 5.0 * math.sqrt(n * want * (1 - want)) + 1


def _positions(w, n):
    tb = oracle.Tables(w)
    return tb, np.array([tb.emit_state(pid)[0][:3] for pid in range(n)])


def _barycentric(v, x):
    """Barycentric coordinates of points x (n, 3) in the tetrahedron v (4, 3), by solving the
    3 x 3 system of the edges."""
    E = np.stack([v[1] - v[0], v[2] - v[0], v[3] - v[0]], axis=1)
    b = np.linalg.solve(E, (x - v[0]).T).T
    return np.concatenate([1.0 - b.sum(axis=1, keepdims=True), b], axis=1)


def test_heat_source_points_are_uniform_in_a_tetrahedron():
    """The heat source in one tetrahedron (section 3.2: arbitrary regions built from tetrahedra):
    every emitted point lies inside it, each barycentric coordinate follows its law for a uniform
    point (P(b <= x) = 1 - (1 - x)^3, Kolmogorov-Smirnov), and mean and covariance are the
    simplex's: the centroid and (1/20) sum_i (v_i - c)(v_i - c)^T."""
    from scipy import stats
    w = W.heated_box(N=20_000)
    v = np.asarray(w["problem"]["heat"]["tets"][0])
    tb, x = _positions(w, 20_000)
    b = _barycentric(v, x)
    assert b.min() > -1e-12 and b.max() < 1.0 + 1e-12
    for k in range(4):
        assert stats.kstest(b[:, k], lambda q: 1.0 - (1.0 - np.clip(q, 0, 1)) ** 3).pvalue > 1e-4, k
    c = v.mean(axis=0)
    cov = sum(np.outer(vi - c, vi - c) for vi in v) / 20.0
    n = len(x)
    se = np.sqrt(np.diag(cov) / n)
    assert np.all(np.abs(x.mean(axis=0) - c) < 5.0 * se)
    emp = np.cov(x.T)
    assert np.abs(emp - cov).max() < 0.05 * np.abs(cov).max()


def test_tetrahedra_of_a_cuboid_heat_it_as_the_cuboid_does():
    """The cuboid region as six tetrahedra: the same energy (volumes add up to the cuboid's, 1e-12),
    points uniform along each axis of the cuboid (Kolmogorov-Smirnov), each tetrahedron chosen
    with its share of the volume (1/6, binomial 5 sigma); and two tetrahedra of unequal volume are
    chosen in proportion to their volumes."""
    from scipy import stats
    lo, hi = np.array([50e-9, 40e-9, 30e-9]), np.array([350e-9, 240e-9, 130e-9])
    cube = W.heated_box(N=100, tets=W.cube_tets(lo, hi))
    box = W.with_(cube)
    box["problem"]["heat"] = dict(box["problem"]["heat"], lo=tuple(lo), hi=tuple(hi), tets=None)
    assert abs(oracle.Tables(cube).E_tot - oracle.Tables(box).E_tot) <= 1e-12 * oracle.Tables(box).E_tot
    n = 12_000
    tb, x = _positions(W.with_(cube, **{"problem.N": n}), n)
    for a in range(3):
        assert stats.kstest((x[:, a] - lo[a]) / (hi[a] - lo[a]), "uniform").pvalue > 1e-4, a
    tets = W.cube_tets(lo, hi)
    inside = np.array([[np.all(_barycentric(t, x[i:i + 1]) >= -1e-12) for t in tets] for i in range(2000)])
    share = inside.sum(axis=0) / 2000.0
    assert np.all(np.abs(share - 1.0 / 6.0) < 5.0 * math.sqrt((1 / 6) * (5 / 6) / 2000))
    small = np.array([[0, 0, 0], [100e-9, 0, 0], [0, 100e-9, 0], [0, 0, 100e-9]]) + 20e-9
    big = np.array([[0, 0, 0], [200e-9, 0, 0], [0, 200e-9, 0], [0, 0, 150e-9]]) + np.array([150e-9, 50e-9, 20e-9])
    two = W.heated_box(N=n, tets=np.array([small, big]))
    tb2, x2 = _positions(two, n)
    in_small = np.all(_barycentric(small, x2) >= -1e-12, axis=1)
    p = 1.0 / (1.0 + (2 * 2 * 1.5))          # volume ratio 1 : 6
    assert abs(in_small.sum() - n * p) < 5.0 * math.sqrt(n * p * (1 - p))
