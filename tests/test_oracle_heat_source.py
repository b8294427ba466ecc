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
