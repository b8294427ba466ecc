"""Pins of the oracle's per-row specularity tables (section 3.5.3: the degree of specularity of a
boundary depends on the phonon's wavelength).

* Special cases that reduce to what is already pinned: a table holding one value d everywhere
  traces exactly as the constant specularity d; a table holding 1 below a cutoff frequency and d
  above it traces exactly as the cutoff form (event logs and raw sums identical).
* The lookup itself: with a table of zeros and ones drawn at random per row, every logged
  reflection of a row must be specular exactly when its entry is 1 (faces, the pore, line walls).
* Physics: in a film whose walls are partly specular with a probability chosen per row, each row
  obeys Fuchs' partially specular suppression with its own p, so kappa is the sum of the rows'
  Fuchs conductivities (random p per row, and Ziman's roughness model).
"""
import os

import numpy as np

import closed_forms as cf
import oracle
import workloads as W

THREADS = min(8, os.cpu_count() or 1)
EV_SPEC, EV_DIFF = 2, 3


def _same_trace(wa, wb, n=3000):
    ra = oracle.trace(wa, n=n, n_log=n, log_stride=96, threads=THREADS)
    rb = oracle.trace(wb, n=n, n_log=n, log_stride=96, threads=THREADS)
    assert np.array_equal(ra["counts"], rb["counts"])
    assert np.array_equal(ra["log"], rb["log"])
    assert np.array_equal(ra["raw"], rb["raw"])
    return ra


def test_constant_table_traces_as_the_constant_specularity():
    base = W.film(N=3000, specularity=0.35)
    M = len(base["modes"])
    tab = W.with_spec_table(base, np.full(M, 0.35))
    r = _same_trace(base, tab)
    c = dict(zip(oracle.COUNT_NAMES, (int(x) for x in r["counts"])))
    assert c["specular"] > 0 and c["diffuse"] > 0


def test_step_table_traces_as_the_cutoff_frequency():
    """Film walls, the pore of the periodic cell and the walls of the walled film, each with
    d = 0.3 above a 2 THz cutoff and specular below it, against the same table."""
    for w in (W.film(N=3000, specularity=0.3, spec_omega=W.OMEGA_2THZ),
              W.porous_cell(N=3000, specularity=0.3, spec_omega=W.OMEGA_2THZ)):
        step = np.where(w["modes"]["omega"] < W.OMEGA_2THZ, 1.0, 0.3)
        _same_trace(w, W.with_spec_table(w, step))
    ww = W.walled_film(N=3000, specularity=0.3)
    ww["geometry"]["walls"] = [tuple(c[:9]) + (W.OMEGA_2THZ,) for c in ww["geometry"]["walls"]]
    step = np.where(ww["modes"]["omega"] < W.OMEGA_2THZ, 1.0, 0.3)
    _same_trace(ww, W.with_spec_table(ww, step))


def _reflections(r):
    """(event kind, boundary id, row) of every logged reflection."""
    out = []
    for row in r["log"]:
        n = min(int(row[0]), len(row) - 1)
        for e in row[1:1 + n]:
            e = int(e)
            kind = e >> 28
            if kind in (EV_SPEC, EV_DIFF):
                out.append((kind, (e >> 20) & 0xFF, e & 0xFFFFF))
    return out


def test_binary_table_decides_every_reflection_by_the_row():
    """Rows drawn specular (1) or diffuse (0) at random: each logged reflection off the film walls,
    the pore, or the line walls is specular exactly when its row's entry is 1."""
    cases = [W.film(N=4000, n_scat_max=4), W.porous_cell(N=4000, n_scat_max=4),
             W.walled_film(N=4000, n_scat_max=4)]
    for w in cases:
        table = W.random_specularity(len(w["modes"]), seed=11, binary=True)
        r = oracle.trace(W.with_spec_table(w, table), n_log=4000, log_stride=96, threads=THREADS)
        ev = _reflections(r)
        assert len(ev) > 500, w["name"]
        assert len({m for _, _, m in ev}) > 100
        for kind, bnd, m in ev:
            assert (kind == EV_SPEC) == (table[m] == 1.0), (w["name"], kind, bnd, m)
        assert {EV_SPEC, EV_DIFF} == {k for k, _, _ in ev}


def test_film_with_per_row_specularity_matches_per_row_fuchs():
    """50 nm film, each row's walls specular with its own probability p_i (uniform at random per
    row): kappa = sum_i C_i v_i^2 tau_i / 3 S(d / Lambda_i, p_i) within 3 standard errors (the
    partly specular draw against each row's own threshold; the binary test pins the lookup).
    Ziman's roughness model (eta = 0.2 nm) likewise."""
    d = 50e-9
    w = W.film(N=1_000_000, d=d, n_scat_max=10)
    table = W.random_specularity(len(w["modes"]), seed=5)
    r = oracle.run(W.with_spec_table(w, table), threads=THREADS)
    C = r["tables"].get("C")
    m = w["modes"]
    lam = m["v"] * m["tau"]
    kb = C * m["v"] ** 2 * m["tau"] / 3.0

    def fuchs(p):
        return sum(kb[i] * cf.fs_suppression(d / lam[i], p[i]) for i in range(len(m)))

    k_ref = fuchs(table)
    assert abs(r["kappa"] - k_ref) < 3.0 * r["kappa_sigma"], (r["kappa"], r["kappa_sigma"], k_ref)
    zim = W.ziman_specularity(m, 0.2e-9)
    assert zim.min() < 0.05 and zim.max() > 0.95
    rz = oracle.run(W.with_spec_table(w, zim), threads=THREADS)
    kz = fuchs(zim)
    assert abs(rz["kappa"] - kz) < 3.0 * rz["kappa_sigma"], (rz["kappa"], rz["kappa_sigma"], kz)
    assert abs(kz - k_ref) > 10.0 * r["kappa_sigma"]
