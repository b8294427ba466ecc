"""The C-ABI library on the CPU: it loads, exports every declared entry point, builds host-side
tables identical to the oracle's, and rejects bad input with the documented codes.  No kernel
is launched here."""
import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

import oracle
import paper_2104_03573_amd as M
import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "mcbte.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mcbte_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    names = declared_functions()
    assert len(names) >= 11
    lib = M.lib()
    for n in names:
        assert hasattr(lib, n), n
    dyn = subprocess.run(["nm", "-D", "--defined-only", M.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (mcbte_\w+)", dyn))
    assert set(names) <= exported, set(names) - exported
    assert set(M.EXPORTED) == set(names)


@pytest.mark.parametrize("make", [lambda: W.gray_slab(N=1000), lambda: W.film(N=1000),
                                  lambda: W.transient_bump(N=1000), lambda: W.porous_cell(N=1000),
                                  lambda: W.ballistic_transient(N=100), lambda: W.bulk_gradient(N=10),
                                  lambda: W.film(N=7, d=3e-8, T=100.0, specularity=0.3),
                                  lambda: W.heated_slab(N=100, t_max=100e-12, n_times=4, n_cells=4),
                                  lambda: W.heated_box(N=100)])
def test_host_tables_identical_to_oracle(make):
    w = make()
    t = M.Tables(w, device=-1)
    o = oracle.Tables(w)
    inf = t.info
    assert inf["device"] == -1
    for k, v in (("C_tot", o.C_tot), ("E_tot", o.E_tot), ("V_solid", o.V_solid), ("e_eff", o.e_eff),
                 ("sum_Cv", o.Wv), ("kappa_bulk", o.kappa_bulk)):
        assert inf[k] == v, k
    assert (inf["n_modes"], inf["n_sources"], inf["n_cells"], inf["n_cols"]) == (o.M, o.S, o.n_cells, o.n_cols)
    for k in ("C", "thr_ic", "thr_wall", "thr_rel", "src_E", "thr_src", "src_sign"):
        assert np.array_equal(M.table_export(t, k), o.get(k)), k
    base = 256 + o.n_cells * o.n_cols * 4 * 8
    # a pore lattice's buffer also holds the list of particles its FP32 trace starts first (4096 ids)
    lattice = w["name"] == "porous_cell"
    assert inf["tally_bytes"] == ((base + 255) // 256 * 256 + 8 * 4096 if lattice else base)


def _status(w, device=-1):
    try:
        M.Tables(w, device)
        return 0
    except M.MCBTEError as e:
        return e.status


def test_invalid_inputs_are_rejected():
    w = W.gray_slab(N=10)
    bad = W.with_(w)
    bad["modes"]["v"][0] = 0.0
    assert _status(bad) == M.mcbte.EINVAL
    assert _status(W.with_(w, **{"problem.N": 0})) == M.mcbte.EINVAL
    assert _status(W.with_(w, **{"geometry.faces": {5: (W.PERIODIC, 0, 0, 1e-7), 6: (W.ISOTHERMAL, 299.0, 0, 0)}})) \
        == M.mcbte.EGEOM
    assert _status(W.with_(w, **{"geometry.faces": {5: (W.ISOTHERMAL, 300.0, 0, 0),
                                                     6: (W.ISOTHERMAL, 300.0, 0, 0)}})) == M.mcbte.ETABLE
    assert _status(W.with_(w, **{"detectors.mask": 0})) == M.mcbte.EINVAL
    assert _status(W.with_(w, **{"detectors.n": (0, 0, 5), "detectors.hi": (0, 0, -1.0)})) == M.mcbte.EINVAL
    p = W.porous_cell(N=10)
    assert _status(W.with_(p, **{"geometry.cylinders": [(0.1e-7, 2.5e-7, 1.4e-7, 7, W.ADIABATIC, 0.0)]})) \
        == M.mcbte.EGEOM
    assert _status(W.with_(p, **{"geometry.faces": {**p["geometry"]["faces"], 1: (W.PERIODIC, 0, 1e-7, 0)}})) \
        == M.mcbte.EGEOM
    f = W.film(N=10)
    assert _status(W.with_(f, **{"geometry.faces": {5: (W.ADIABATIC, 1.5, 0, 0), 6: (W.ADIABATIC, 0, 0, 0)}})) \
        == M.mcbte.EGEOM
    zero = W.with_(f)
    zero["modes"]["dos"][:] = 0.0
    assert _status(zero) == M.mcbte.ETABLE
    tr = W.transient_bump(N=10)
    assert _status(W.with_(tr, **{"problem.transient": False})) == M.mcbte.EINVAL   # IC needs a transient run
    unsorted = W.with_(tr)
    unsorted["problem"]["t_meas"] = unsorted["problem"]["t_meas"][::-1].copy()
    assert _status(unsorted) == M.mcbte.EINVAL


def test_device_calls_reject_host_only_tables():
    t = M.Tables(W.gray_slab(N=10), device=-1)
    run = M.make_run(1, 64)
    L = M.lib()
    dummy = C.c_void_p(1)
    assert L.mcbte_trace(t.h, C.byref(run), 0, 10, None, dummy, None) == M.mcbte.ENODEV
    assert L.mcbte_emit(t.h, C.byref(run), 0, 10, dummy, 10, None) == M.mcbte.ENODEV
    res = M.mcbte.Result()
    assert L.mcbte_tally(t.h, dummy, None, 0, C.byref(res), None) == M.mcbte.ENODEV
    run.precision = 16
    assert L.mcbte_trace(t.h, C.byref(run), 0, 10, None, dummy, None) == M.mcbte.EINVAL
    assert L.mcbte_trace(None, C.byref(run), 0, 10, None, dummy, None) == M.mcbte.EINVAL


def test_finalize_calls_check_their_arguments_before_the_device():
    """mcbte_kappa_cumulative needs a steady, unbinned problem whose tally holds the flux along the
    score axis, and a known order; both finalize calls check buffer lists and output sizes, then refuse tables
    without a device."""
    L = M.lib()
    dummy = C.c_void_p(1)
    one = (C.c_void_p * 1)(dummy)
    two_null = (C.c_void_p * 2)(dummy, None)
    out = np.zeros(4000)
    d = out.ctypes.data_as(C.POINTER(C.c_double))
    film = M.Tables(W.film(N=10), device=-1)
    M_rows, nb = film.info["n_modes"], film.info["n_bins"]
    assert L.mcbte_kappa_cumulative(film.h, one, 1, M.mcbte.CUM_MFP, d, d, d, M_rows, None) == M.mcbte.ENODEV
    assert L.mcbte_kappa_cumulative(film.h, one, 1, M.mcbte.CUM_OMEGA, None, d, None, nb, None) == M.mcbte.ENODEV
    assert L.mcbte_kappa_cumulative(film.h, one, 1, M.mcbte.CUM_MFP, d, d, d, M_rows - 1, None) == M.mcbte.ESIZE
    assert L.mcbte_kappa_cumulative(film.h, one, 1, M.mcbte.CUM_OMEGA, d, d, d, nb - 1, None) == M.mcbte.ESIZE
    assert L.mcbte_kappa_cumulative(film.h, one, 1, 2, d, d, d, M_rows, None) == M.mcbte.EINVAL
    assert L.mcbte_kappa_cumulative(film.h, one, 0, 0, d, d, d, M_rows, None) == M.mcbte.EINVAL
    assert L.mcbte_kappa_cumulative(film.h, C.cast(two_null, C.POINTER(C.c_void_p)), 2, 0, d, d, d, M_rows,
                                    None) == M.mcbte.EINVAL
    assert L.mcbte_kappa_cumulative(film.h, one, 1, 0, d, None, d, M_rows, None) == M.mcbte.EINVAL
    for w in (W.gray_slab(N=10), W.film(N=10, z_bins=4), W.transient_bump(N=10),
              W.with_(W.film(N=10), **{"detectors.mask": W.MASK_T | W.MASK_QX})):
        t = M.Tables(w, device=-1)
        assert L.mcbte_kappa_cumulative(t.h, one, 1, 0, d, d, d, 4000, None) == M.mcbte.EINVAL, w["name"]
    slab = M.Tables(W.gray_slab(N=10), device=-1)
    n = slab.info["n_cells"] * slab.info["n_cols"] * 4
    assert L.mcbte_tally_batches(slab.h, one, 1, d, d, n, None) == M.mcbte.ENODEV
    assert L.mcbte_tally_batches(slab.h, one, 1, None, d, n, None) == M.mcbte.ENODEV
    assert L.mcbte_tally_batches(slab.h, one, 1, d, d, n - 1, None) == M.mcbte.ESIZE
    assert L.mcbte_tally_batches(slab.h, one, 1, None, None, n, None) == M.mcbte.EINVAL
    assert L.mcbte_tally_batches(slab.h, one, 0, d, d, n, None) == M.mcbte.EINVAL
    assert L.mcbte_tally_batches(slab.h, C.cast(two_null, C.POINTER(C.c_void_p)), 2, d, d, n,
                                 None) == M.mcbte.EINVAL


def test_specularity_table_inputs():
    """A boundary's per-row table: a known number, on an adiabatic boundary whose own d and cutoff
    are 0; table values in [0, 1]; reserved words 0.  Equal to the oracle's checks."""
    base = W.film(N=10)
    M_rows = len(base["modes"])
    ok = W.with_spec_table(base, np.linspace(0.0, 1.0, M_rows))
    assert _status(ok) == 0
    assert M.Tables(ok, device=-1).info["n_modes"] == M_rows

    def face5(w, f):
        w = W.with_(w)
        w["geometry"]["faces"][5] = f
        return w

    bad_geom = [face5(ok, (W.ADIABATIC, 0.0, 0.0, 0.0, 2)),          # no table 2
                face5(ok, (W.ADIABATIC, 0.2, 0.0, 0.0, 1)),          # own d with a table
                face5(ok, (W.ADIABATIC, 0.0, 1e13, 0.0, 1)),         # own cutoff with a table
                face5(ok, (W.ISOTHERMAL, 300.0, 0.0, 0.0, 1)),       # not adiabatic
                face5(ok, (W.ADIABATIC, 0.0, 0.0, 0.0, -1))]
    cell = W.with_spec_table(W.porous_cell(N=10), np.full(M_rows, 0.5))
    c = list(cell["geometry"]["cylinders"][0])
    c[5] = 0.5
    bad_geom.append(W.with_(cell, **{"geometry.cylinders": [tuple(c)]}))
    slab = W.walled_slab(N=10)
    walls = [tuple(x[:9]) + (0.0, 1) for x in slab["geometry"]["walls"]]
    bad_geom.append(W.with_(slab, **{"geometry.walls": walls, "problem.spec_tables": np.zeros((1, 1))}))
    for w in bad_geom:
        assert _status(w) == M.mcbte.EGEOM, w["geometry"]["faces"].get(5)
        with pytest.raises(ValueError):
            oracle.Tables(w)
    for vals in (np.full(M_rows, 1.5), np.full(M_rows, -0.1), np.full(M_rows, np.nan)):
        w = W.with_spec_table(base, np.zeros(M_rows))
        w["problem"]["spec_tables"] = vals[None, :]
        assert _status(w) == M.mcbte.EINVAL
        with pytest.raises(ValueError):
            oracle.Tables(w)


def test_heat_source_inputs():
    """The external heat source: transient only, ascending edges inside [0, t_max], finite power
    densities, a cuboid inside the box that no pore reaches into, no line walls; the library and
    the oracle refuse the same inputs."""
    ok = W.heated_slab(N=10, t_max=100e-12, n_times=4, n_cells=4)
    assert _status(ok) == 0
    t = M.Tables(ok, device=-1)
    heat = ok["problem"]["heat"]
    assert t.info["n_sources"] == len(heat["P"]) == oracle.Tables(ok).S

    def hv(**kw):
        w = W.with_(ok)
        w["problem"]["heat"] = dict(heat, **kw)
        return w

    cell = W.with_(W.porous_cell(N=10), **{"problem.transient": True, "problem.t_max": 1e-11,
                                           "problem.t_meas": np.array([5e-12])})
    bad = [W.with_(ok, **{"problem.transient": False, "problem.t_meas": np.zeros(0)}),
           hv(t=heat["t"][::-1].copy()),                                   # not ascending
           hv(t=heat["t"] + 1.0),                                          # past t_max
           hv(P=np.full(len(heat["P"]), np.inf)),
           hv(lo=(0.0, 0.0, 0.5e-6), hi=(1.0, 1.0, 2e-6)),                 # outside the box
           hv(lo=(0.0, 0.0, 0.6e-6), hi=(1.0, 1.0, 0.5e-6)),               # empty
           W.with_(cell, **{"problem.heat": {"lo": (100e-9, 0.0, 0.0), "hi": (200e-9, 500e-9, 500e-9),
                                             "t": np.array([0.0, 1e-12]), "P": np.array([1e16])}})]   # the pore
    for w in bad:
        assert _status(w) == M.mcbte.EINVAL
        with pytest.raises(ValueError):
            oracle.Tables(w)
    beside = W.with_(cell, **{"problem.heat": {"lo": (0.0, 0.0, 0.0), "hi": (100e-9, 500e-9, 500e-9),
                                               "t": np.array([0.0, 1e-12]), "P": np.array([1e16])}})
    assert _status(beside) == 0
    oracle.Tables(beside)
    # regions built from tetrahedra: inside the box, positive volume, clear of the pores
    box = W.heated_box(N=10)
    assert _status(box) == 0
    tet = np.asarray(box["problem"]["heat"]["tets"][0])

    def with_tets(w, tets):
        w = W.with_(w)
        w["problem"]["heat"] = dict(w["problem"]["heat"], tets=np.asarray(tets, dtype=np.float64))
        return w
    flat = tet.copy()
    flat[3] = flat[0]                                                               # no volume
    outside = tet.copy()
    outside[3, 2] = 250e-9                                                          # the box is 200 nm high
    in_pore = np.array([[200e-9, 200e-9, 10e-9], [300e-9, 220e-9, 10e-9], [220e-9, 320e-9, 10e-9],
                        [230e-9, 230e-9, 100e-9]])
    nan = tet.copy()
    nan[1, 0] = np.nan
    for w in (with_tets(box, [flat]), with_tets(box, [outside]), with_tets(box, [nan]),
              with_tets(W.with_(cell, **{"problem.heat": {"lo": (0.0, 0.0, 0.0), "hi": (100e-9, 500e-9, 500e-9),
                                                          "t": np.array([0.0, 1e-12]), "P": np.array([1e16])}}),
                        [in_pore])):
        assert _status(w) == M.mcbte.EINVAL
        with pytest.raises(ValueError):
            oracle.Tables(w)
    cubes = with_tets(box, W.cube_tets((50e-9, 40e-9, 30e-9), (350e-9, 240e-9, 130e-9)))
    t6 = M.Tables(cubes, device=-1)
    assert t6.info["E_tot"] == oracle.Tables(cubes).E_tot


def test_sizes_and_messages():
    assert M.state_bytes(32, 1000) == 9 * 4096 + 7 * 4096
    assert M.state_bytes(64, 1) == 16 * 256
    with pytest.raises(M.MCBTEError):
        M.state_bytes(16, 10)
    assert M.batch_queue_bytes(64) > 64 * 8 * 3
    assert M.strerror(0) == "ok"
    assert "geometry" in M.strerror(-6)
    tb = M.Tables(W.gray_slab(N=10), device=-1)
    out = np.zeros(1)
    assert M.lib().mcbte_table_export(tb.h, 3, out.ctypes.data_as(C.c_void_p), 0) == M.mcbte.ESIZE


def test_two_phonon_clock_inputs():
    """tau_imp: >= 0 and finite (0: no two-phonon process); the bulk kappa the tables report uses
    the summed rates, as the oracle's does; the sensitivity estimators refuse two-clock tables."""
    w = W.bulk_gradient(N=10, modes=W.silicon_like_modes(300.0, impurity_clock=True))
    for bad_val in (-1e-12, float("inf"), float("nan")):
        bad = W.with_(w)
        bad["modes"]["tau_imp"][3] = bad_val
        assert _status(bad) == M.mcbte.EINVAL
        with pytest.raises(ValueError):
            oracle.Tables(bad)
    t = M.Tables(w, device=-1)
    o = oracle.Tables(w)
    assert t.info["kappa_bulk"] == pytest.approx(o.kappa_bulk, rel=1e-13)
    one = M.Tables(W.bulk_gradient(N=10, modes=W.silicon_like_modes(300.0)), device=-1)
    assert t.info["kappa_bulk"] == pytest.approx(one.info["kappa_bulk"], rel=1e-12)
    run = M.make_run(1, 32)
    dummy = C.c_void_p(1)
    assert M.lib().mcbte_adjoint(t.h, C.byref(run), M.mcbte.SENS_SCORE, 0.0, 0, 10, dummy, dummy, None) \
        == M.mcbte.EINVAL


def test_specular_cutoff_inputs():
    """A boundary's cutoff frequency must be >= 0 and finite; the replays refuse such tables."""
    for bad_val in (-1.0, float("inf"), float("nan")):
        f = W.film(N=10, spec_omega=bad_val)
        assert _status(f) == M.mcbte.EGEOM
        with pytest.raises(ValueError):
            oracle.Tables(f)
        p = W.porous_cell(N=10, spec_omega=bad_val)
        assert _status(p) == M.mcbte.EGEOM
    t = M.Tables(W.film(N=10, spec_omega=W.OMEGA_2THZ), device=-1)
    run = M.make_run(1, 32)
    dummy = C.c_void_p(1)
    assert M.lib().mcbte_adjoint(t.h, C.byref(run), M.mcbte.SENS_SCORE, 0.0, 0, 10, dummy, dummy, None) \
        == M.mcbte.EINVAL


def test_line_wall_inputs():
    """Walls: adiabatic, inside the box, a unit normal, ids after the pores', a given volume; the
    host and the oracle refuse the same inputs; the replays refuse walled tables."""
    base = W.square_pore_cell(N=10)
    assert _status(base) == 0
    def bad(mutate):
        w = W.with_(base)
        mutate(w)
        return w
    cases = [
        lambda w: w["geometry"]["walls"].__setitem__(0, (0.0, 0.0, 6e-7, 0.0, 0.0, 1.0, 7, W.ADIABATIC, 0.0)),  # outside
        lambda w: w["geometry"]["walls"].__setitem__(0, w["geometry"]["walls"][0][:4] + (0.0, 0.5, 7, W.ADIABATIC, 0.0)),
        lambda w: w["geometry"]["walls"].__setitem__(1, w["geometry"]["walls"][1][:6] + (7, W.ADIABATIC, 0.0)),
        lambda w: w["geometry"]["walls"].__setitem__(0, w["geometry"]["walls"][0][:7] + (W.ISOTHERMAL, 0.0)),
    ]
    for mutate in cases:
        w = bad(mutate)
        assert _status(w) == M.mcbte.EGEOM
        with pytest.raises(ValueError):
            oracle.Tables(w)
    hot = W.walled_slab(N=10)
    assert _status(hot) == 0
    cold0 = W.with_(hot)
    cold0["geometry"]["walls"][0] = cold0["geometry"]["walls"][0][:8] + (0.0,)       # T_b must be > 0
    assert _status(cold0) == M.mcbte.EGEOM
    with pytest.raises(ValueError):
        oracle.Tables(cold0)
    assert M.Tables(hot, device=-1).info["n_sources"] == oracle.Tables(hot).S == 2
    novol = W.with_(base, **{"geometry.volume": 0.0})
    assert _status(novol) == M.mcbte.EINVAL
    t = M.Tables(base, device=-1)
    run = M.make_run(1, 32)
    dummy = C.c_void_p(1)
    assert M.lib().mcbte_adjoint(t.h, C.byref(run), M.mcbte.SENS_SCORE, 0.0, 0, 10, dummy, dummy, None) \
        == M.mcbte.EINVAL
