"""Specularity per material row (section 3.5.3) in the FP32 form, through the C ABI, against the
FP64 oracle.  The FP64 form's event sequences are checked bit for bit with the other FP64 cases.

A boundary's per-row table gives each phonon its own reflection class: the film's wave-cooperative
bouncing runs only the rows whose walls are diffuse, and the pore lattice walks only the rows the
pore reflects either diffusely or specularly (partly specular rows step one segment at a time).
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


def test_fp32_film_with_ziman_specularity_against_the_oracle():
    """100 nm film, Ziman's roughness model (eta = 0.2 nm) per row, 2e5 particles: kappa within 2e-4
    of the oracle on the same particles, the specular and diffuse counts within 1e-4."""
    M = _pkg()
    w = W.film(N=200_000)
    w = W.with_spec_table(w, W.ziman_specularity(w["modes"], 0.2e-9))
    got = M.run(w, precision=32)
    ref = oracle.run(w, threads=THREADS)
    rel = abs(got["kappa"] - ref["kappa"]) / abs(ref["kappa"])
    c, r = got["counts"], ref["counts"]
    _say(f"[spec table, FP32 film] kappa {got['kappa']:.6g} vs {ref['kappa']:.6g} (rel {rel:.2e}); specular "
         f"{c['specular']} / {r['specular']}, diffuse {c['diffuse']} / {r['diffuse']}")
    assert rel <= 2e-4
    for k in ("specular", "diffuse"):
        assert abs(c[k] - r[k]) <= 1e-4 * r[k] + 2
    assert c["particles"] == r["particles"] and c["relaxations"] == r["relaxations"]


@pytest.mark.parametrize("binary", [True, False])
def test_fp32_pore_lattice_with_per_row_specularity(binary):
    """The 500 nm periodic cell, pore specularity per row (0 / 1 at random: every row walked from pore
    to pore; or random in [0, 1): partly specular rows step one segment at a time), 4e5 particles:
    the walk, the one-segment FP32 stepping and the FP64 oracle trace the same particles (counts
    within 1 %, kappa within 3 standard errors), and the walk does not depend on the launch shape."""
    M = _pkg()
    w = W.porous_cell(N=400_000)
    w = W.with_spec_table(w, W.random_specularity(len(w["modes"]), 21, binary=binary))
    got = M.run(w, precision=32)
    seg = M.run(w, precision=32, segments=True)
    ref = oracle.run(w, threads=THREADS)
    r = ref["counts"]
    for name, x in (("walk", got), ("segments", seg)):
        c = x["counts"]
        _say(f"[spec table, FP32 cell, binary={binary}] {name}: kappa {x['kappa']:.5g} vs {ref['kappa']:.5g} "
             f"(sigma {ref['kappa_sigma']:.3g}); specular {c['specular']} / {r['specular']}, diffuse "
             f"{c['diffuse']} / {r['diffuse']}")
        for k in ("particles", "relaxations", "nscat_end"):
            assert c[k] == r[k], (name, k)
        for k in ("flights", "periodic", "specular", "diffuse"):
            assert abs(c[k] - r[k]) <= 0.01 * r[k] + 5, (name, k)
        assert abs(x["kappa"] - ref["kappa"]) < 3.0 * ref["kappa_sigma"]
    shape = M.run(w, precision=32, block=64, refill=1)
    assert np.array_equal(shape["counts_raw"], got["counts_raw"])


@pytest.mark.parametrize("cap", [0, 60])
def test_fp32_specular_film_crossings_run_at_once(cap):
    """A 20 nm film whose walls reflect specularly (d = 1; and the rows below 2 THz of a cutoff
    film): the FP32 trace runs a phonon's wall-to-wall crossings up to the end of its free path at
    once.  The counters match the oracle's (specular reflections and segments within 1e-4, the
    cap's ends within a few when a cap of 60 segments cuts the longest paths), kappa within 2e-4."""
    M = _pkg()
    extra = {"problem.max_events": cap} if cap else {}
    for w in (W.with_(W.film(N=200_000, d=20e-9, specularity=1.0), **extra),
              W.with_(W.film(N=200_000, d=20e-9, spec_omega=W.OMEGA_2THZ), **extra)):
        got = M.run(w, precision=32)
        ref = oracle.run(w, threads=THREADS)
        c, r = got["counts"], ref["counts"]
        rel = abs(got["kappa"] - ref["kappa"]) / abs(ref["kappa"])
        _say(f"[specular crossings, cap {cap}] d={w['geometry']['faces'][5][1]}: kappa rel {rel:.2e}; specular "
             f"{c['specular']} / {r['specular']}, flights {c['flights']} / {r['flights']}, cap_end {c['cap_end']} / "
             f"{r['cap_end']}")
        assert r["specular"] > 0.5 * w["problem"]["N"]
        for k in ("specular", "flights"):
            assert abs(c[k] - r[k]) <= 1e-4 * r[k] + 2, k
        for k in ("particles", "relaxations", "nscat_end", "diffuse"):
            assert abs(c[k] - r[k]) <= 1e-4 * r[k] + 2, k
        assert abs(c["cap_end"] - r["cap_end"]) <= 1e-3 * r["cap_end"] + 3
        if cap:
            assert r["cap_end"] > 20
        assert rel <= 2e-4


@pytest.mark.parametrize("d", [0.3, 0.9])
def test_fp32_partly_specular_film_bounces_by_the_wave(d):
    """Partly specular film walls (constant d): the FP32 trace hands a long free path's bounces to
    the whole wave, each lane deciding its reflection by its own record and a specular one keeping
    the last diffuse direction with the film-axis component flipped.  Against the oracle on the
    same particles: specular and diffuse counts and segments within 1e-4, kappa within 2e-4; a cap
    of 40 segments ends the same particles."""
    M = _pkg()
    for cap in (0, 40):
        w = W.film(N=200_000, d=20e-9, specularity=d)
        if cap:
            w = W.with_(w, **{"problem.max_events": cap})
        got = M.run(w, precision=32)
        ref = oracle.run(w, threads=THREADS)
        c, r = got["counts"], ref["counts"]
        rel = abs(got["kappa"] - ref["kappa"]) / abs(ref["kappa"])
        _say(f"[partly specular film d={d} cap={cap}] kappa rel {rel:.2e}; specular {c['specular']} / {r['specular']}, "
             f"diffuse {c['diffuse']} / {r['diffuse']}, flights {c['flights']} / {r['flights']}, cap_end "
             f"{c['cap_end']} / {r['cap_end']}")
        for k in ("specular", "diffuse", "flights", "relaxations"):
            assert abs(c[k] - r[k]) <= 1e-4 * r[k] + 2, k
        assert abs(c["cap_end"] - r["cap_end"]) <= 1e-3 * r["cap_end"] + 3
        assert rel <= 2e-4
