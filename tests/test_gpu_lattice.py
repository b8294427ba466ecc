"""The FP32 form's pore-to-pore walk of long free paths through a periodic lattice of pores.

A cell periodic in x and y with one pore tiles a lattice; a transfer through a periodic face
reinserts the particle unchanged at the partner face (Eq. periodic_lin_final), i.e. the particle
flies on through the lattice.  The FP32 kernel follows a particle with a long free path from pore
to pore with its whole wave, counting the transfers from the cells crossed.  These tests check
that walk against the oracle's one-segment-at-a-time trajectories (FP64) and against the FP32
kernel stepping one segment at a time (MCBTE_RUN_SEGMENTS), through the C ABI.
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


def _gray_lattice(lam, N, r=None, spec=0.0, n_scat_max=3, **extra):
    w = W.porous_cell(N=N, modes=W.gray_modes(6400.0, lam / 6400.0), specularity=spec, n_scat_max=n_scat_max)
    changes = {"problem.format": 2}
    if r is not None:
        cyl = list(w["geometry"]["cylinders"][0])
        cyl[2] = r
        changes["geometry.cylinders"] = [tuple(cyl)]
    changes.update(extra)
    return W.with_(w, **changes)


def test_walk_counts_the_transfers_of_nearly_straight_flights_like_the_oracle():
    """A pore of 2 nm in the 500 nm cell: free paths of 20 um (tens to thousands of cells) seldom
    meet it, so the number of periodic transfers is a property of the flights' lines, and a
    flight that does meet it leaves with a direction close to the oracle's (the same random
    numbers; a hit point on so small a pore carries FP32 rounding of about 1e-3 of its radius).
    The walk counts the transfers from the cells crossed, the oracle steps face to face in FP64,
    the FP32 one-segment stepping beside it: the counts agree to a few 1e-4."""
    M = _pkg()
    w = _gray_lattice(20e-6, 20000, r=2e-9)
    got = M.run(w, precision=32)
    seg = M.run(w, precision=32, segments=True)
    ref = oracle.run(w, threads=THREADS)
    c, s, r = got["counts"], seg["counts"], ref["counts"]
    _say(f"[walk, nearly straight flights] periodic {c['periodic']} / segments {s['periodic']} / oracle "
         f"{r['periodic']}; flights {c['flights']} / {s['flights']} / {r['flights']}; pore hits {c['diffuse']} / "
         f"{s['diffuse']} / {r['diffuse']}")
    for k in ("particles", "relaxations", "nscat_end", "rejections"):
        assert c[k] == r[k], k
    assert c["periodic"] > 100 * w["problem"]["N"]
    assert r["diffuse"] > 1000
    # (measured: walk 2e-4, one-segment FP32 stepping 5e-4 -- a particle whose pore hits differ from the
    # oracle's draws its later records at other indices, so agreement is to the few that do)
    for x in (c, s):
        assert abs(x["periodic"] - r["periodic"]) <= 1e-3 * r["periodic"]
        assert abs(x["flights"] - r["flights"]) <= 1e-3 * r["flights"]
        assert abs(x["diffuse"] - r["diffuse"]) <= 0.02 * r["diffuse"] + 10
    assert c["escaped"] == 0 and c["cap_end"] == 0


@pytest.mark.parametrize("spec", [0.0, 1.0])
def test_walk_against_oracle_and_segment_stepping(spec):
    """Free paths of 20 um between diffuse or specular pores (the lattice a dispersing billiard):
    the FP32 walk, the FP32 one-segment stepping and the FP64 oracle trace the same particles;
    trajectories part after some reflections (FP32 rounding grows by flight length over pore radius
    at each), so the counts agree statistically (1 %) and kappa within 3 oracle standard errors."""
    M = _pkg()
    w = _gray_lattice(20e-6, 40000, spec=spec)
    got = M.run(w, precision=32)
    seg = M.run(w, precision=32, segments=True)
    ref = oracle.run(w, threads=THREADS)
    r = ref["counts"]
    hits = lambda x: x["diffuse"] + x["specular"]
    for name, x in (("walk", got), ("segments", seg)):
        c = x["counts"]
        _say(f"[walk vs oracle] spec {spec} {name}: kappa {x['kappa']:.5g} vs {ref['kappa']:.5g} "
             f"(sigma {ref['kappa_sigma']:.3g}); periodic {c['periodic']} vs {r['periodic']}, "
             f"pore hits {hits(c)} vs {hits(r)}")
        for k in ("particles", "relaxations", "nscat_end", "rejections"):
            assert c[k] == r[k], (name, k)
        for k in ("flights", "periodic"):
            assert abs(c[k] - r[k]) <= 0.01 * r[k], (name, k)
        assert abs(hits(c) - hits(r)) <= 0.01 * hits(r) + 5
        assert c["escaped"] == 0 and c["cap_end"] == 0
        assert abs(x["kappa"] - ref["kappa"]) < 3.0 * ref["kappa_sigma"]
    assert got["counts"]["periodic"] > 20 * w["problem"]["N"]


def test_walk_does_not_depend_on_the_launch_shape():
    """The walk depends only on the walked particle (its own random stream), not on which lanes
    share its wave: the counters and particle scores are the same for three launch shapes (one of
    them a one-wave grid, where lanes also walk alone), the tally sums to rounding of the atomics;
    the same with the phonons below 2 THz reflected specularly (the class is per phonon)."""
    M = _pkg()
    for w in (_gray_lattice(50e-6, 3000), W.porous_cell(N=200000),
              W.porous_cell(N=100000, spec_omega=W.OMEGA_2THZ)):
        base = M.run(w, precision=32)
        for shape in ({"block": 64, "refill": 1}, {"block": 256, "refill": 32, "grid": 2}):
            r = M.run(w, precision=32, **shape)
            assert np.array_equal(r["counts_raw"], base["counts_raw"]), shape
            scale = np.abs(base["raw"]).max()
            assert np.abs(r["raw"] - base["raw"]).max() <= 1e-10 * scale
            assert np.allclose(r["moments"], base["moments"], rtol=1e-10,
                               atol=1e-10 * np.abs(base["moments"]).max())


def test_walk_stops_short_of_the_segment_cap():
    """A cap of 300 segments with free paths of hundreds of cells: the walk hands the particle to
    the one-segment step once a step could pass the cap, and that step ends it at the cap, as the
    oracle does (flights past a 2 nm pore, nearly all of them straight lines)."""
    M = _pkg()
    w = _gray_lattice(200e-6, 5000, r=2e-9, **{"problem.max_events": 300})
    got = M.run(w, precision=32)
    ref = oracle.run(w, threads=THREADS)
    c, r = got["counts"], ref["counts"]
    _say(f"[walk, cap 300] cap_end {c['cap_end']} / {r['cap_end']}, flights {c['flights']} / {r['flights']}")
    assert r["cap_end"] > 0.3 * w["problem"]["N"]
    assert abs(c["cap_end"] - r["cap_end"]) <= 3e-3 * r["cap_end"] + 2
    assert c["flights"] <= 300 * w["problem"]["N"]
    assert abs(c["flights"] - r["flights"]) <= 1e-3 * r["flights"]


def test_segments_flag_and_the_pathwise_replay():
    """The pathwise replay carries its tangents through every segment, so an FP32 pore lattice
    needs its forward trace and replay stepped one segment at a time: without the flag the library
    refuses; with it (the binding's default for that estimator) the replay runs.  The flag word is
    checked (unknown bits are refused)."""
    import torch
    M = _pkg()
    w = _gray_lattice(100e-9, 2000)
    t = M.Tables(w)
    F = torch.zeros(2000, dtype=torch.float64, device="cuda")
    adj = torch.zeros(t.info["adj_doubles"], dtype=torch.float64, device="cuda")
    tl = t.new_tally()
    M.trace(t, M.make_run(int(w["seed"]), 32, particle_F=F), 0, 2000, None, tl)
    with pytest.raises(M.MCBTEError) as e:
        M.adjoint(t, M.make_run(int(w["seed"]), 32), M.ESTIMATORS["pathwise"], 0, 2000, F, adj)
    assert e.value.status == M.mcbte.EINVAL
    out = M.sensitivities(w, precision=32, estimator="pathwise", tables=t)
    assert np.isfinite(out["dkappa_dlntau"]).all()
    bad = M.make_run(int(w["seed"]), 32)
    bad.flags = 2
    with pytest.raises(M.MCBTEError):
        M.trace(t, bad, 0, 100, None, tl)


def test_long_first_flights_started_first_change_no_count():
    """Particles whose first free flight passes 1000 cell widths are listed before the trace and
    started first (their walks then run beside the others).  Order changes no particle: gray
    medium with a 100 um mean free path, where e^-5 of the first flights qualify.  One call over
    1e6 particles (6700 listed: more than the list holds, so the scheduling is off) and two calls
    over its halves (3400 listed each, scheduled) give the same counters; so do launch shapes; the
    listed count is the qualifying share (binomial, 5 sigma)."""
    import math
    M = _pkg()
    w = _gray_lattice(100e-6, 1_000_000, n_scat_max=2)
    t = M.Tables(w)
    whole = M.run(w, precision=32, tables=t)
    tl = t.new_tally()
    listed = []
    for first in (0, 500_000):
        M.trace(t, M.make_run(int(w["seed"]), 32), first, 500_000, None, tl)
        listed.append(int(tl[200:208].view(__import__("torch").int64).item()))
    halves = M.tally(t, tl)
    p = math.exp(-5.0)
    _say(f"[scheduling] listed {listed} of 500000 each (expected {500000 * p:.0f}); counts {whole['counts']}")
    for k in listed:
        assert abs(k - 500000 * p) < 5.0 * math.sqrt(500000 * p * (1 - p))
        assert k <= 4096
    assert np.array_equal(halves["counts_raw"], whole["counts_raw"])
    assert abs(halves["kappa"] - whole["kappa"]) <= 1e-9 * abs(whole["kappa"])
    small = W.with_(w, **{"problem.N": 300_000})
    base = M.run(small, precision=32, tables=t)
    for shape in ({"block": 64, "refill": 1}, {"block": 256, "refill": 32, "grid": 2}):
        r = M.run(small, precision=32, tables=t, **shape)
        assert np.array_equal(r["counts_raw"], base["counts_raw"]), shape
    assert base["counts"]["particles"] == 300_000
