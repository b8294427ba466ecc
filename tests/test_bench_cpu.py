"""The benchmark's host-side contract (no GPU): the one-GPU guard and the algorithmic work model
behind its roofline figure."""
import math
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_algorithmic_work_model_counts_each_event_once():
    import bench
    O = bench.OPS
    info = {"n_modes": 1400, "n_sources": 3}
    geom = {"unbounded": (True, True, False), "cylinders": []}
    counts = {"particles": 10, "flights": 100, "relaxations": 60, "nscat_end": 10, "diffuse": 30,
              "rejections": 2}
    got = bench.algorithmic_lane_ops(counts, info, geom, ncomp=2, transient=False)
    steps_m, steps_s = math.ceil(math.log2(1401)), math.ceil(math.log2(4))
    emit = 10 * (4 * O["philox_block"] + (steps_s + steps_m) * O["search_step"] + O["cos_dir"]
                 + O["free_flight"] + O["emit_misc"])
    flights = 100 * (O["flight_base"] + 1 * O["face_axis"] + 2 * O["tally_comp"])
    relax = 50 * (2 * O["philox_block"] + steps_m * O["search_step"] + O["iso_dir"] + O["free_flight"])
    diffuse = 30 * (O["philox_block"] + O["cos_dir"])
    assert got == emit + flights + relax + diffuse + 2 * 2 * O["philox_block"]
    # a pore adds its ray test to every flight
    geom2 = {"unbounded": (False, False, False), "cylinders": [(0, 0, 1, 7, 2, 0.0)]}
    got2 = bench.algorithmic_lane_ops(counts, info, geom2, ncomp=2, transient=False)
    assert got2 - got == 100 * (2 * O["face_axis"] + O["pore"])


def test_traffic_figure_is_withheld_for_an_unprofiled_kernel():
    import bench
    assert bench.profiled_traffic("no_such_kernel_profile") is None


def test_work_model_adds_the_two_phonon_clock_draws():
    import bench
    O = bench.OPS
    info = {"n_modes": 1400, "n_sources": 3}
    geom = {"unbounded": (True, True, False), "cylinders": []}
    counts = {"particles": 10, "flights": 100, "relaxations": 60, "nscat_end": 10, "diffuse": 30,
              "rejections": 0, "two_phonon": 7}
    one = bench.algorithmic_lane_ops(counts, info, geom, ncomp=2, transient=False)
    two = bench.algorithmic_lane_ops(counts, info, geom, ncomp=2, transient=False, two_clocks=True)
    clock = O["philox_block"] + O["free_flight"]
    assert two - one == 7 * (O["philox_block"] + O["iso_dir"] + clock) + (10 + 50) * clock


def test_snapshot_count_only_where_it_is_fixed():
    """The transient bump (initial condition only, specular walls): every particle that reaches
    t_max scores each of the 200 measurement times once.  A heat source, a steady problem, or a
    particle that did not reach t_max leave the snapshots uncounted."""
    import bench
    import workloads as W
    w = W.transient_bump(N=1000)
    assert bench.exact_snapshots(w, {"timeouts": 1000, "particles": 1000}) == 1000 * 200
    assert bench.exact_snapshots(w, {"timeouts": 999, "particles": 1000}) == 0
    assert bench.exact_snapshots(W.heated_slab(N=10), {"timeouts": 10, "particles": 10}) == 0
    assert bench.exact_snapshots(W.film(N=10), {"timeouts": 0, "particles": 10}) == 0
    base = bench.algorithmic_lane_ops({"particles": 10, "flights": 100, "relaxations": 50, "nscat_end": 0,
                                       "diffuse": 0, "rejections": 0}, {"n_modes": 1400, "n_sources": 100},
                                      w["geometry"], 2, True)
    more = bench.algorithmic_lane_ops({"particles": 10, "flights": 100, "relaxations": 50, "nscat_end": 0,
                                       "diffuse": 0, "rejections": 0}, {"n_modes": 1400, "n_sources": 100},
                                      w["geometry"], 2, True, snapshots=2000, binned_axes=1)
    assert more - base == 2000 * (bench.OPS["snapshot_axis"] + 2 * bench.OPS["tally_comp"])


def test_lone_walker_is_one_long_walk_through_the_pore_lattice():
    """The lone-walker workload: one phonon of the pore cell whose free path (10 cm) spans ~1e5
    pore reflections, in the geometry the pore-lattice walk takes (periodic in x and y, one pore,
    no line walls), traced by the oracle on the CPU: a single relaxation ends it, and its pore
    reflections and periodic transfers number in the tens of thousands."""
    import bench
    import oracle
    w, name = bench.workload("lone_walker")
    assert w["problem"]["N"] == 1 and w["problem"]["n_scat_max"] == 1
    assert bench.is_pore_lattice(w)
    assert "Lambda10cm" in name
    lam = float(w["modes"]["v"][0] * w["modes"]["tau"][0])
    assert abs(lam - 0.1) < 1e-12
    c = oracle.trace(w)["counts"]
    particles, flights, relax, spec, diffuse, periodic = (int(x) for x in c[:6])
    assert particles == 1 and relax == 1 and spec == 0
    assert diffuse > 10_000 and periodic > diffuse
    assert flights == diffuse + periodic + relax
