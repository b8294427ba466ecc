"""Unit pins of the CPU oracle's building blocks (no GPU)."""
import math
import os

import numpy as np
import pytest
from scipy import integrate, stats

import closed_forms as cf
import oracle
import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_philox_known_answers():
    """Philox4x32-10 against the published known-answer vectors (exact)."""
    rows = [l.split() for l in open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")) if not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        vals = [int(x, 16) for x in r if x != "->"]
        ctr, key, want = vals[0:4], vals[4:6], vals[6:10]
        assert [int(x) for x in oracle.philox(ctr, key)] == want


def test_record_layout_is_two_consecutive_blocks():
    seed, inst, pid, rec = 0x0123456789ABCDEF, 7, (5 << 32) + 11, 1234
    W8 = oracle.record(seed, inst, pid, rec)
    key = [seed & 0xFFFFFFFF, seed >> 32]
    b0 = oracle.philox([2 * rec, pid & 0xFFFFFFFF, pid >> 32, inst], key)
    b1 = oracle.philox([2 * rec + 1, pid & 0xFFFFFFFF, pid >> 32, inst], key)
    assert list(W8) == list(b0) + list(b1)


def test_philox_stream_uniformity():
    """chi^2 of the top 4 bits of 8 * 20000 words from consecutive records and particles."""
    words = np.concatenate([oracle.record(W.SEED_BASE, 0, pid, r) for pid in range(2000) for r in range(10)])
    hist = np.bincount(words >> 28, minlength=16)
    p = stats.chisquare(hist).pvalue
    assert p > 1e-4, p


def _linear_pick(thr, last, K):
    for j, t in enumerate(thr):
        if K < int(t):
            return j
    return last


def test_cdf_inversion_edges_and_zero_weights():
    w = np.array([0.0, 1.0, 0.0, 0.0, 2.0, 1e-300, 0.5, 0.0, 0.0])
    thr, last = oracle.cdf_build(w)
    assert last == 6
    assert int(thr[-1]) == 2 ** 64 - 1 and int(thr[6]) == 2 ** 64 - 1
    # edges: K = thr_j - 1 picks j (or earlier), K = thr_j picks a later bin
    for j in range(len(w)):
        t = int(thr[j])
        if 0 < t < 2 ** 64 - 1:
            assert oracle.cdf_pick(thr, last, t - 1) == _linear_pick(thr, last, t - 1) <= j
            assert oracle.cdf_pick(thr, last, t) == _linear_pick(thr, last, t) > j
    assert oracle.cdf_pick(thr, last, 2 ** 64 - 1) == last
    assert oracle.cdf_pick(thr, last, 0) == 1
    rng = np.random.default_rng(1)
    for K in rng.integers(0, 2 ** 63, 4000, dtype=np.uint64):
        K = int(K) * 2 + int(rng.integers(0, 2))
        j = oracle.cdf_pick(thr, last, K)
        assert j == _linear_pick(thr, last, K)
        assert w[j] > 0.0


def test_cdf_frequencies_match_weights():
    rng = np.random.default_rng(2)
    w = rng.random(40) ** 3
    thr, last = oracle.cdf_build(w)
    Ks = rng.integers(0, 2 ** 64 - 1, 200000, dtype=np.uint64, endpoint=True)
    # vectorised definition: first j with K < thr_j
    picks = np.searchsorted(thr, Ks, side="right")
    picks = np.where(picks >= len(w), last, picks)
    for K in Ks[:500]:
        assert oracle.cdf_pick(thr, last, int(K)) == int(np.searchsorted(thr, K, side="right"))
    hist = np.bincount(picks, minlength=len(w))
    p = stats.chisquare(hist, w / w.sum() * len(Ks)).pvalue
    assert p > 1e-4, p


def test_tiny_probability_bin_is_reachable_with_64_bit_keys():
    """Bins far below 2^-32 (relaxation bins reach ~1e-17) keep a non-empty key interval."""
    w = np.array([1e-17, 1.0])
    thr, last = oracle.cdf_build(w)
    assert 0 < int(thr[0]) < 2 ** 64 // 10 ** 15
    assert oracle.cdf_pick(thr, last, int(thr[0]) - 1) == 0


def test_isotropic_directions_moments():
    rng = np.random.default_rng(3)
    u = rng.random((40000, 2))
    d = np.array([oracle.dir_iso(a, b) for a, b in u])
    n = len(d)
    assert np.allclose(np.linalg.norm(d, axis=1), 1.0, atol=1e-15)
    se = np.sqrt(1.0 / 3.0 / n)
    assert np.all(np.abs(d.mean(0)) < 4 * se)
    se2 = np.sqrt((1 / 5 - 1 / 9) / n)                    # Var(mu^2) for mu uniform on [-1, 1]
    assert np.all(np.abs((d ** 2).mean(0) - 1 / 3) < 4 * se2)


@pytest.mark.parametrize("normal", [(0, 0, 1), (0, 0, -1), (1, 0, 0), (0, -1, 0), (0.6, -0.8, 0.0),
                                    (0.2, 0.3, -0.9327379053088815)])
def test_cosine_weighted_directions(normal):
    n = np.array(normal, dtype=float)
    n /= np.linalg.norm(n)
    rng = np.random.default_rng(4)
    u = rng.random((30000, 2))
    d = np.array([oracle.dir_cos(a, b, n) for a, b in u])
    N = len(d)
    assert np.allclose(np.linalg.norm(d, axis=1), 1.0, atol=1e-14)
    mu = d @ n
    assert np.all(mu >= 0.0)
    # Lambert law: p(mu) = 2 mu -> E[mu] = 2/3, E[mu^2] = 1/2
    assert abs(mu.mean() - 2 / 3) < 4 * np.sqrt((1 / 2 - 4 / 9) / N)
    assert abs((mu ** 2).mean() - 1 / 2) < 4 * np.sqrt((1 / 3 - 1 / 4) / N)
    # no preferred azimuth: tangential components average to zero
    tang = d - mu[:, None] * n[None, :]
    assert np.all(np.abs(tang.mean(0)) < 4 * np.sqrt(0.25 / N))


@pytest.mark.parametrize("T", [50.0, 100.0, 300.0, 400.0])
def test_dedT_is_derivative_of_bose_einstein_energy(T):
    for w in np.geomspace(1e10, 7.5e13, 25):
        h = 1e-4 * T
        fd = (cf.bose_einstein_energy(w, T + h) - cf.bose_einstein_energy(w, T - h)) / (2 * h)
        assert oracle.dedT(w, T) == pytest.approx(fd, rel=1e-7)


def test_heat_capacity_per_row_matches_exact_bin_integral():
    """C_m (first format: DOS x delta-omega x de/dT) equals the exact integral of the continuous
    dispersion over the bin up to the midpoint-rule error.  For the omega^2 leading behaviour
    of the integrand that error is -1/(12 (i + 1/2)^2 + 1) in bin i; rows near the zone edge
    (1/v singularity of the DOS) are excluded."""
    T = 300.0
    w = W.film(N=10)
    tb = oracle.Tables(w)
    Cm = tb.get("C")
    m = w["modes"]
    k_max = 2 * math.pi / W.A_SI
    a = math.pi / k_max
    checked = 0
    for i in list(range(0, 12)) + list(range(12, len(m), 37)):
        wm = W.OMEGA_MAX_LA if m["branch"][i] == 1 else W.OMEGA_MAX_TA
        g = 1.0 if m["branch"][i] == 1 else 2.0
        lo, hi = m["omega"][i] - 0.5 * m["domega"][i], m["omega"][i] + 0.5 * m["domega"][i]
        if hi > 0.8 * wm:
            continue
        k_of = lambda om: (2 / a) * math.asin(om / wm)

        def f(k):
            om = wm * math.sin(0.5 * a * k)
            x = cf.HBAR * om / (cf.KB * T)
            return g * k * k / (2 * math.pi ** 2) * cf.KB * (x / 2) ** 2 / math.sinh(x / 2) ** 2

        exact = integrate.quad(f, k_of(lo), k_of(hi), epsrel=1e-12)[0]
        mid_err = 1.0 / (12.0 * (m["bin"][i] + 0.5) ** 2 + 1.0)
        assert abs(Cm[i] / exact - 1.0 + mid_err) < 0.05 * mid_err + 2e-5, i
        checked += 1
    assert checked > 20


def test_bulk_kappa_matches_continuous_integral():
    tb = oracle.Tables(W.film(N=10))
    C_int, k_int = cf.dispersion_integrals(300.0)
    assert tb.kappa_bulk == pytest.approx(k_int, rel=1e-3)
    # the binned heat capacity is below the continuous one only through the 1/v zone-edge
    # singularity of the DOS, which the centre-of-bin rows under-sample
    assert 0.95 < tb.C_tot / C_int < 1.0


def _brute_segment(tb, w, x0, o, d, m, s=1.0, n=200000):
    det = w["detectors"]
    raw = np.zeros(tb.raw_size).reshape(tb.n_cells, tb.n_cols, 4)
    ts = (np.arange(n) + 0.5) * (d / n)
    x = x0[None, :] + ts[:, None] * o[None, :]
    inside = np.ones(n, bool)
    idx = np.zeros(n, np.int64)
    for a in range(3):
        nb = det["n"][a]
        if nb > 0:
            inside &= (x[:, a] >= det["lo"][a]) & (x[:, a] <= det["hi"][a])
            ci = np.clip(np.floor((x[:, a] - det["lo"][a]) / ((det["hi"][a] - det["lo"][a]) / nb)), 0, nb - 1)
            idx = idx * nb + ci.astype(np.int64)
    v = w["modes"]["v"][m]
    for c, cnt in zip(*np.unique(idx[inside], return_counts=True)):
        l = cnt * d / n
        raw[c, m] += [s * l / v, s * l * o[0], s * l * o[1], s * l * o[2]]
    return raw.ravel()


def test_steady_segment_clipping_matches_brute_force():
    w = W.gray_slab(N=10)
    w3 = W.with_(w, **{"detectors.lo": (0.0, 0.0, 0.0), "detectors.hi": (3e-8, 2e-8, 1e-7),
                       "detectors.n": (3, 2, 5)})
    rng = np.random.default_rng(5)
    for ww in (w, w3):
        tb = oracle.Tables(ww)
        det = ww["detectors"]
        for k in range(40):
            x0 = rng.random(3) * np.array([4e-8, 3e-8, 1e-7]) - np.array([5e-9, 5e-9, 0])
            o = rng.normal(size=3)
            o /= np.linalg.norm(o)
            if k % 2:   # start exactly on an outer face or an interior plane of the grid
                a = int(rng.integers(0, 3))
                nb = max(det["n"][a], 1)
                x0[a] = det["lo"][a] + (det["hi"][a] - det["lo"][a]) * int(rng.integers(0, nb + 1)) / nb
            d = rng.random() * 8e-8
            got = tb.segment(x0, o, d, 0, -1.0)
            want = _brute_segment(tb, ww, x0, o, d, 0, -1.0)
            assert np.allclose(got, want, atol=2e-5 * d, rtol=0), (x0, o, d)


def _march(w, x, o, step):
    """First boundary met by marching along the ray (brute force): returns (distance, id)."""
    g = w["geometry"]
    L = np.array(g["L"])
    face_of = {(1, 0): 1, (0, 1): 2, (1, 1): 3, (0, 0): 4, (2, 0): 5, (2, 1): 6}
    ks = np.arange(1, 500000, dtype=np.float64)
    P = x[None, :] + o[None, :] * (ks * step)[:, None]
    first, who = np.inf, 0
    for a in range(3):
        if g["unbounded"][a]:
            continue
        for side, bad in ((0, P[:, a] < 0), (1, P[:, a] > L[a])):
            idx = np.flatnonzero(bad)
            if idx.size and ks[idx[0]] * step < first:
                first, who = ks[idx[0]] * step, face_of[(a, side)]
    for (cx, cy, r, cid) in (c[:4] for c in g["cylinders"]):
        idx = np.flatnonzero((P[:, 0] - cx) ** 2 + (P[:, 1] - cy) ** 2 < r * r)
        if idx.size and ks[idx[0]] * step < first:
            first, who = ks[idx[0]] * step, cid
    return first, who


def test_next_boundary_matches_ray_march():
    """Box faces and the z-axis cylinder: distance and id of the first boundary hit."""
    w = W.porous_cell(N=10)
    tb = oracle.Tables(w)
    cx, cy, r = w["geometry"]["cylinders"][0][:3]
    Wd = w["geometry"]["L"][0]
    rng = np.random.default_rng(6)
    n_cyl = 0
    step = 2e-12
    for _ in range(120):
        while True:
            x = rng.random(3) * Wd
            if (x[0] - cx) ** 2 + (x[1] - cy) ** 2 > r * r:
                break
        o = rng.normal(size=3)
        o /= np.linalg.norm(o)
        d, hit = tb.next_boundary(x, o)
        dm, hm = _march(w, x, o, step)
        assert hit == hm and abs(d - dm) <= step, (x, o, d, hit, dm, hm)
        n_cyl += hit == 7
    assert n_cyl > 20
    # a ray leaving the cylinder surface outward does not hit it again
    x = np.array([cx + r, cy, 1e-7])
    d, hit = tb.next_boundary(x, np.array([1.0, 0.0, 0.0]))
    assert hit == 2 and d == pytest.approx(Wd - cx - r)
    # an axis-parallel ray misses the cylinder
    d, hit = tb.next_boundary(np.array([1e-8, 1e-8, 2e-7]), np.array([0.0, 0.0, -1.0]))
    assert hit == 5 and d == pytest.approx(2e-7)
    # a corner: equal distances to two faces resolve to the lower id
    d, hit = tb.next_boundary(np.array([Wd - 1e-8, 1e-8, 3e-7]), np.array([1.0, -1.0, 0.0]) / math.sqrt(2))
    assert hit == 1


@pytest.mark.parametrize("cap", [1, 5])
def test_segment_cap_ends_each_walk_after_cap_segments(cap):
    """The per-particle segment cap: no particle takes more than `cap` segments; a particle that
    has not ended otherwise by then ends there (counted as a cap end), and the event log records
    exactly `cap` segment-ending events before the cap event for those particles."""
    w = W.with_(W.porous_cell(N=400, modes=W.gray_modes(6400.0, 5e-6 / 6400.0), n_scat_max=3),
                **{"problem.format": 2, "problem.max_events": cap})
    r = oracle.trace(w, n_log=400, log_stride=32, threads=4)
    c = dict(zip(oracle.COUNT_NAMES, (int(x) for x in r["counts"])))
    assert c["flights"] <= cap * c["particles"]
    ended = c["nscat_end"] + c["cap_end"] + c["absorbed"] + c["escaped"] + c["timeouts"]
    assert ended == c["particles"]
    assert c["cap_end"] > 0
    cap_code = next(k for k, v in oracle.EV_NAMES.items() if v == "cap_end")
    n_cap = 0
    for row in r["log"]:
        n = int(row[0])
        kinds = [int(e) >> 28 for e in row[1:1 + n]]
        if kinds and kinds[-1] == cap_code:
            # the emission, one event closing each of the `cap` segments, then the cap
            assert len(kinds) == cap + 2
            n_cap += 1
    assert n_cap == c["cap_end"]


def _march_walls(w, x, o, step):
    """First boundary met by marching: box faces as in _march, line walls by a sign change of the
    signed distance to the wall's line while the projection falls on the segment."""
    first, who = _march(w, x, o, step)
    ks = np.arange(1, 500000, dtype=np.float64)
    P = x[None, :] + o[None, :] * (ks * step)[:, None]
    for (x1, y1, x2, y2, nx, ny, wid) in (c[:7] for c in w["geometry"]["walls"]):
        if o[0] * nx + o[1] * ny >= 0.0:
            continue                       # met only from the side the normal points to
        s0 = (x[0] - x1) * nx + (x[1] - y1) * ny
        sd = (P[:, 0] - x1) * nx + (P[:, 1] - y1) * ny
        e = np.array([x2 - x1, y2 - y1])
        t = ((P[:, 0] - x1) * e[0] + (P[:, 1] - y1) * e[1]) / (e @ e)
        idx = np.flatnonzero((np.sign(sd) != np.sign(s0)) & (t >= 0) & (t <= 1))
        if idx.size and ks[idx[0]] * step < first:
            first, who = ks[idx[0]] * step, wid
    return first, who


def test_next_boundary_with_line_walls_matches_ray_march():
    """The square pore of four internal line walls (the paper's nanomesh layout): distance and id
    of the first boundary; walls are met only from the solid side."""
    w = W.square_pore_cell(N=10)
    tb = oracle.Tables(w)
    Wd = w["geometry"]["L"][0]
    a, b = 0.5 * (Wd - 250e-9), 0.5 * (Wd + 250e-9)
    rng = np.random.default_rng(7)
    n_wall = 0
    step = 2e-12
    for _ in range(120):
        while True:
            x = rng.random(3) * Wd
            if not (a < x[0] < b and a < x[1] < b):
                break
        o = rng.normal(size=3)
        o /= np.linalg.norm(o)
        d, hit = tb.next_boundary(x, o)
        dm, hm = _march_walls(w, x, o, step)
        assert hit == hm and abs(d - dm) <= step, (x, o, d, hit, dm, hm)
        n_wall += hit >= 7
    assert n_wall > 20
    # leaving a wall toward the solid: the wall is not met again
    d, hit = tb.next_boundary(np.array([0.5 * Wd, a, 1e-7]), np.array([0.0, -1.0, 0.0]))
    assert hit == 1 and d == pytest.approx(a)
    # from inside the pore (behind the walls) nothing but the box is met
    d, hit = tb.next_boundary(np.array([0.5 * Wd, 0.5 * Wd, 1e-7]), np.array([0.0, -1.0, 0.0]))
    assert hit == 1 and d == pytest.approx(0.5 * Wd)
