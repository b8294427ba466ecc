"""Pins of the oracle's specular reflection off curved and internal boundaries (section 3.5.3,
Eq. specular: the wave vector's normal component flips, the tangential one is kept).

Single particles are traced by the oracle in a box whose x faces are black isothermal walls (the
sources, and where every particle ends) and whose y faces are specular, around a specular pore or
a tilted square of specular line walls.  With tau -> infinity every trajectory is a deterministic
broken line, so each particle's raw track-length sums -- s * (time, displacement along x, y, z) --
are fixed by its emitted state alone.  A tracer written here, independently of the oracle's
formulas, follows the same line: boundary distances by its own constructions (the quadratic's
entering root for the cylinder, the signed distance to a wall's line and the position along it)
and reflections as mirror images by angle: the in-plane direction angle psi becomes 2 beta - psi
for a surface whose tangent has angle beta (beta = alpha + pi/2 on the cylinder, alpha the angle
of the normal at the hit point), with |Omega_xy| and Omega_z kept.  A wrong factor, normal or hit
point in the oracle's reflection changes the sums of the particles that meet the surface.
"""
import math

import numpy as np

import oracle
import workloads as W

V = 6400.0
L_BOX = 1.0e-6


def _box(extra_geometry: dict, volume: float = 0.0) -> dict:
    faces = {4: (W.ISOTHERMAL, 301.0, 0, 0), 2: (W.ISOTHERMAL, 299.0, 0, 0),
             1: (W.ADIABATIC, 1.0, 0, 0), 3: (W.ADIABATIC, 1.0, 0, 0)}
    g = W._geometry((L_BOX, L_BOX, 1.0), (False, False, True), faces, volume=volume, **extra_geometry)
    return {"name": "reflection_pin", "modes": W.gray_modes(V, 1.0), "geometry": g,
            "detectors": W._detectors(mask=W.MASK_ALL),
            "problem": W._problem(400, 300.0, 0, score_axis=0, fmt=2), "seed": W.SEED_BASE + 77}


def _mirror(o, beta):
    """o reflected in the line of angle beta (x-y plane), by angles."""
    rho = math.hypot(o[0], o[1])
    psi = math.atan2(o[1], o[0])
    psi2 = 2.0 * beta - psi
    return np.array([rho * math.cos(psi2), rho * math.sin(psi2), o[2]])


def _trace(x, o, cyl=None, walls=()):
    """Ballistic broken line until an x face absorbs it: (time, displacement, reflections)."""
    x = np.array(x, float)
    o = np.array(o, float)
    t, disp, n_ref = 0.0, np.zeros(3), 0
    for _ in range(100000):
        best = (math.inf, None, None)
        for a in (0, 1):
            if o[a] != 0.0:
                target = L_BOX if o[a] > 0.0 else 0.0
                s = (target - x[a]) / o[a]
                if s < best[0]:
                    best = (s, "face", a)
        if cyl is not None:
            cx, cy, r = cyl
            # |p + s q|^2 = r^2 with p = x - c, q = o (x-y parts): the smaller root enters
            px, py = x[0] - cx, x[1] - cy
            A = o[0] ** 2 + o[1] ** 2
            B = 2.0 * (px * o[0] + py * o[1])
            Cq = px * px + py * py - r * r
            disc = B * B - 4.0 * A * Cq
            if A > 0.0 and disc >= 0.0:
                s = (-B - math.sqrt(disc)) / (2.0 * A)
                if 0.0 < s < best[0]:
                    best = (s, "pore", None)
        for k, (x1, y1, x2, y2, nx, ny) in enumerate(walls):
            on = o[0] * nx + o[1] * ny
            if on >= 0.0:
                continue                         # met only from the side its normal points to
            h = (x[0] - x1) * nx + (x[1] - y1) * ny    # signed distance to the wall's line
            s = -h / on
            if s < 0.0:
                continue
            ln = math.hypot(x2 - x1, y2 - y1)
            ex, ey = (x2 - x1) / ln, (y2 - y1) / ln
            u = ((x[0] + s * o[0] - x1) * ex + (x[1] + s * o[1] - y1) * ey) / ln
            if 0.0 <= u <= 1.0 and s < best[0]:
                best = (s, "wall", k)
        s, kind, a = best
        t += s / V
        disp += s * o
        x = x + s * o
        if kind == "face":
            if a == 0:
                return t, disp, n_ref            # absorbed by an isothermal x wall
            o[1] = -o[1]                         # specular y face
            x[1] = L_BOX if x[1] > 0.5 * L_BOX else 0.0
        elif kind == "pore":
            alpha = math.atan2(x[1] - cyl[1], x[0] - cyl[0])
            o = _mirror(o, alpha + 0.5 * math.pi)
        else:
            x1, y1, x2, y2, _, _ = walls[a]
            o = _mirror(o, math.atan2(y2 - y1, x2 - x1))
        n_ref += 1
    raise AssertionError("trajectory did not end")


def _check_particles(w, cyl=None, walls=(), n=400):
    tb = oracle.Tables(w)
    met = 0
    worst = 0.0
    for pid in range(n):
        d8, i4 = tb.emit_state(pid)
        x0, o0, s = d8[0:3], d8[3:6], float(i4[1])
        assert abs(np.linalg.norm(o0) - 1.0) < 1e-14
        t, disp, n_ref = _trace(x0, o0, cyl, walls)
        raw, counts, _, _ = tb.trace_range(int(w["seed"]), 0, pid, 1, 0, 2)
        got = np.asarray(raw).reshape(-1)[:4]
        want = s * np.array([t, disp[0], disp[1], disp[2]])
        scale = max(np.abs(want).max(), 1e-30)
        err = np.abs(got - want).max() / scale
        worst = max(worst, err)
        assert err < 1e-9, (pid, got, want)
        assert int(counts[3]) == n_ref, (pid, int(counts[3]), n_ref)   # specular reflections
        assert int(counts[4]) == 0 and int(counts[6]) == 1
        # Omega_z is kept: the z displacement is Omega_z times the path length
        assert abs(disp[2] - o0[2] * V * t) <= 1e-12 * V * t
        met += n_ref > 0
    return met, worst


def test_specular_pore_reflection_is_a_mirror_image():
    """Pore of radius 300 nm in the middle of the 1 um box, specular: per particle, the oracle's
    time and displacement sums equal the independent tracer's (1e-9), reflection counts equal."""
    cyl = (0.5e-6, 0.5e-6, 0.3e-6)
    w = _box({"cylinders": [cyl + (7, W.ADIABATIC, 1.0, 0.0)]})
    met, worst = _check_particles(w, cyl=cyl)
    assert met > 100, met              # enough particles meet the pore (or the specular y faces)


def test_specular_line_walls_reflection_is_a_mirror_image():
    """A square of four specular line walls turned by 20 degrees (no wall along an axis), normals
    pointing out of the square into the solid: the same per-particle comparison."""
    c, h, th = 0.5e-6, 0.2e-6, math.radians(20.0)
    corners = [(c + h * (math.cos(th + k * math.pi / 2) - math.sin(th + k * math.pi / 2)),
                c + h * (math.sin(th + k * math.pi / 2) + math.cos(th + k * math.pi / 2))) for k in range(4)]
    walls = []
    for k in range(4):
        (x1, y1), (x2, y2) = corners[k], corners[(k + 1) % 4]
        mx, my = 0.5 * (x1 + x2) - c, 0.5 * (y1 + y2) - c
        ln = math.hypot(mx, my)
        walls.append((x1, y1, x2, y2, mx / ln, my / ln))
    rows = [wl + (7 + k, W.ADIABATIC, 1.0) for k, wl in enumerate(walls)]
    side = 2.0 * h
    w = _box({"walls": rows}, volume=(L_BOX * L_BOX - side * side) * 1.0)
    met, worst = _check_particles(w, walls=walls)
    assert met > 100, met


def test_specular_walled_channel_recovers_bulk():
    """A channel between two specular line walls does not resist flow along it: kappa of the
    gray medium equals the bulk value C v^2 tau / 3 (as the specular film does for faces)."""
    gray = W.gray_modes(V, 100e-9 / V)
    w = W.walled_film(N=100000, specularity=1.0, n_scat_max=1, modes=gray)
    w["problem"]["format"] = 2
    r = oracle.run(w, threads=8)
    k_ref = 1e6 * V ** 2 * (100e-9 / V) / 3.0
    assert abs(r["kappa"] - k_ref) < 3.0 * r["kappa_sigma"], (r["kappa"], r["kappa_sigma"], k_ref)
    assert r["counts"]["specular"] > 0 and r["counts"]["diffuse"] == 0
