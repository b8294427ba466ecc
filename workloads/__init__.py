"""Seeded synthetic workloads for the deviational phonon Monte Carlo tracer.

This module only *describes problems*: material rows in the form of the
paper's material-data file (section "MATLAB code I/O", material data), box
geometry and boundary table (same section, geometry and boundary
conditions), detector grids, run parameters and seeds.  It holds none of the
method's arithmetic (no heat capacities from the Bose-Einstein derivative, no
source energies, no distributions, no random draws).  Both the CPU oracle and
the HIP library consume exactly these descriptions, each through its own
binding.

Units are SI throughout (m, s, rad/s, J, K).

Face identifiers follow the paper's boundary-table order:
    1: y = 0,  2: x = Lx,  3: y = Ly,  4: x = 0,  5: z = 0,  6: z = Lz,
    7+: internal boundaries (here: z-axis cylindrical pores).
Boundary types follow the same table: 1 isothermal (data0 = T_b),
2 adiabatic (data0 = specularity d), 3 periodic (data = translation vector).
"""
from __future__ import annotations

import copy
import math

import numpy as np

ISOTHERMAL, ADIABATIC, PERIODIC = 1, 2, 3
FACE_AXIS_SIDE = {1: (1, 0), 2: (0, 1), 3: (1, 1), 4: (0, 0), 5: (2, 0), 6: (2, 1)}

MODE_DTYPE = np.dtype([
    ("omega", "f8"), ("dos", "f8"), ("v", "f8"), ("domega", "f8"),
    ("tau", "f8"), ("C", "f8"), ("tau_imp", "f8"), ("bin", "i4"), ("branch", "i4"),
])

# Tally component mask bits: T (energy / temperature), q_x, q_y, q_z.
MASK_T, MASK_QX, MASK_QY, MASK_QZ = 1, 2, 4, 8
MASK_ALL = 15

SEED_BASE = 0x4D43425445000000  # "MCBTE" followed by the config number

# Synthetic silicon-like dispersion of the frequency-dependent workloads:
# omega = omega_max * sin(k a / 2) per branch, zone edge k_max = 2 pi / a_Si,
# a = pi / k_max so that omega(k_max) = omega_max.
A_SI = 5.431e-10
OMEGA_MAX_LA = 7.5e13
OMEGA_MAX_TA = 3.0e13
TAU_A = 1.3e-45      # s^3     (impurity-like  A omega^4)
TAU_B = 1.7e-19      # s / K   (Umklapp-like   B omega^2 T exp(-C/T))
TAU_C = 137.0        # K
OMEGA_2THZ = 2.0 * math.pi * 2.0e12   # rad/s: the cutoff below which the paper's nanomesh reflects specularly


def silicon_like_modes(T: float, n_bins: int = 1000, impurity_clock: bool = False) -> np.ndarray:
    """Material rows of the synthetic silicon-like crystal at temperature T.

    Rows are in the paper's first material-data format (omega, DOS, V_g,
    delta-omega, tau, polarization): one LA row per frequency bin and one TA
    row (degeneracy 2 folded into the DOS) for every bin centre below the TA
    zone-edge frequency.  Bin i has centre (i + 1/2) * delta-omega with
    delta-omega = omega_max(LA) / n_bins.  The DOS of an isotropic branch is
    g k^2 / (2 pi^2 V_g) per unit volume and unit angular frequency; the
    relaxation time is 1 / (A omega^4 + B omega^2 T exp(-C/T)).  Heat
    capacities are *not* computed here (the method derives them from the DOS).

    impurity_clock: the impurity-like A omega^4 term becomes the separate two-phonon process
    (tau_imp = 1 / (A omega^4)) and tau keeps the Umklapp-like term alone (three-phonon).
    """
    k_max = 2.0 * math.pi / A_SI
    a_eff = math.pi / k_max
    dw = OMEGA_MAX_LA / n_bins
    rows = []
    for branch, (wmax, g) in enumerate(((OMEGA_MAX_LA, 1.0), (OMEGA_MAX_TA, 2.0))):
        for i in range(n_bins):
            w = (i + 0.5) * dw
            if w >= wmax:
                continue
            k = (2.0 / a_eff) * math.asin(w / wmax)
            v = 0.5 * a_eff * math.sqrt(wmax * wmax - w * w)
            dos = g * k * k / (2.0 * math.pi ** 2 * v)
            r_imp = TAU_A * w ** 4
            r_3ph = TAU_B * w * w * T * math.exp(-TAU_C / T)
            if impurity_clock:
                rows.append((w, dos, v, dw, 1.0 / r_3ph, 0.0, 1.0 / r_imp, i, branch + 1))
            else:
                rows.append((w, dos, v, dw, 1.0 / (r_imp + r_3ph), 0.0, 0.0, i, branch + 1))
    return np.array(rows, dtype=MODE_DTYPE)


def gray_modes(v: float, tau: float, C: float = 1.0e6, tau_imp: float = 0.0) -> np.ndarray:
    """One gray mode in the paper's second material-data format (omega, V_g, tau, C); tau_imp > 0
    adds the separate two-phonon clock."""
    return np.array([(1.0e13, 0.0, v, 0.0, tau, C, tau_imp, 0, 1)], dtype=MODE_DTYPE)


def _geometry(L, unbounded=(False, False, False), faces=None, cylinders=(), gradT=(0.0, 0.0, 0.0),
              volume=0.0, walls=()):
    return {
        "L": tuple(float(x) for x in L),
        "unbounded": tuple(bool(u) for u in unbounded),
        "faces": {int(k): tuple(float(x) for x in v) for k, v in (faces or {}).items()},
        "cylinders": [tuple(c) for c in cylinders],
        # internal line walls (x1, y1, x2, y2, nx, ny, id, type, specularity[, cutoff omega])
        "walls": [tuple(c) for c in walls],
        "gradT": tuple(float(x) for x in gradT),
        "volume": float(volume),
    }


def _problem(N, T_lin=300.0, n_scat_max=0, transient=False, t_max=0.0, t_meas=(), ic=None,
             max_events=10_000_000, score_axis=2, fmt=1):
    p = {
        "N": int(N), "T_lin": float(T_lin), "n_scat_max": int(n_scat_max),
        "transient": bool(transient), "t_max": float(t_max),
        "t_meas": np.asarray(t_meas, dtype=np.float64),
        "ic_axis": 2, "ic_edges": np.zeros(0), "ic_dT": np.zeros(0),
        "max_events": int(max_events), "score_axis": int(score_axis), "format": int(fmt),
    }
    if ic is not None:
        p["ic_axis"] = int(ic[0])
        p["ic_edges"] = np.asarray(ic[1], dtype=np.float64)
        p["ic_dT"] = np.asarray(ic[2], dtype=np.float64)
    return p


def _detectors(lo=(0.0, 0.0, 0.0), hi=(0.0, 0.0, 0.0), n=(0, 0, 0), mask=MASK_ALL):
    return {"lo": tuple(float(x) for x in lo), "hi": tuple(float(x) for x in hi),
            "n": tuple(int(x) for x in n), "mask": int(mask)}


def gaussian_cell_average(edges: np.ndarray, centre: float, sigma: float, peak: float) -> np.ndarray:
    """Cell averages of peak * exp(-(z - centre)^2 / (2 sigma^2)) over [edges[c], edges[c+1])."""
    from scipy.special import erf
    s2 = sigma * math.sqrt(2.0)
    a, b = edges[:-1], edges[1:]
    integral = peak * sigma * math.sqrt(math.pi / 2.0) * (erf((b - centre) / s2) - erf((a - centre) / s2))
    return integral / (b - a)


# --------------------------------------------------------------------------------------------
# Named workloads.  Each returns a fresh dict; callers may override any field.
# --------------------------------------------------------------------------------------------

def gray_slab(N=100_000, Lambda=100e-9, L=100e-9, v=6400.0, T_hot=301.0, T_cold=299.0, bins=50,
              seed=SEED_BASE + 1):
    """Steady 1-D cross-plane slab between two black isothermal walls, gray medium."""
    return {
        "name": "gray_slab",
        "modes": gray_modes(v, Lambda / v),
        "geometry": _geometry((1.0, 1.0, L), (True, True, False),
                              {5: (ISOTHERMAL, T_hot, 0, 0), 6: (ISOTHERMAL, T_cold, 0, 0)}),
        "detectors": _detectors((0, 0, 0), (0, 0, L), (0, 0, bins)),
        "problem": _problem(N, 300.0, 0, score_axis=2, fmt=2),
        "seed": seed,
    }


def film(N=1_000_000, d=100e-9, T=300.0, gradT=-1.0e7, specularity=0.0, n_scat_max=10,
         z_bins=0, seed=SEED_BASE + 2, modes=None, spec_omega=0.0):
    """Steady in-plane thin film: diffuse (or partially specular) walls at z = 0, d; in-plane
    axes unbounded; uniform gradient along y driving the spatially varying control.
    spec_omega > 0: phonons with omega below it reflect specularly off the walls (boundary data
    word 2 of an adiabatic wall)."""
    det = _detectors((0, 0, 0), (0, 0, d), (0, 0, z_bins), MASK_T | MASK_QY)
    return {
        "name": "film",
        "modes": silicon_like_modes(T) if modes is None else modes,
        "geometry": _geometry((1.0, 1.0, d), (True, True, False),
                              {5: (ADIABATIC, specularity, spec_omega, 0), 6: (ADIABATIC, specularity, spec_omega, 0)},
                              gradT=(0.0, gradT, 0.0)),
        "detectors": det,
        "problem": _problem(N, T, n_scat_max, score_axis=1, fmt=1),
        "seed": seed,
    }


def transient_bump(N=10_000_000, L=1e-6, T=300.0, sigma=50e-9, peak=1.0, n_cells=1000,
                   n_times=200, dt_meas=10e-12, bins=100, seed=SEED_BASE + 3, modes=None, fmt=1):
    """Transient 1-D slab with specular walls, seeded by a Gaussian temperature bump."""
    edges = np.linspace(0.0, L, n_cells + 1)
    dT = gaussian_cell_average(edges, 0.5 * L, sigma, peak)
    t_meas = np.arange(n_times, dtype=np.float64) * dt_meas
    return {
        "name": "transient_bump",
        "modes": silicon_like_modes(T) if modes is None else modes,
        "geometry": _geometry((1.0, 1.0, L), (True, True, False),
                              {5: (ADIABATIC, 1.0, 0, 0), 6: (ADIABATIC, 1.0, 0, 0)}),
        "detectors": _detectors((0, 0, 0), (0, 0, L), (0, 0, bins), MASK_T | MASK_QZ),
        "problem": _problem(N, T, 0, transient=True, t_max=n_times * dt_meas, t_meas=t_meas,
                            ic=(2, edges, dT), score_axis=2, fmt=fmt),
        "seed": seed,
    }


def film_sweep(scale=1.0, seed=SEED_BASE + 4):
    """The batched sweep: 16 log-spaced thicknesses (10 nm .. 10 um) x 4 temperatures.

    Instance j (thickness index) carries round(10^(5 + log10(40) j / 15)) particles times
    `scale`; instance id = 16 * t_index + j.
    """
    out = []
    for ti, T in enumerate((100.0, 200.0, 300.0, 400.0)):
        modes = silicon_like_modes(T)
        for j in range(16):
            d = 10.0 ** (-8.0 + 3.0 * j / 15.0)
            N = max(1, int(round(scale * 10.0 ** (5.0 + math.log10(40.0) * j / 15.0))))
            w = film(N=N, d=d, T=T, seed=seed, modes=modes)
            w["name"] = f"film_sweep[T={T:.0f},d={d:.3e}]"
            w["instance"] = 16 * ti + j
            out.append(w)
    return out


# Relaxation cap of the periodic cell's benchmark configuration.  The cell has no absorbing
# boundary, so every particle ends at the cap, and the part of its score past the cap is dropped;
# next to the pore a relaxed particle still has a mean displacement ahead of it, so the cap biases
# kappa until the particle's position in the cell has mixed.  Per-particle scores of the same 1e8
# particles under caps 20 ... 640 (FP32) put the bias at +2.7 % of kappa at cap 20, +0.6 % at
# cap 40 and within the paired statistical error (0.1 - 0.2 %) from cap 80 on
# (tests/test_gpu_convergence.py repeats the comparison on 2e7 particles).
C5_NSCAT = 80


def porous_cell(N=100_000_000, W=500e-9, porosity=0.25, T=300.0, gradT=-2.0e6, n_scat_max=10,
                specularity=0.0, seed=SEED_BASE + 5, modes=None, spec_omega=0.0):
    """3-D periodic cubic cell with a centred z-axis cylindrical pore (diffuse pore wall);
    spec_omega > 0: phonons with omega below it reflect specularly off the pore."""
    r = W * math.sqrt(porosity / math.pi)
    faces = {1: (PERIODIC, 0, W, 0), 3: (PERIODIC, 0, -W, 0), 2: (PERIODIC, -W, 0, 0),
             4: (PERIODIC, W, 0, 0), 5: (PERIODIC, 0, 0, W), 6: (PERIODIC, 0, 0, -W)}
    return {
        "name": "porous_cell",
        "modes": silicon_like_modes(T) if modes is None else modes,
        "geometry": _geometry((W, W, W), (False, False, False), faces,
                              cylinders=[(0.5 * W, 0.5 * W, r, 7, ADIABATIC, specularity, spec_omega)],
                              gradT=(0.0, gradT, 0.0)),
        "detectors": _detectors(mask=MASK_T | MASK_QY),
        "problem": _problem(N, T, n_scat_max, score_axis=1, fmt=1),
        "seed": seed,
    }


def square_pore_cell(N=1_000_000, W=500e-9, side=250e-9, T=300.0, gradT=-2.0e6, n_scat_max=10,
                     specularity=0.0, seed=SEED_BASE + 9, modes=None):
    """3-D periodic cubic cell with a centred square pore bounded by four internal line walls
    (the paper's nanomesh layout: walls in the x-y plane through the thickness, normals pointing
    into the solid; ids 7..10)."""
    a, b = 0.5 * (W - side), 0.5 * (W + side)
    walls = [(a, a, b, a, 0.0, -1.0, 7, ADIABATIC, specularity),
             (b, a, b, b, 1.0, 0.0, 8, ADIABATIC, specularity),
             (b, b, a, b, 0.0, 1.0, 9, ADIABATIC, specularity),
             (a, b, a, a, -1.0, 0.0, 10, ADIABATIC, specularity)]
    faces = {1: (PERIODIC, 0, W, 0), 3: (PERIODIC, 0, -W, 0), 2: (PERIODIC, -W, 0, 0),
             4: (PERIODIC, W, 0, 0), 5: (PERIODIC, 0, 0, W), 6: (PERIODIC, 0, 0, -W)}
    return {
        "name": "square_pore_cell",
        "modes": silicon_like_modes(T) if modes is None else modes,
        "geometry": _geometry((W, W, W), (False, False, False), faces, gradT=(0.0, gradT, 0.0),
                              volume=(W * W - side * side) * W, walls=walls),
        "detectors": _detectors(mask=MASK_T | MASK_QY),
        "problem": _problem(N, T, n_scat_max, score_axis=1, fmt=1),
        "seed": seed,
    }


def walled_film(N=1_000_000, d=100e-9, H=300e-9, Lx=200e-9, T=300.0, gradT=-1.0e7, n_scat_max=10,
                specularity=0.0, seed=SEED_BASE + 10, modes=None):
    """The thin film of `film` made of internal line walls: a channel of thickness d between
    walls at y = (H - d)/2 and (H + d)/2 spanning a box periodic in x, unbounded in z, with the
    gradient along x.  The regions below and above the channel are closed loops of walls (the
    channel walls plus walls along the box edges, which no particle reaches), so emission leaves
    them out."""
    y0, y1 = 0.5 * (H - d), 0.5 * (H + d)
    A, S = ADIABATIC, specularity
    walls = [(0.0, y0, Lx, y0, 0.0, 1.0, 7, A, S), (Lx, y0, Lx, 0.0, 1.0, 0.0, 8, A, S),
             (Lx, 0.0, 0.0, 0.0, 0.0, -1.0, 9, A, S), (0.0, 0.0, 0.0, y0, -1.0, 0.0, 10, A, S),
             (Lx, y1, 0.0, y1, 0.0, -1.0, 11, A, S), (0.0, y1, 0.0, H, -1.0, 0.0, 12, A, S),
             (0.0, H, Lx, H, 0.0, 1.0, 13, A, S), (Lx, H, Lx, y1, 1.0, 0.0, 14, A, S)]
    faces = {2: (PERIODIC, -Lx, 0, 0), 4: (PERIODIC, Lx, 0, 0),
             1: (ADIABATIC, 0.0, 0, 0), 3: (ADIABATIC, 0.0, 0, 0)}
    return {
        "name": "walled_film",
        "modes": silicon_like_modes(T) if modes is None else modes,
        "geometry": _geometry((Lx, H, 1.0), (False, False, True), faces, gradT=(gradT, 0.0, 0.0),
                              volume=Lx * d * 1.0, walls=walls),
        "detectors": _detectors(mask=MASK_T | MASK_QX),
        "problem": _problem(N, T, n_scat_max, score_axis=0, fmt=1),
        "seed": seed,
    }


def walled_slab(N=100_000, Lambda=100e-9, L=100e-9, H=300e-9, Lx=200e-9, v=6400.0, T_hot=301.0,
                T_cold=299.0, seed=SEED_BASE + 11):
    """The gray slab of `gray_slab` between two isothermal internal line walls: hot at
    y = (H - L)/2 (normal +y), cold at (H + L)/2 (normal -y), periodic in x, unbounded in z; the
    regions beyond the walls are closed loops (adiabatic walls along the box edges close them)."""
    y0, y1 = 0.5 * (H - L), 0.5 * (H + L)
    A, I = ADIABATIC, ISOTHERMAL
    walls = [(0.0, y0, Lx, y0, 0.0, 1.0, 7, I, T_hot), (Lx, y0, Lx, 0.0, 1.0, 0.0, 8, A, 0.0),
             (Lx, 0.0, 0.0, 0.0, 0.0, -1.0, 9, A, 0.0), (0.0, 0.0, 0.0, y0, -1.0, 0.0, 10, A, 0.0),
             (Lx, y1, 0.0, y1, 0.0, -1.0, 11, I, T_cold), (0.0, y1, 0.0, H, -1.0, 0.0, 12, A, 0.0),
             (0.0, H, Lx, H, 0.0, 1.0, 13, A, 0.0), (Lx, H, Lx, y1, 1.0, 0.0, 14, A, 0.0)]
    faces = {2: (PERIODIC, -Lx, 0, 0), 4: (PERIODIC, Lx, 0, 0),
             1: (ADIABATIC, 0.0, 0, 0), 3: (ADIABATIC, 0.0, 0, 0)}
    return {
        "name": "walled_slab",
        "modes": gray_modes(v, Lambda / v),
        "geometry": _geometry((Lx, H, 1.0), (False, False, True), faces, volume=Lx * L * 1.0, walls=walls),
        "detectors": _detectors(mask=MASK_ALL),
        "problem": _problem(N, 300.0, 0, score_axis=1, fmt=2),
        "seed": seed,
    }


def ballistic_transient(N=200_000, L=3000e-9, v=12360.0, tau=1.0, T_l=303.0, T_r=297.0,
                        t_max=1.0e-9, t_meas=(5e-12, 50e-12, 100e-12, 200e-12, 300e-12, 900e-12),
                        bins=60, seed=SEED_BASE + 6):
    """The paper's ballistic benchmark: walls impulsively set to T_l / T_r at t = 0."""
    return {
        "name": "ballistic_transient",
        "modes": gray_modes(v, tau),
        "geometry": _geometry((1.0, 1.0, L), (True, True, False),
                              {5: (ISOTHERMAL, T_l, 0, 0), 6: (ISOTHERMAL, T_r, 0, 0)}),
        "detectors": _detectors((0, 0, 0), (0, 0, L), (0, 0, bins), MASK_T | MASK_QZ),
        "problem": _problem(N, 300.0, 0, transient=True, t_max=t_max, t_meas=t_meas, score_axis=2,
                            fmt=2),
        "seed": seed,
    }


def gaussian_pulse_profile(t0: float, sigma: float, peak: float, n: int, span: float = 3.0):
    """A Gaussian pulse peak exp(-(t - t0)^2 / (2 sigma^2)) as n equal piecewise-constant intervals
    over t0 +- span sigma, each holding the pulse's exact mean over it: (edges, values)."""
    edges = np.linspace(t0 - span * sigma, t0 + span * sigma, n + 1)
    z = (edges - t0) / (math.sqrt(2.0) * sigma)
    integral = np.array([0.5 * math.sqrt(2.0 * math.pi) * sigma * (math.erf(z[k + 1]) - math.erf(z[k]))
                         for k in range(n)])
    return edges, peak * integral / np.diff(edges)


def heated_slab(N=10_000_000, L=1e-6, T=300.0, depth=20e-9, sigma=5e-12, peak=None, t_max=2e-9, n_times=200,
                n_cells=100, n_profile=12, n_scat_max=0, modes=None, specularity=0.0, seed=SEED_BASE + 12):
    """Time-domain heating of a free-standing slab (the thermoreflectance setting of the paper's
    summary): a slab of thickness L along z (in-plane unbounded, adiabatic faces of specularity
    `specularity`) heated in its top `depth` by a Gaussian pulse of width sigma centred at 3 sigma,
    tabulated as n_profile intervals; T and q_z in n_cells bins at n_times equally spaced times
    over (0, t_max).  peak (W/m^3) defaults to the power that deposits 1 K of heat capacity 1.66e6
    J/(m^3 K) (silicon-like) across the heated layer."""
    if peak is None:
        peak = 1.66e6 / (math.sqrt(2.0 * math.pi) * sigma)
    edges, vals = gaussian_pulse_profile(3.0 * sigma, sigma, peak, n_profile)
    t_meas = (np.arange(n_times) + 0.5) * (t_max / n_times)
    prob = _problem(N, T, n_scat_max, transient=True, t_max=t_max, t_meas=t_meas, score_axis=2)
    prob["heat"] = {"lo": (0.0, 0.0, L - depth), "hi": (1.0, 1.0, L), "t": edges, "P": vals}
    return {
        "name": "heated_slab",
        "modes": silicon_like_modes(T) if modes is None else modes,
        "geometry": _geometry((1.0, 1.0, L), (True, True, False),
                              {5: (ADIABATIC, specularity, 0, 0), 6: (ADIABATIC, specularity, 0, 0)}),
        "detectors": _detectors((0, 0, 0), (0, 0, L), (0, 0, n_cells), MASK_T | MASK_QZ),
        "problem": prob,
        "seed": seed,
    }


def cube_tets(lo, hi) -> np.ndarray:
    """The cuboid [lo, hi] as six tetrahedra sharing its diagonal lo-hi (one per order of the
    three axes: lo, lo + the first axis' edge, + the second's, hi): array (6, 4, 3)."""
    import itertools
    lo, hi = np.asarray(lo, dtype=np.float64), np.asarray(hi, dtype=np.float64)
    out = []
    for perm in itertools.permutations(range(3)):
        v = [lo.copy()]
        for a in perm:
            nxt = v[-1].copy()
            nxt[a] = hi[a]
            v.append(nxt)
        out.append(np.array(v))
    return np.array(out)


def heated_box(N=200_000, L=(400e-9, 300e-9, 200e-9), tets=None, modes=None, specularity=1.0, t_max=40e-12,
               n_times=4, bins=(4, 1, 1), seed=SEED_BASE + 13):
    """A closed box (all six faces adiabatic, of specularity `specularity`) heated over [0, 10 ps)
    in the union of the tetrahedra `tets` (default: one tetrahedron in a corner), gray medium by
    default; T and q in a grid of bins at n_times times."""
    if tets is None:
        tets = np.array([[[20e-9, 20e-9, 20e-9], [300e-9, 40e-9, 30e-9], [60e-9, 250e-9, 40e-9],
                          [80e-9, 60e-9, 180e-9]]])
    faces = {i: (ADIABATIC, specularity, 0, 0) for i in range(1, 7)}
    t_meas = (np.arange(n_times) + 0.5) * (t_max / n_times)
    prob = _problem(N, 300.0, 0, transient=True, t_max=t_max, t_meas=t_meas, score_axis=0,
                    fmt=2 if modes is None else 1)
    prob["heat"] = {"lo": (0.0, 0.0, 0.0), "hi": tuple(L), "t": np.array([0.0, 10e-12]), "P": np.array([1e17]),
                    "tets": np.asarray(tets, dtype=np.float64)}
    return {
        "name": "heated_box",
        "modes": gray_modes(6400.0, 50e-9 / 6400.0) if modes is None else modes,
        "geometry": _geometry(tuple(L), (False, False, False), faces),
        "detectors": _detectors((0, 0, 0), tuple(L), tuple(bins), MASK_ALL),
        "problem": prob,
        "seed": seed,
    }


def bulk_gradient(N=200_000, v=6400.0, Lambda=100e-9, gradT=-1.0e7, n_scat_max=1, modes=None,
                  seed=SEED_BASE + 7, T=300.0):
    """Unbounded bulk driven only by the gradient source (no boundaries at all)."""
    gray = modes is None
    return {
        "name": "bulk_gradient",
        "modes": gray_modes(v, Lambda / v) if gray else modes,
        "geometry": _geometry((1.0, 1.0, 1.0), (True, True, True), {}, gradT=(0.0, gradT, 0.0)),
        "detectors": _detectors(mask=MASK_ALL),
        "problem": _problem(N, T, n_scat_max, score_axis=1, fmt=2 if gray else 1),
        "seed": seed,
    }


def gray_diffusive_bump(N=100_000, L=1e-6, v=6400.0, Lambda=10e-9, sigma=50e-9, peak=1.0,
                        n_cells=1000, t_end=2e-9, n_times=5, bins=50, seed=SEED_BASE + 8):
    """Gray analogue of the transient bump with a short mean free path (diffusive regime)."""
    w = transient_bump(N=N, L=L, sigma=sigma, peak=peak, n_cells=n_cells, n_times=n_times,
                       dt_meas=t_end / n_times, bins=bins, seed=seed, modes=gray_modes(v, Lambda / v),
                       fmt=2)
    w["name"] = "gray_diffusive_bump"
    # measure at the end of each interval, the last exactly one interval before t_max
    w["problem"]["t_meas"] = np.arange(1, n_times + 1) * (t_end / n_times) - 0.5 * (t_end / n_times)
    w["problem"]["t_max"] = t_end
    return w


def ziman_specularity(modes: np.ndarray, eta: float) -> np.ndarray:
    """Per-row specularity of the silicon-like crystal's rows for a surface of rms roughness eta
    (m), by Ziman's model exp(-16 pi^2 eta^2 / lambda^2) = exp(-4 eta^2 k^2): the wave vector of
    each row from its branch's dispersion omega = omega_max sin(k a / 2) (branch 1 LA, 2 TA)."""
    k_max = 2.0 * math.pi / A_SI
    a_eff = math.pi / k_max
    out = np.zeros(len(modes))
    for i, r in enumerate(modes):
        wmax = OMEGA_MAX_LA if int(r["branch"]) == 1 else OMEGA_MAX_TA
        k = (2.0 / a_eff) * math.asin(min(1.0, float(r["omega"]) / wmax))
        out[i] = math.exp(-4.0 * eta * eta * k * k)
    return out


def random_specularity(n_rows: int, seed: int, binary: bool = False) -> np.ndarray:
    """A seeded per-row specularity table: uniform in [0, 1), or 0 / 1 with equal odds."""
    rng = np.random.default_rng(seed)
    return (rng.random(n_rows) < 0.5).astype(np.float64) if binary else rng.random(n_rows)


def with_spec_table(w: dict, table) -> dict:
    """Copy of w whose adiabatic boundaries (faces, pores, adiabatic line walls) read their
    specularity per material row from `table` (section 3.5.3): the table becomes the problem's
    per-row table 1 and every such boundary's own d and cutoff are set to 0."""
    w = copy.deepcopy(w)
    table = np.asarray(table, dtype=np.float64)
    assert table.shape == (len(w["modes"]),)
    w["problem"]["spec_tables"] = table[None, :]
    g = w["geometry"]
    for fid, f in list(g["faces"].items()):
        if int(f[0]) == ADIABATIC:
            g["faces"][fid] = (ADIABATIC, 0.0, 0.0, 0.0, 1)
    g["cylinders"] = [tuple(c[:5]) + (0.0, 0.0, 1) for c in g["cylinders"]]
    g["walls"] = [tuple(c[:8]) + ((0.0, 0.0, 1) if int(c[7]) == ADIABATIC else (c[8], 0.0, 0))
                  for c in g.get("walls", [])]
    return w


def with_(w: dict, **changes) -> dict:
    """Deep copy of a workload with dotted-path overrides, e.g. with_(w, **{"problem.N": 10})."""
    w = copy.deepcopy(w)
    for key, val in changes.items():
        node = w
        parts = key.split(".")
        for p in parts[:-1]:
            node = node[p]
        node[parts[-1]] = val
    return w


CONFIGS = {
    "C1": gray_slab,
    "C2": film,
    "C3": transient_bump,
    "C5": lambda **kw: porous_cell(**{"n_scat_max": C5_NSCAT, **kw}),
}
