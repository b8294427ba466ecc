"""The paper's input and output files (its "MATLAB code I/O" section), host side only.

Reads a case directory in the paper's plain-text formats into a workload description (the same
dict layout as `workloads`), and writes results in the paper's output formats:

inputs
  mat_data.txt          first format: omega, DOS, V_g, delta-omega, tau, polarization [, tau_imp]
                        second format: omega, V_g, tau, C [, tau_imp]
                        (the optional last column is the impurity relaxation time; rows of equal
                        omega share one frequency bin)
  Out_bnd.txt           x_length y_length z_length (one corner at the origin)
  In_bnd.txt            internal line walls x1 y1 x2 y2 nx ny nz (through the thickness; their
                        Boundary_prop rows are ids 7, 8, ... in the same order)
  Boundary_prop.txt     bnd_ID bnd_type bnd_data1 bnd_data2 bnd_data3 (types 1 isothermal, 2
                        adiabatic, 3 periodic; ids 1..6: y=0, x=L, y=L, x=0, z=0, z=L)
  Thermal_gradient.txt  bnd_ID1 bnd_ID2 grad_x grad_y grad_z
  Sim_param.txt         N  N_scat^max  V  T_lin
  Measure_time.txt      measurement times (a transient run when present)
  Measure_region.txt    xmin xmax ymin ymax zmin zmax n  (one region, refined into 2^(3n) cuboids)

outputs
  detector_location.txt one detector per row: xmin xmax ymin ymax zmin zmax
  T{T_lin}.txt, Qx{T_lin}.txt, Qy{T_lin}.txt, Qz{T_lin}.txt
                        one row per detector; columns are the measurement times (transient) or
                        the frequency bins (steady state); T is the deviation from T_lin

Values are whitespace or comma separated; blank lines and lines starting with '#' or '%' are
skipped.  Nothing here traces particles: the workload goes to `run` (or the C ABI) as usual.
"""
from __future__ import annotations

import os

import numpy as np

MODE_DTYPE = np.dtype([
    ("omega", "f8"), ("dos", "f8"), ("v", "f8"), ("domega", "f8"),
    ("tau", "f8"), ("C", "f8"), ("tau_imp", "f8"), ("bin", "i4"), ("branch", "i4"),
])


def _rows(path: str) -> list[list[float]]:
    out = []
    with open(path) as fh:
        for line in fh:
            s = line.strip()
            if not s or s[0] in "#%":
                continue
            out.append([float(x) for x in s.replace(",", " ").split()])
    return out


def read_mat_data(path: str, fmt: int) -> np.ndarray:
    """Material rows of mat_data.txt in the first (fmt=1) or second (fmt=2) format."""
    rows = _rows(path)
    ncol = (6, 7) if fmt == 1 else (4, 5)
    if fmt not in (1, 2) or not rows or any(len(r) not in ncol for r in rows):
        raise ValueError(f"{path}: expected {ncol[0]} or {ncol[1]} columns per row (format {fmt})")
    omegas = sorted({r[0] for r in rows})
    bin_of = {w: i for i, w in enumerate(omegas)}
    out = np.zeros(len(rows), dtype=MODE_DTYPE)
    for i, r in enumerate(rows):
        if fmt == 1:
            w, dos, v, dw, tau, pol = r[:6]
            out[i] = (w, dos, v, dw, tau, 0.0, r[6] if len(r) == 7 else 0.0, bin_of[w], int(pol))
        else:
            w, v, tau, C = r[:4]
            out[i] = (w, 0.0, v, 0.0, tau, C, r[4] if len(r) == 5 else 0.0, bin_of[w], 1)
    return out


def read_case(directory: str, fmt: int, seed: int = 1, transient: bool | None = None,
              max_events: int = 10_000_000, score_axis: int | None = None) -> dict:
    """A workload description from a directory of the paper's input files."""
    p = lambda name: os.path.join(directory, name)
    modes = read_mat_data(p("mat_data.txt"), fmt)
    (L,) = _rows(p("Out_bnd.txt"))
    if len(L) != 3 or min(L) <= 0:
        raise ValueError("Out_bnd.txt: three positive lengths expected")
    in_bnd = _rows(p("In_bnd.txt")) if os.path.exists(p("In_bnd.txt")) else []
    if any(len(r) != 7 for r in in_bnd):
        raise ValueError("In_bnd.txt: x1 y1 x2 y2 nx ny nz per wall")
    faces, inner = {}, {}
    for r in _rows(p("Boundary_prop.txt")):
        bid, ty = int(r[0]), int(r[1])
        data = list(r[2:5]) + [0.0] * (3 - len(r[2:5]))
        if ty not in (1, 2, 3):
            raise ValueError(f"Boundary_prop.txt: unknown type {ty} for id {bid}")
        if 1 <= bid <= 6:
            faces[bid] = (ty, *data)
        else:
            inner[bid] = (ty, *data)
    if sorted(faces) != [1, 2, 3, 4, 5, 6]:
        raise ValueError("Boundary_prop.txt: ids 1..6 must each appear once")
    if sorted(inner) != list(range(7, 7 + len(in_bnd))):
        raise ValueError("Boundary_prop.txt: one row per In_bnd wall, ids 7, 8, ... in order")
    walls = []
    for k, (x1, y1, x2, y2, nx, ny, nz) in enumerate(in_bnd):
        ty, d0, d1, _ = inner[7 + k]
        if ty not in (1, 2) or nz != 0.0:
            raise NotImplementedError("internal walls: isothermal or adiabatic, perpendicular to the x-y plane")
        walls.append((x1, y1, x2, y2, nx, ny, 7 + k, ty, d0, d1 if ty == 2 else 0.0))
    gradT = (0.0, 0.0, 0.0)
    if os.path.exists(p("Thermal_gradient.txt")):
        g = _rows(p("Thermal_gradient.txt"))
        if g:
            gradT = tuple(float(x) for x in g[0][2:5])
    (sim,) = _rows(p("Sim_param.txt"))
    N, nscat, V, T_lin = int(sim[0]), int(sim[1]), float(sim[2]), float(sim[3])
    t_meas = np.zeros(0)
    if os.path.exists(p("Measure_time.txt")):
        t_meas = np.array([x for r in _rows(p("Measure_time.txt")) for x in r], dtype=np.float64)
    if transient is None:
        transient = t_meas.size > 0
    regions = _rows(p("Measure_region.txt")) if os.path.exists(p("Measure_region.txt")) else []
    if len(regions) > 1:
        raise NotImplementedError("Measure_region.txt: one region (one detector grid) per case")
    if regions:
        x0, x1, y0, y1, z0, z1, n = regions[0]
        k = 2 ** int(n)
        det = {"lo": (x0, y0, z0), "hi": (x1, y1, z1), "n": (k, k, k), "mask": 15}
    else:
        det = {"lo": (0.0, 0.0, 0.0), "hi": (0.0, 0.0, 0.0), "n": (0, 0, 0), "mask": 15}
    if score_axis is None:   # the axis of the driving gradient, else of the first wall pair
        nz = [a for a in range(3) if gradT[a] != 0.0]
        iso = [a for bid, f in faces.items() if f[0] == 1 for a in [(1, 0, 1, 0, 2, 2)[bid - 1]]]
        score_axis = nz[0] if nz else (iso[0] if iso else 2)
    t_max = float(t_meas.max()) if transient and t_meas.size else 0.0
    return {
        "name": os.path.basename(os.path.normpath(directory)),
        "modes": modes,
        "geometry": {"L": tuple(L), "unbounded": (False, False, False),
                     "faces": {int(k): tuple(float(x) for x in v) for k, v in faces.items()},
                     "cylinders": [], "walls": walls, "gradT": gradT, "volume": V},
        "detectors": det,
        "problem": {"N": N, "T_lin": T_lin, "n_scat_max": nscat, "transient": bool(transient),
                    "t_max": t_max, "t_meas": t_meas, "ic_axis": 2, "ic_edges": np.zeros(0),
                    "ic_dT": np.zeros(0), "max_events": int(max_events), "score_axis": int(score_axis),
                    "format": int(fmt)},
        "seed": int(seed),
    }


def write_case(w: dict, directory: str) -> None:
    """The paper's input files for a workload (box geometry, no pores, one detector grid refined
    equally on all axes or none)."""
    g, pr, d = w["geometry"], w["problem"], w["detectors"]
    if g["cylinders"] or any(g["unbounded"]):
        raise NotImplementedError("the paper's files describe bounded boxes with line walls only")
    walls = g.get("walls", [])
    if [c[6] for c in walls] != list(range(7, 7 + len(walls))):
        raise NotImplementedError("the paper's files number the line walls 7, 8, ... in order")
    os.makedirs(directory, exist_ok=True)
    p = lambda name: os.path.join(directory, name)
    m = w["modes"]
    two = bool((m["tau_imp"] > 0).any())
    with open(p("mat_data.txt"), "w") as fh:
        for r in m:
            if pr["format"] == 1:
                cols = [r["omega"], r["dos"], r["v"], r["domega"], r["tau"], r["branch"]]
            else:
                cols = [r["omega"], r["v"], r["tau"], r["C"]]
            if two:
                cols.append(r["tau_imp"])
            fh.write(" ".join(repr(float(c)) for c in cols) + "\n")
    with open(p("Out_bnd.txt"), "w") as fh:
        fh.write(" ".join(repr(float(x)) for x in g["L"]) + "\n")
    with open(p("In_bnd.txt"), "w") as fh:
        for c in walls:
            fh.write(" ".join(repr(float(x)) for x in c[:6]) + " 0.0\n")
    with open(p("Boundary_prop.txt"), "w") as fh:
        for bid in range(1, 7):
            ty, *data = g["faces"][bid]
            fh.write(f"{bid} {int(ty)} " + " ".join(repr(float(x)) for x in data) + "\n")
        for c in walls:
            wc = float(c[9]) if len(c) > 9 else 0.0
            fh.write(f"{int(c[6])} {int(c[7])} {float(c[8])!r} {wc!r} 0.0\n")
    with open(p("Thermal_gradient.txt"), "w") as fh:
        fh.write("1 3 " + " ".join(repr(float(x)) for x in g["gradT"]) + "\n")
    with open(p("Sim_param.txt"), "w") as fh:
        fh.write(f"{int(pr['N'])} {int(pr['n_scat_max'])} {float(g['volume'])!r} {float(pr['T_lin'])!r}\n")
    if pr["transient"]:
        with open(p("Measure_time.txt"), "w") as fh:
            fh.write("\n".join(repr(float(t)) for t in pr["t_meas"]) + "\n")
    if any(d["n"]):
        k = d["n"][0]
        if not (d["n"][0] == d["n"][1] == d["n"][2]) or k & (k - 1):
            raise NotImplementedError("Measure_region.txt refines all three axes into 2^n cells")
        with open(p("Measure_region.txt"), "w") as fh:
            lo, hi = d["lo"], d["hi"]
            fh.write(" ".join(repr(float(x)) for x in (lo[0], hi[0], lo[1], hi[1], lo[2], hi[2]))
                     + f" {int(k).bit_length() - 1}\n")


def detector_cuboids(det: dict, L) -> np.ndarray:
    """The detectors' cuboids (xmin xmax ymin ymax zmin zmax), in the tallies' cell order (the
    last axis fastest); an axis without cells spans the box."""
    axes = []
    for a in range(3):
        n = det["n"][a]
        if n > 0:
            e = np.linspace(det["lo"][a], det["hi"][a], n + 1)
        else:
            e = np.array([0.0, float(L[a])])
        axes.append(e)
    out = []
    for i in range(len(axes[0]) - 1):
        for j in range(len(axes[1]) - 1):
            for k in range(len(axes[2]) - 1):
                out.append((axes[0][i], axes[0][i + 1], axes[1][j], axes[1][j + 1], axes[2][k], axes[2][k + 1]))
    return np.array(out)


def write_results(w: dict, result: dict, directory: str) -> list[str]:
    """detector_location.txt and T/Qx/Qy/Qz{T_lin}.txt from a finalized result (`T` of shape
    (cells, columns), `q` of shape (cells, columns, 3)).  Steady runs report per frequency bin
    (the rows of a bin summed); transient runs per measurement time."""
    os.makedirs(directory, exist_ok=True)
    T = np.asarray(result["T"], dtype=np.float64)
    q = np.asarray(result["q"], dtype=np.float64)
    if not w["problem"]["transient"]:
        bins = w["modes"]["bin"]
        nb = int(bins.max()) + 1
        Tb = np.zeros((T.shape[0], nb))
        qb = np.zeros((q.shape[0], nb, 3))
        np.add.at(Tb, (slice(None), bins), T)
        for a in range(3):
            np.add.at(qb[..., a], (slice(None), bins), q[..., a])
        T, q = Tb, qb
    tag = f"{w['problem']['T_lin']:g}"
    files = []
    cub = detector_cuboids(w["detectors"], w["geometry"]["L"])
    name = os.path.join(directory, "detector_location.txt")
    np.savetxt(name, cub)
    files.append(name)
    for label, arr in (("T", T), ("Qx", q[..., 0]), ("Qy", q[..., 1]), ("Qz", q[..., 2])):
        name = os.path.join(directory, f"{label}{tag}.txt")
        np.savetxt(name, np.atleast_2d(arr))
        files.append(name)
    return files


def run_case(directory: str, fmt: int, out_dir: str | None = None, precision: int = 32, seed: int = 1,
             device: int = 0) -> dict:
    """Read a case directory, trace it on the GPU and write the paper's output files (into
    `out_dir`, default the case directory)."""
    from .mcbte import run
    w = read_case(directory, fmt, seed=seed)
    res = run(w, precision=precision, device=device)
    write_results(w, res, out_dir or directory)
    return res
