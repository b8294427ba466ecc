"""CPU oracle for the deviational phonon Monte Carlo tracer -- test infrastructure.

The arithmetic lives in ``mcbte_oracle.c`` (plain FP64 C, one particle at a time,
built with ``-ffp-contract=off``).  This module builds that file with gcc, marshals the
workload descriptions of :mod:`workloads` into the oracle's own structs, runs particle
ranges (optionally split over threads, each range with its own tally arrays, summed in
range order) and normalises the raw sums into temperatures, fluxes and kappa.

Only the test suite, the smoke check and the CPU-baseline leg of the benchmark may
import this package.  It shares no code with the HIP library.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess
import threading
from concurrent.futures import ThreadPoolExecutor

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mcbte_oracle.c")
_HDR = os.path.join(_HERE, "mcbte_oracle.h")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

N_COUNTS = 16
COUNT_NAMES = ["particles", "flights", "relaxations", "specular", "diffuse", "periodic", "absorbed",
               "timeouts", "nscat_end", "cap_end", "escaped", "rejections", "two_phonon"]
EV_NAMES = {0: "emit+", 1: "relax", 2: "specular", 3: "diffuse", 4: "periodic", 5: "absorb",
            6: "timeout", 7: "nscat_end", 8: "cap_end", 9: "emit-", 10: "escape"}


class Mode(C.Structure):
    _fields_ = [("omega", C.c_double), ("dos", C.c_double), ("v", C.c_double), ("domega", C.c_double),
                ("tau", C.c_double), ("C", C.c_double), ("tau_imp", C.c_double),
                ("bin", C.c_int32), ("branch", C.c_int32)]


class Face(C.Structure):
    _fields_ = [("type", C.c_int32), ("spec_table", C.c_int32), ("data", C.c_double * 3)]


class Cyl(C.Structure):
    _fields_ = [("cx", C.c_double), ("cy", C.c_double), ("r", C.c_double), ("id", C.c_int32),
                ("type", C.c_int32), ("spec", C.c_double), ("spec_wc", C.c_double), ("spec_table", C.c_int32),
                ("pad", C.c_int32)]


class Wall(C.Structure):
    _fields_ = [("x1", C.c_double), ("y1", C.c_double), ("x2", C.c_double), ("y2", C.c_double),
                ("nx", C.c_double), ("ny", C.c_double), ("id", C.c_int32), ("type", C.c_int32),
                ("spec", C.c_double), ("spec_wc", C.c_double), ("spec_table", C.c_int32), ("pad", C.c_int32)]


class Geom(C.Structure):
    _fields_ = [("L", C.c_double * 3), ("unbounded", C.c_int32 * 3), ("n_cyl", C.c_int32),
                ("face", Face * 6), ("cyl", Cyl * 8), ("gradT", C.c_double * 3), ("volume", C.c_double),
                ("n_wall", C.c_int32), ("pad_w", C.c_int32), ("wall", Wall * 16)]


class Det(C.Structure):
    _fields_ = [("lo", C.c_double * 3), ("hi", C.c_double * 3), ("n", C.c_int32 * 3), ("mask", C.c_int32)]


class Problem(C.Structure):
    _fields_ = [("N", C.c_int64), ("max_events", C.c_int64), ("T_lin", C.c_double), ("t_max", C.c_double),
                ("n_scat_max", C.c_int32), ("format", C.c_int32), ("transient", C.c_int32),
                ("score_axis", C.c_int32), ("n_times", C.c_int32), ("ic_axis", C.c_int32),
                ("n_ic", C.c_int32), ("n_spec_tables", C.c_int32),
                ("t_meas", C.POINTER(C.c_double)), ("ic_edges", C.POINTER(C.c_double)),
                ("ic_dT", C.POINTER(C.c_double)), ("spec_table", C.POINTER(C.c_double)),
                ("n_heat", C.c_int32), ("n_heat_tet", C.c_int32), ("heat_lo", C.c_double * 3),
                ("heat_hi", C.c_double * 3), ("heat_t", C.POINTER(C.c_double)), ("heat_P", C.POINTER(C.c_double)),
                ("heat_tet", C.POINTER(C.c_double))]


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain FP64: no contraction, no fast-math)."""
    with _lock:
        stale = (not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC)
                 or os.path.getmtime(_LIB) < os.path.getmtime(_HDR))
        if force or stale:
            tmp = _LIB + ".tmp%d" % os.getpid()
            subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
                                   "-shared", "-o", tmp, _SRC, "-lm"])
            os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(_LIB)
        p = C.c_void_p
        L.orc_build.argtypes = [C.POINTER(Mode), C.c_int32, C.POINTER(Geom), C.POINTER(Det), C.POINTER(Problem),
                                C.POINTER(p)]
        L.orc_build.restype = C.c_int
        L.orc_free.argtypes = [p]
        L.orc_info.argtypes = [p, C.POINTER(C.c_double), C.POINTER(C.c_int64)]
        L.orc_get.argtypes = [p, C.c_int32, p, C.c_int64]
        L.orc_get.restype = C.c_int
        L.orc_trace.argtypes = [p, C.c_uint64, C.c_uint32, C.c_int64, C.c_int64, p, p, p, p, C.c_int64, C.c_int32]
        L.orc_trace.restype = C.c_int
        L.orc_philox4x32_10.argtypes = [p, p, p]
        L.orc_record.argtypes = [C.c_uint64, C.c_uint32, C.c_int64, C.c_uint32, p]
        L.orc_cdf_pick.argtypes = [p, C.c_int64, C.c_int64, C.c_uint64]
        L.orc_cdf_pick.restype = C.c_int64
        L.orc_cdf_build.argtypes = [p, C.c_int64, p, p]
        L.orc_dir_iso.argtypes = [C.c_double, C.c_double, p]
        L.orc_dir_cos.argtypes = [C.c_double, C.c_double, p, p]
        L.orc_dedT.argtypes = [C.c_double, C.c_double]
        L.orc_dedT.restype = C.c_double
        L.orc_tally_segment.argtypes = [p, p, p, C.c_double, C.c_int32, C.c_double, p]
        L.orc_emit_state.argtypes = [p, C.c_uint64, C.c_uint32, C.c_int64, p, p]
        L.orc_emit_state.restype = C.c_int
        L.orc_emit_clocks.argtypes = [p, C.c_uint64, C.c_uint32, C.c_int64, p, p]
        L.orc_emit_clocks.restype = C.c_int
        L.orc_adjoint.argtypes = [p, C.c_uint64, C.c_uint32, C.c_int64, C.c_int64, C.c_int32, C.c_double, p, p, p, p, p]
        L.orc_adjoint.restype = C.c_int
        L.orc_next_boundary.argtypes = [p, p, p, p]
        L.orc_next_boundary.restype = C.c_double
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


# ----------------------------------------------------------------------------------------------
# building blocks (exposed for the pins)
# ----------------------------------------------------------------------------------------------

def philox(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def record(seed: int, instance: int, pid: int, rec: int) -> np.ndarray:
    out = np.zeros(8, dtype=np.uint32)
    lib().orc_record(seed, instance, pid, rec, _ptr(out))
    return out


def cdf_build(w) -> tuple[np.ndarray, int]:
    w = np.ascontiguousarray(w, dtype=np.float64)
    thr = np.zeros(len(w), dtype=np.uint64)
    last = np.zeros(1, dtype=np.int64)
    lib().orc_cdf_build(_ptr(w), len(w), _ptr(thr), _ptr(last))
    return thr, int(last[0])


def cdf_pick(thr: np.ndarray, last: int, K: int) -> int:
    thr = np.ascontiguousarray(thr, dtype=np.uint64)
    return int(lib().orc_cdf_pick(_ptr(thr), len(thr), last, K))


def dir_iso(u1: float, u2: float) -> np.ndarray:
    out = np.zeros(3)
    lib().orc_dir_iso(u1, u2, _ptr(out))
    return out


def dir_cos(u1: float, u2: float, n) -> np.ndarray:
    n = np.ascontiguousarray(n, dtype=np.float64)
    out = np.zeros(3)
    lib().orc_dir_cos(u1, u2, _ptr(n), _ptr(out))
    return out


def dedT(omega: float, T: float) -> float:
    return lib().orc_dedT(omega, T)


# ----------------------------------------------------------------------------------------------
# problem tables
# ----------------------------------------------------------------------------------------------

class Tables:
    """The oracle's tables for one workload (see ``orc_build``)."""

    def __init__(self, w: dict):
        L = lib()
        self.w = w
        modes = np.ascontiguousarray(w["modes"])
        self._modes = (Mode * len(modes))()
        for i, r in enumerate(modes):
            self._modes[i] = Mode(float(r["omega"]), float(r["dos"]), float(r["v"]), float(r["domega"]),
                                  float(r["tau"]), float(r["C"]), float(r["tau_imp"]), int(r["bin"]),
                                  int(r["branch"]))
        g = w["geometry"]
        G = Geom()
        for a in range(3):
            G.L[a] = g["L"][a]
            G.unbounded[a] = int(g["unbounded"][a])
            G.gradT[a] = g["gradT"][a]
        for fid, f in g["faces"].items():
            G.face[fid - 1].type = int(f[0])
            G.face[fid - 1].data[0], G.face[fid - 1].data[1], G.face[fid - 1].data[2] = f[1], f[2], f[3]
            G.face[fid - 1].spec_table = int(f[4]) if len(f) > 4 else 0
        G.n_cyl = len(g["cylinders"])
        for i, c in enumerate(g["cylinders"]):
            cx, cy, r, cid, ty, spec = c[:6]
            G.cyl[i] = Cyl(cx, cy, r, int(cid), int(ty), spec, float(c[6]) if len(c) > 6 else 0.0,
                           int(c[7]) if len(c) > 7 else 0, 0)
        walls = g.get("walls", [])
        if len(walls) > 16:
            raise ValueError("at most 16 internal line walls")
        G.n_wall = len(walls)
        for i, c in enumerate(walls):
            x1, y1, x2, y2, nx, ny, wid, ty, spec = c[:9]
            G.wall[i] = Wall(x1, y1, x2, y2, nx, ny, int(wid), int(ty), spec, float(c[9]) if len(c) > 9 else 0.0,
                             int(c[10]) if len(c) > 10 else 0, 0)
        G.volume = g["volume"]
        self._geom = G
        d = w["detectors"]
        D = Det()
        for a in range(3):
            D.lo[a], D.hi[a], D.n[a] = d["lo"][a], d["hi"][a], d["n"][a]
        D.mask = d["mask"]
        self._det = D
        p = w["problem"]
        self._t_meas = np.ascontiguousarray(p["t_meas"], dtype=np.float64)
        self._ic_edges = np.ascontiguousarray(p["ic_edges"], dtype=np.float64)
        self._ic_dT = np.ascontiguousarray(p["ic_dT"], dtype=np.float64)
        self._spec = np.ascontiguousarray(p.get("spec_tables", np.zeros((0, len(modes)))), dtype=np.float64)
        dp = C.POINTER(C.c_double)
        P = Problem(p["N"], p["max_events"], p["T_lin"], p["t_max"], p["n_scat_max"], p["format"],
                    int(p["transient"]), p["score_axis"], len(self._t_meas) if p["transient"] else 0,
                    p["ic_axis"], len(self._ic_dT), self._spec.shape[0],
                    self._t_meas.ctypes.data_as(dp), self._ic_edges.ctypes.data_as(dp),
                    self._ic_dT.ctypes.data_as(dp), self._spec.ctypes.data_as(dp) if self._spec.shape[0] else None)
        heat = p.get("heat")
        if heat is not None:
            self._heat_t = np.ascontiguousarray(heat["t"], dtype=np.float64)
            self._heat_P = np.ascontiguousarray(heat["P"], dtype=np.float64)
            P.n_heat = len(self._heat_P)
            for a in range(3):
                P.heat_lo[a], P.heat_hi[a] = heat["lo"][a], heat["hi"][a]
            P.heat_t, P.heat_P = self._heat_t.ctypes.data_as(dp), self._heat_P.ctypes.data_as(dp)
            if heat.get("tets") is not None:
                self._heat_tet = np.ascontiguousarray(heat["tets"], dtype=np.float64).reshape(-1, 12)
                P.n_heat_tet = self._heat_tet.shape[0]
                P.heat_tet = self._heat_tet.ctypes.data_as(dp)
        self._prob = P
        h = C.c_void_p()
        rc = L.orc_build(self._modes, len(modes), C.byref(G), C.byref(D), C.byref(P), C.byref(h))
        if rc != 0:
            raise ValueError(f"oracle table build failed with status {rc}")
        self.h = h
        dd = (C.c_double * 6)()
        ii = (C.c_int64 * 5)()
        L.orc_info(h, dd, ii)
        self.C_tot, self.Wv, self.e_eff, self.V_solid, self.E_tot, self.kappa_bulk = list(dd)
        self.M, self.S, self.n_cells, self.n_cols, self.n_bins = list(ii)

    def __del__(self):
        # at interpreter shutdown the module's globals may already be gone
        if getattr(self, "h", None) and callable(globals().get("lib")):
            lib().orc_free(self.h)
            self.h = None

    def get(self, which: str) -> np.ndarray:
        code, n, dt = {"C": (0, self.M, np.float64), "thr_ic": (1, self.M, np.uint64),
                       "thr_wall": (2, self.M, np.uint64), "thr_rel": (3, self.M, np.uint64),
                       "src_E": (4, self.S, np.float64), "thr_src": (5, self.S, np.uint64),
                       "src_sign": (6, self.S, np.int32), "last": (7, 4, np.int64),
                       "P_bin": (8, self.n_bins, np.float64), "bin": (9, self.M, np.int32)}[which]
        out = np.zeros(n, dtype=dt)
        if lib().orc_get(self.h, code, _ptr(out), n) != 0:
            raise ValueError(which)
        return out

    @property
    def raw_size(self) -> int:
        return self.n_cells * self.n_cols * 4

    def trace_range(self, seed: int, instance: int, first_pid: int, n: int, n_log: int = 0, log_stride: int = 64):
        raw = np.zeros(self.raw_size)
        counts = np.zeros(N_COUNTS, dtype=np.uint64)
        mom = np.zeros(4)
        log = np.zeros((max(n_log, 0), log_stride), dtype=np.uint32)
        rc = lib().orc_trace(self.h, seed, instance, first_pid, n, _ptr(raw), _ptr(counts), _ptr(mom),
                             _ptr(log) if n_log > 0 else None, n_log, log_stride)
        if rc != 0:
            raise ValueError(f"oracle trace failed with status {rc}")
        return raw, counts, mom, log

    def emit_state(self, pid: int, seed: int | None = None, instance: int = 0):
        """(x, o, t, dt_rem) as float64[8] and (mode, sign, source, rejections) as int32[4]."""
        d8 = np.zeros(8)
        i4 = np.zeros(4, dtype=np.int32)
        sd = int(self.w["seed"]) if seed is None else int(seed)
        if lib().orc_emit_state(self.h, sd, instance, pid, _ptr(d8), _ptr(i4)) != 0:
            raise ValueError("emission failed")
        return d8, i4

    def emit_clocks(self, pid: int, seed: int | None = None, instance: int = 0):
        """Two-clock tables: (lead of the later clock, 1 if the two-phonon clock fires first)."""
        lead = np.zeros(1)
        nx2 = np.zeros(1, dtype=np.int32)
        sd = int(self.w["seed"]) if seed is None else int(seed)
        if lib().orc_emit_clocks(self.h, sd, instance, pid, _ptr(lead), _ptr(nx2)) != 0:
            raise ValueError("emission failed")
        return float(lead[0]), int(nx2[0])

    def next_boundary(self, x, o) -> tuple[float, int]:
        x = np.ascontiguousarray(x, dtype=np.float64)
        o = np.ascontiguousarray(o, dtype=np.float64)
        hit = np.zeros(1, dtype=np.int32)
        d = lib().orc_next_boundary(self.h, _ptr(x), _ptr(o), _ptr(hit))
        return d, int(hit[0])

    def segment(self, x0, o, d, m, s=1.0) -> np.ndarray:
        raw = np.zeros(self.raw_size)
        x0 = np.ascontiguousarray(x0, dtype=np.float64)
        o = np.ascontiguousarray(o, dtype=np.float64)
        lib().orc_tally_segment(self.h, _ptr(x0), _ptr(o), float(d), int(m), float(s), _ptr(raw))
        return raw


def trace(w: dict, n: int | None = None, first_pid: int = 0, threads: int = 1, n_log: int = 0,
          log_stride: int = 64, tables: Tables | None = None, instance: int | None = None) -> dict:
    """Trace particles [first_pid, first_pid + n) of workload w; returns the raw sums."""
    tb = tables or Tables(w)
    n = w["problem"]["N"] if n is None else int(n)
    inst = int(w.get("instance", 0) if instance is None else instance)
    threads = max(1, min(int(threads), n)) if n > 0 else 1
    bounds = [first_pid + (n * i) // threads for i in range(threads + 1)]

    def one(i):
        lo, hi = bounds[i], bounds[i + 1]
        nl = max(0, min(n_log - (lo - first_pid), hi - lo))
        return tb.trace_range(int(w["seed"]), inst, lo, hi - lo, nl, log_stride)

    if threads == 1:
        parts = [one(0)]
    else:
        with ThreadPoolExecutor(threads) as ex:
            parts = list(ex.map(one, range(threads)))
    raw = np.zeros(tb.raw_size)
    counts = np.zeros(N_COUNTS, dtype=np.uint64)
    mom = np.zeros(4)
    logs = []
    for r, c, m, lg in parts:        # fixed range order
        raw += r
        counts += c
        mom += m
        logs.append(lg)
    log = np.concatenate(logs, axis=0) if logs else np.zeros((0, log_stride), np.uint32)
    return {"raw": raw, "counts": counts, "moments": mom, "log": log[:max(n_log, 0)], "tables": tb}


def finalize(res: dict) -> dict:
    """Raw sums -> deviational temperature and heat flux per detector (section 3.4 for transient
    snapshots, section 3.6 for steady track lengths), kappa and its standard error."""
    tb: Tables = res["tables"]
    w = tb.w
    raw = res["raw"].reshape(tb.n_cells, tb.n_cols, 4)
    n = int(res["counts"][0])
    if n == 0:                                        # no particle traced: nothing to normalise
        z = np.zeros((tb.n_cells, tb.n_cols))
        return {"T": z, "q": np.zeros((tb.n_cells, tb.n_cols, 3)), "e_eff": math.nan, "V_cell": math.nan,
                "counts": dict(zip(COUNT_NAMES, [int(x) for x in res["counts"][:len(COUNT_NAMES)]]))}
    e = tb.E_tot / n                                  # effective energy (rate) per particle
    det, g = w["detectors"], w["geometry"]
    if all(k == 0 for k in det["n"]):
        Vc = tb.V_solid
    else:
        Vc = 1.0
        for a in range(3):
            if det["n"][a] > 0:
                Vc *= (det["hi"][a] - det["lo"][a]) / det["n"][a]
            elif not g["unbounded"][a]:
                Vc *= g["L"][a]
    out = {"T": e / (tb.C_tot * Vc) * raw[..., 0], "q": e / Vc * raw[..., 1:], "e_eff": e, "V_cell": Vc,
           "counts": dict(zip(COUNT_NAMES, [int(x) for x in res["counts"][:len(COUNT_NAMES)]]))}
    if not w["problem"]["transient"] and n > 1:
        m = res["moments"]
        sa = w["problem"]["score_axis"]
        var_q = max(m[3] - m[2] * m[2] / n, 0.0) / (n - 1)
        var_T = max(m[1] - m[0] * m[0] / n, 0.0) / (n - 1)
        out["q_score"] = tb.E_tot / tb.V_solid * m[2] / n
        out["q_score_sigma"] = tb.E_tot / tb.V_solid * np.sqrt(var_q / n)
        out["T_mean"] = tb.E_tot / (tb.C_tot * tb.V_solid) * m[0] / n
        out["T_mean_sigma"] = tb.E_tot / (tb.C_tot * tb.V_solid) * np.sqrt(var_T / n)
        gs = g["gradT"][sa]
        if gs != 0.0:
            out["kappa"] = -out["q_score"] / gs
            out["kappa_sigma"] = out["q_score_sigma"] / abs(gs)
            out["kappa_cell_avg"] = out["kappa"] * tb.V_solid / (np.prod([g["L"][a] if not g["unbounded"][a]
                                                                          else 1.0 for a in range(3)]))
    return out


def run(w: dict, n: int | None = None, threads: int = 1, **kw) -> dict:
    res = trace(w, n=n, threads=threads, **kw)
    res.update(finalize(res))
    return res


def run_batches(w: dict, n_batches: int, n: int | None = None, threads: int = 8) -> list[dict]:
    """Split particles [0, n) into n_batches contiguous ranges; finalize each range on its own
    (batch means give the statistical error of binned tallies)."""
    tb = Tables(w)
    n = w["problem"]["N"] if n is None else int(n)
    bounds = [(n * i) // n_batches for i in range(n_batches + 1)]
    inst = int(w.get("instance", 0))

    def one(i):
        raw, counts, mom, _ = tb.trace_range(int(w["seed"]), inst, bounds[i], bounds[i + 1] - bounds[i])
        res = {"raw": raw, "counts": counts, "moments": mom, "tables": tb}
        res.update(finalize(res))
        return res

    with ThreadPoolExecutor(max(1, min(threads, n_batches))) as ex:
        return list(ex.map(one, range(n_batches)))


def batch_statistics(batches: list[dict], key=None) -> dict:
    """Particle-weighted mean over independently traced particle groups (each finalized on its
    own) and the standard error of that mean from the spread of the group values (batch means;
    trajectories are independent, section 6): mean = sum_b n_b X_b / N and
    sigma^2 = sum_b n_b (X_b - mean)^2 / ((B - 1) N) over the B groups that traced particles (NaN
    for fewer than two; a group without particles weighs nothing).  key(batch) picks the
    finalized array (default: T and q stacked as [..., 4])."""
    pick = key or (lambda b: np.concatenate([b["T"][..., None], b["q"]], axis=-1))
    X = np.stack([np.asarray(pick(b), dtype=np.float64) for b in batches])
    nb = np.array([float(b["counts"]["particles"]) for b in batches])
    N = nb.sum()
    shape = (-1,) + (1,) * (X.ndim - 1)
    if not N > 0:                                   # no particle at all
        return {"mean": np.zeros(X.shape[1:]), "sigma": np.full(X.shape[1:], np.nan)}
    mean = (nb.reshape(shape) * X).sum(axis=0) / N
    used = int((nb > 0).sum())                      # groups that traced particles
    if used < 2:
        sigma = np.full(mean.shape, np.nan)
    else:
        sigma = np.sqrt((nb.reshape(shape) * (X - mean) ** 2).sum(axis=0) / ((used - 1) * N))
    return {"mean": mean, "sigma": sigma}


def kappa_cumulative(batches: list[dict], order: str = "mfp") -> dict:
    """Cumulative thermal conductivity from the per-row steady flux columns (section 4.5's
    frequency-resolved output, accumulated as in section 5.6).  Each row's kappa is
    -q_score,row / gradT_score; order "mfp" sums rows in ascending mean free path v tau (two clocks
    combined by Matthiessen's rule), order "omega" sums frequency bins in ascending order of their
    lowest row frequency (a bin without rows last); ties keep index order.  Batch means over the
    given groups as batch_statistics."""
    w = batches[0]["tables"].w
    modes = w["modes"]
    sa = int(w["problem"]["score_axis"])
    gs = float(w["geometry"]["gradT"][sa])
    if w["problem"]["transient"] or any(int(x) > 0 for x in w["detectors"]["n"]) or gs == 0.0:
        raise ValueError("cumulative kappa needs a steady problem, one detector cell and a gradient")
    tau = np.asarray(modes["tau"], dtype=np.float64)
    t2 = np.asarray(modes["tau_imp"], dtype=np.float64)
    tau_eff = np.where(t2 > 0.0, 1.0 / (1.0 / tau + 1.0 / np.where(t2 > 0.0, t2, 1.0)), tau)
    if order == "mfp":
        keys_all = np.asarray(modes["v"], dtype=np.float64) * tau_eff
    elif order == "omega":
        bins = np.asarray(modes["bin"], dtype=np.int64)
        keys_all = np.full(int(bins.max()) + 1, np.inf)
        for r in range(len(modes)):
            keys_all[bins[r]] = min(keys_all[bins[r]], float(modes["omega"][r]))
    else:
        raise ValueError(order)
    idx = np.argsort(keys_all, kind="stable")

    def cum(b):
        q = np.asarray(b["q"], dtype=np.float64)
        assert q.shape[0] == 1 and q.shape[1] == len(modes)
        k_row = -q[0, :, sa] / gs
        if order == "mfp":
            part = k_row
        else:
            part = np.zeros(len(keys_all))
            for r in range(len(modes)):
                part[bins[r]] += k_row[r]
        return np.cumsum(part[idx])

    st = batch_statistics(batches, key=cum)
    return {"keys": keys_all[idx], "kappa_cum": st["mean"], "kappa_cum_sigma": st["sigma"]}


def default_lambda_split(w: dict) -> float:
    """The geometric length below which a mode's flights take the local pathwise form: the smallest
    bounded extent of the cell or pore diameter (infinite for the unbounded bulk)."""
    g = w["geometry"]
    sizes = [float(L) for L, u in zip(g["L"], g["unbounded"]) if not u]
    sizes += [2.0 * float(c[2]) for c in g["cylinders"]]
    return min(sizes) if sizes else math.inf


def adjoint(w: dict, n: int | None = None, first_pid: int = 0, threads: int = 1, n_batches: int = 1,
            tables: Tables | None = None, estimator: str = "score", per_particle: bool = False,
            lambda_split: float | None = None) -> dict:
    """Estimate of dkappa / dln tau_i (per frequency bin) over particles [first_pid, first_pid + n),
    with batch-mean standard errors when n_batches > 1.  estimator "score": likelihood ratios of
    the free flights (Eq. time_to_scat) and of the relaxation draws (Eq. norm_post_coll);
    "pathwise": the flights differentiated through their lengths (tangents carried along the
    trajectory), the draws by their likelihood ratios; "local": for modes with v tau <= lambda_split
    (default: the smallest bounded extent or pore diameter) a flight's own flux through its length
    and what follows by its likelihood ratio, other flights and the draws as for "score".

    dkappa/dln tau_i = -E_tot / (V_solid gradT_s n) * (sparse_i + P_i B), the same normalisation
    as kappa = -E_tot / (V_solid gradT_s n) * sum_p F_p (section 3.6, Eq. flux_x_steady).
    per_particle (pathwise only): also return each particle's tangent terms per bin, unscaled."""
    kind = {"score": 0, "pathwise": 1, "local": 2}[estimator]
    split = default_lambda_split(w) if lambda_split is None else float(lambda_split)
    tb = tables or Tables(w)
    n = w["problem"]["N"] if n is None else int(n)
    inst = int(w.get("instance", 0))
    nb = max(1, int(n_batches))
    bounds = [first_pid + (n * i) // nb for i in range(nb + 1)]

    def one(i):
        lo, hi = bounds[i], bounds[i + 1]
        sp = np.zeros(tb.n_bins)
        de = np.zeros(1)
        F = np.zeros(hi - lo)
        pp = np.zeros((hi - lo, tb.n_bins)) if per_particle else None
        bad = np.zeros(1, dtype=np.int64)
        rc = lib().orc_adjoint(tb.h, int(w["seed"]), inst, lo, hi - lo, kind, split, _ptr(sp), _ptr(de), _ptr(F),
                               _ptr(pp) if pp is not None else None, _ptr(bad))
        if rc != 0:
            raise ValueError(f"oracle adjoint failed with status {rc}")
        return sp, float(de[0]), F, pp, int(bad[0])

    with ThreadPoolExecutor(max(1, min(threads, nb))) as ex:
        parts = list(ex.map(one, range(nb)))
    g = w["geometry"]["gradT"][w["problem"]["score_axis"]]
    P = tb.get("P_bin")
    per_batch = []
    for (sp, de, F, _, _), lo, hi in zip(parts, bounds[:-1], bounds[1:]):
        scale = -tb.E_tot / (tb.V_solid * g * (hi - lo))
        per_batch.append(scale * (sp + P * de))
    sp = sum(p[0] for p in parts)
    de = sum(p[1] for p in parts)
    F = np.concatenate([p[2] for p in parts])
    scale = -tb.E_tot / (tb.V_solid * g * n)
    out = {"dkappa_dlntau": scale * (sp + P * de), "sparse": sp, "dense": de, "F": F, "P_bin": P,
           "kappa": scale * F.sum(), "tables": tb, "scale": scale, "n_nonfinite": sum(p[4] for p in parts)}
    if per_particle:
        out["per_particle"] = np.concatenate([p[3] for p in parts])
    if nb > 1:
        arr = np.array(per_batch)
        out["dkappa_dlntau_sigma"] = arr.std(0, ddof=1) / math.sqrt(nb)
        out["per_batch"] = arr
    return out
