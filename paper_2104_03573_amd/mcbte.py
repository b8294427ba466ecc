"""ctypes binding of libmcbte.so (include/mcbte.h): argument marshalling only.

Every step of the Monte Carlo path runs in the HIP kernels of the library; this module
only converts workload descriptions into the ABI structs, hands device pointers of torch
tensors and the current HIP stream to the library, and raises on error codes.  If the
library is not built, loading fails loudly: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libmcbte.so")

OK, EINVAL, ENOMEM, EHIP, ENODEV, ETABLE, EGEOM, ESIZE, ERANGE, ELIMIT = 0, -1, -2, -3, -4, -5, -6, -7, -8, -9
STATIC_MAX_INSTANCES = 64
N_COUNTS = 16
COUNT_NAMES = ["particles", "flights", "relaxations", "specular", "diffuse", "periodic", "absorbed",
               "timeouts", "nscat_end", "cap_end", "escaped", "rejections", "two_phonon"]
MAX_PORES = 8
TALLY_HEADER_BYTES = 256


class Mode(C.Structure):
    _fields_ = [("omega", C.c_double), ("dos", C.c_double), ("v", C.c_double), ("domega", C.c_double),
                ("tau", C.c_double), ("C", C.c_double), ("tau_imp", C.c_double),
                ("bin", C.c_int32), ("branch", C.c_int32)]


class Face(C.Structure):
    _fields_ = [("type", C.c_int32), ("spec_table", C.c_int32), ("data", C.c_double * 3)]


class Pore(C.Structure):
    _fields_ = [("cx", C.c_double), ("cy", C.c_double), ("r", C.c_double), ("id", C.c_int32),
                ("type", C.c_int32), ("specularity", C.c_double), ("spec_omega", C.c_double),
                ("spec_table", C.c_int32), ("reserved", C.c_int32)]


class Wall(C.Structure):
    _fields_ = [("x1", C.c_double), ("y1", C.c_double), ("x2", C.c_double), ("y2", C.c_double),
                ("nx", C.c_double), ("ny", C.c_double), ("id", C.c_int32), ("type", C.c_int32),
                ("data", C.c_double), ("spec_omega", C.c_double), ("spec_table", C.c_int32),
                ("reserved", C.c_int32)]


MAX_WALLS = 16


class Geometry(C.Structure):
    _fields_ = [("L", C.c_double * 3), ("unbounded", C.c_int32 * 3), ("n_pores", C.c_int32),
                ("face", Face * 6), ("pore", Pore * MAX_PORES), ("gradT", C.c_double * 3), ("volume", C.c_double),
                ("n_walls", C.c_int32), ("reserved_w", C.c_int32), ("wall", Wall * MAX_WALLS)]


class Detectors(C.Structure):
    _fields_ = [("lo", C.c_double * 3), ("hi", C.c_double * 3), ("n", C.c_int32 * 3), ("mask", C.c_int32)]


class ProblemC(C.Structure):
    _fields_ = [("N", C.c_int64), ("max_events", C.c_int64), ("T_lin", C.c_double), ("t_max", C.c_double),
                ("n_scat_max", C.c_int32), ("format", C.c_int32), ("transient", C.c_int32),
                ("score_axis", C.c_int32), ("n_times", C.c_int32), ("ic_axis", C.c_int32), ("n_ic", C.c_int32),
                ("n_spec_tables", C.c_int32), ("t_meas", C.POINTER(C.c_double)),
                ("ic_edges", C.POINTER(C.c_double)), ("ic_dT", C.POINTER(C.c_double)),
                ("spec_table", C.POINTER(C.c_double)), ("n_heat", C.c_int32), ("n_heat_tet", C.c_int32),
                ("heat_lo", C.c_double * 3), ("heat_hi", C.c_double * 3), ("heat_t", C.POINTER(C.c_double)),
                ("heat_P", C.POINTER(C.c_double)), ("heat_tet", C.POINTER(C.c_double))]


class Info(C.Structure):
    _fields_ = [("C_tot", C.c_double), ("sum_Cv", C.c_double), ("E_tot", C.c_double), ("e_eff", C.c_double),
                ("V_solid", C.c_double), ("kappa_bulk", C.c_double), ("n_modes", C.c_int64),
                ("n_sources", C.c_int64), ("n_cells", C.c_int64), ("n_cols", C.c_int64),
                ("tally_bytes", C.c_int64), ("n_bins", C.c_int64), ("adj_doubles", C.c_int64),
                ("device", C.c_int32), ("reserved", C.c_int32)]


class Run(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("instance", C.c_uint32), ("precision", C.c_int32), ("block", C.c_int32),
                ("refill", C.c_int32), ("grid", C.c_int32), ("log_stride", C.c_int32), ("n_log", C.c_int64),
                ("event_log", C.c_void_p), ("particle_F", C.c_void_p), ("flags", C.c_int32),
                ("reserved", C.c_int32)]


RUN_SEGMENTS = 1


class Result(C.Structure):
    _fields_ = [("counts", C.c_uint64 * N_COUNTS), ("moments", C.c_double * 4), ("e_eff", C.c_double),
                ("V_cell", C.c_double), ("T_mean", C.c_double), ("T_mean_sigma", C.c_double),
                ("q_score", C.c_double), ("q_score_sigma", C.c_double), ("kappa", C.c_double),
                ("kappa_sigma", C.c_double), ("kappa_cell_avg", C.c_double)]


EXPORTED = ["mcbte_build_tables", "mcbte_free_tables", "mcbte_table_info", "mcbte_table_export",
            "mcbte_state_bytes", "mcbte_emit", "mcbte_trace", "mcbte_batch_queue_bytes", "mcbte_trace_batch",
            "mcbte_adjoint", "mcbte_adjoint_finalize", "mcbte_tally", "mcbte_strerror", "mcbte_autotune",
            "mcbte_trace_batch_static", "mcbte_tally_batches", "mcbte_kappa_cumulative"]

CUM_MFP = 0
CUM_OMEGA = 1

_lib = None


def lib():
    """Load libmcbte.so (built by ``__graft_entry__.build()``); raises if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                               "(there is no CPU fallback for the HIP path)")
        L = C.CDLL(LIB_PATH)
        p = C.c_void_p
        L.mcbte_build_tables.argtypes = [C.POINTER(Mode), C.c_int32, C.POINTER(Geometry), C.POINTER(Detectors),
                                         C.POINTER(ProblemC), C.c_int32, C.POINTER(p)]
        L.mcbte_build_tables.restype = C.c_int
        L.mcbte_free_tables.argtypes = [p]
        L.mcbte_free_tables.restype = None
        L.mcbte_table_info.argtypes = [p, C.POINTER(Info)]
        L.mcbte_table_info.restype = C.c_int
        L.mcbte_table_export.argtypes = [p, C.c_int32, p, C.c_int64]
        L.mcbte_table_export.restype = C.c_int
        L.mcbte_state_bytes.argtypes = [C.c_int32, C.c_int64]
        L.mcbte_state_bytes.restype = C.c_int64
        L.mcbte_emit.argtypes = [p, C.POINTER(Run), C.c_int64, C.c_int64, p, C.c_int64, p]
        L.mcbte_emit.restype = C.c_int
        L.mcbte_trace.argtypes = [p, C.POINTER(Run), C.c_int64, C.c_int64, p, p, p]
        L.mcbte_trace.restype = C.c_int
        L.mcbte_batch_queue_bytes.argtypes = [C.c_int32]
        L.mcbte_batch_queue_bytes.restype = C.c_int64
        L.mcbte_trace_batch.argtypes = [C.POINTER(p), C.c_int32, C.POINTER(C.c_int64), C.POINTER(C.c_uint32),
                                        C.POINTER(p), C.POINTER(Run), p, p]
        L.mcbte_trace_batch.restype = C.c_int
        L.mcbte_trace_batch_static.argtypes = [C.POINTER(p), C.c_int32, C.POINTER(C.c_int64), C.POINTER(C.c_uint32),
                                               C.POINTER(p), C.POINTER(Run), p]
        L.mcbte_trace_batch_static.restype = C.c_int
        L.mcbte_autotune.argtypes = [C.POINTER(p), C.c_int32, C.POINTER(C.c_int64), C.POINTER(C.c_uint32),
                                     C.POINTER(p), p, C.POINTER(Run), C.c_int64, C.c_int32, C.POINTER(Run),
                                     C.POINTER(C.c_double), C.c_int32, p]
        L.mcbte_autotune.restype = C.c_int
        L.mcbte_adjoint.argtypes = [p, C.POINTER(Run), C.c_int32, C.c_double, C.c_int64, C.c_int64, p, p, p]
        L.mcbte_adjoint.restype = C.c_int
        L.mcbte_adjoint_finalize.argtypes = [p, p, C.c_int64, C.POINTER(C.c_double), C.c_int64, p]
        L.mcbte_adjoint_finalize.restype = C.c_int
        L.mcbte_tally.argtypes = [p, p, C.POINTER(C.c_double), C.c_int64, C.POINTER(Result), p]
        L.mcbte_tally.restype = C.c_int
        L.mcbte_tally_batches.argtypes = [p, C.POINTER(p), C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                          C.c_int64, p]
        L.mcbte_tally_batches.restype = C.c_int
        L.mcbte_kappa_cumulative.argtypes = [p, C.POINTER(p), C.c_int32, C.c_int32, C.POINTER(C.c_double),
                                             C.POINTER(C.c_double), C.POINTER(C.c_double), C.c_int64, p]
        L.mcbte_kappa_cumulative.restype = C.c_int
        L.mcbte_strerror.argtypes = [C.c_int]
        L.mcbte_strerror.restype = C.c_char_p
        _lib = L
    return _lib


class MCBTEError(RuntimeError):
    def __init__(self, fn: str, status: int):
        super().__init__(f"{fn}: {strerror(status)} ({status})")
        self.status = status


def strerror(status: int) -> str:
    return lib().mcbte_strerror(status).decode()


def _check(fn: str, status: int):
    if status != OK:
        raise MCBTEError(fn, status)


def _stream(stream):
    if stream is None:
        import torch
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    return C.c_void_p(stream)


# ------------------------------------------------------------------------------------------
# marshalling of workload descriptions
# ------------------------------------------------------------------------------------------

def structs_from_workload(w: dict):
    """Workload dict (see the workloads package) -> (modes array, Geometry, Detectors, ProblemC, keepalive)."""
    modes_np = np.ascontiguousarray(w["modes"])
    modes = (Mode * len(modes_np))()
    for i, r in enumerate(modes_np):
        modes[i] = Mode(float(r["omega"]), float(r["dos"]), float(r["v"]), float(r["domega"]), float(r["tau"]),
                        float(r["C"]), float(r["tau_imp"]), int(r["bin"]), int(r["branch"]))
    g = w["geometry"]
    G = Geometry()
    for a in range(3):
        G.L[a] = g["L"][a]
        G.unbounded[a] = int(bool(g["unbounded"][a]))
        G.gradT[a] = g["gradT"][a]
    for fid, f in g["faces"].items():
        G.face[fid - 1].type = int(f[0])
        G.face[fid - 1].data[0], G.face[fid - 1].data[1], G.face[fid - 1].data[2] = f[1], f[2], f[3]
        G.face[fid - 1].spec_table = int(f[4]) if len(f) > 4 else 0
    walls = g.get("walls", [])
    if len(walls) > MAX_WALLS:
        raise ValueError(f"at most {MAX_WALLS} internal line walls")
    G.n_walls = len(walls)
    for i, c in enumerate(walls):
        x1, y1, x2, y2, nx, ny, wid, ty, spec = c[:9]
        G.wall[i] = Wall(x1, y1, x2, y2, nx, ny, int(wid), int(ty), spec, float(c[9]) if len(c) > 9 else 0.0,
                         int(c[10]) if len(c) > 10 else 0, 0)
    G.n_pores = len(g["cylinders"])
    for i, c in enumerate(g["cylinders"]):
        cx, cy, r, cid, ty, spec = c[:6]
        G.pore[i] = Pore(cx, cy, r, int(cid), int(ty), spec, float(c[6]) if len(c) > 6 else 0.0,
                         int(c[7]) if len(c) > 7 else 0, 0)
    G.volume = g["volume"]
    d = w["detectors"]
    D = Detectors()
    for a in range(3):
        D.lo[a], D.hi[a], D.n[a] = d["lo"][a], d["hi"][a], d["n"][a]
    D.mask = d["mask"]
    p = w["problem"]
    spec = np.ascontiguousarray(p.get("spec_tables", np.zeros((0, len(modes_np)))), dtype=np.float64)
    keep = [np.ascontiguousarray(p["t_meas"], dtype=np.float64),
            np.ascontiguousarray(p["ic_edges"], dtype=np.float64),
            np.ascontiguousarray(p["ic_dT"], dtype=np.float64), spec]
    dp = C.POINTER(C.c_double)
    P = ProblemC(p["N"], p["max_events"], p["T_lin"], p["t_max"], p["n_scat_max"], p["format"], int(p["transient"]),
                 p["score_axis"], len(keep[0]) if p["transient"] else 0, p["ic_axis"], len(keep[2]), spec.shape[0],
                 keep[0].ctypes.data_as(dp), keep[1].ctypes.data_as(dp), keep[2].ctypes.data_as(dp),
                 spec.ctypes.data_as(dp) if spec.shape[0] else None)
    heat = p.get("heat")
    if heat is not None:
        ht = np.ascontiguousarray(heat["t"], dtype=np.float64)
        hP = np.ascontiguousarray(heat["P"], dtype=np.float64)
        keep += [ht, hP]
        P.n_heat = len(hP)
        for a in range(3):
            P.heat_lo[a], P.heat_hi[a] = heat["lo"][a], heat["hi"][a]
        P.heat_t, P.heat_P = ht.ctypes.data_as(dp), hP.ctypes.data_as(dp)
        if heat.get("tets") is not None:
            tets = np.ascontiguousarray(heat["tets"], dtype=np.float64).reshape(-1, 12)
            keep.append(tets)
            P.n_heat_tet = tets.shape[0]
            P.heat_tet = tets.ctypes.data_as(dp)
    return modes, G, D, P, keep


# ------------------------------------------------------------------------------------------
# the C ABI, one Python function per entry point
# ------------------------------------------------------------------------------------------

def build_tables(w: dict, device: int = 0) -> "Tables":
    return Tables(w, device)


def free_tables(t: "Tables"):
    t.free()


def table_info(t: "Tables") -> dict:
    info = Info()
    _check("mcbte_table_info", lib().mcbte_table_info(t.h, C.byref(info)))
    return {k: getattr(info, k) for k, _ in Info._fields_ if k != "reserved"}


def table_export(t: "Tables", which: str) -> np.ndarray:
    code, dt = {"C": (0, np.float64), "thr_ic": (1, np.uint64), "thr_wall": (2, np.uint64),
                "thr_rel": (3, np.uint64), "src_E": (4, np.float64), "thr_src": (5, np.uint64),
                "src_sign": (6, np.int32)}[which]
    n = t.info["n_modes"] if code <= 3 else t.info["n_sources"]
    out = np.zeros(n, dtype=dt)
    _check("mcbte_table_export", lib().mcbte_table_export(t.h, code, out.ctypes.data_as(C.c_void_p), n))
    return out


def state_bytes(precision: int, capacity: int) -> int:
    n = lib().mcbte_state_bytes(precision, capacity)
    if n < 0:
        raise MCBTEError("mcbte_state_bytes", int(n))
    return int(n)


def make_run(seed: int, precision: int = 32, instance: int = 0, block: int = 0, refill: int = 0, grid: int = 0,
             event_log=None, n_log: int = 0, log_stride: int = 64, particle_F=None, segments: bool = False) -> Run:
    """segments=True sets MCBTE_RUN_SEGMENTS (FP32 pore lattices traced one segment at a time)."""
    return Run(seed & 0xFFFFFFFFFFFFFFFF, instance, precision, block, refill, grid, log_stride,
               n_log if event_log is not None else 0,
               C.c_void_p(event_log.data_ptr()) if event_log is not None else None,
               C.c_void_p(particle_F.data_ptr()) if particle_F is not None else None,
               RUN_SEGMENTS if segments else 0, 0)


def emit(t: "Tables", run: Run, first_pid: int, n: int, state, capacity: int, stream=None):
    _check("mcbte_emit", lib().mcbte_emit(t.h, C.byref(run), first_pid, n, C.c_void_p(state.data_ptr()), capacity,
                                          _stream(stream)))


def trace(t: "Tables", run: Run, first_pid: int, n: int, state, tally, stream=None):
    st = C.c_void_p(state.data_ptr()) if state is not None else None
    _check("mcbte_trace", lib().mcbte_trace(t.h, C.byref(run), first_pid, n, st, C.c_void_p(tally.data_ptr()),
                                            _stream(stream)))


def batch_queue_bytes(n_inst: int) -> int:
    n = lib().mcbte_batch_queue_bytes(n_inst)
    if n < 0:
        raise MCBTEError("mcbte_batch_queue_bytes", int(n))
    return int(n)


def trace_batch(tables: list, n_particles, instance_ids, tallies: list, run: Run, queue, stream=None):
    k = len(tables)
    th = (C.c_void_p * k)(*[t.h for t in tables])
    npart = (C.c_int64 * k)(*[int(x) for x in n_particles])
    ids = (C.c_uint32 * k)(*[int(x) for x in instance_ids])
    tp = (C.c_void_p * k)(*[tl.data_ptr() for tl in tallies])
    _check("mcbte_trace_batch", lib().mcbte_trace_batch(th, k, npart, ids, tp, C.byref(run),
                                                        C.c_void_p(queue.data_ptr()), _stream(stream)))


def trace_batch_static(tables: list, n_particles, instance_ids, tallies: list, run: Run, stream=None):
    """The batched trace with the library's static work queue (no queue buffer; allocates nothing)."""
    k = len(tables)
    th = (C.c_void_p * k)(*[t.h for t in tables])
    npart = (C.c_int64 * k)(*[int(x) for x in n_particles])
    ids = (C.c_uint32 * k)(*[int(x) for x in instance_ids])
    tp = (C.c_void_p * k)(*[tl.data_ptr() for tl in tallies])
    _check("mcbte_trace_batch_static", lib().mcbte_trace_batch_static(th, k, npart, ids, tp, C.byref(run),
                                                                      _stream(stream)))


TUNE_CANDIDATES = 36
TUNE_BLOCKS = (64, 128, 192, 256, 512, 1024)


def tune_candidate(c: int) -> tuple[int, int]:
    """(block, refill) of autotuner candidate c."""
    return TUNE_BLOCKS[c // 6], 1 << (c % 6)


def autotune(tables: list, n_particles, instance_ids, tallies: list, queue, base: Run, n_probe: int,
             reps: int = 3, stream=None) -> tuple[Run, np.ndarray]:
    k = len(tables)
    th = (C.c_void_p * k)(*[t.h for t in tables])
    npart = (C.c_int64 * k)(*[int(x) for x in n_particles])
    ids = (C.c_uint32 * k)(*[int(x) for x in instance_ids])
    tp = (C.c_void_p * k)(*[tl.data_ptr() for tl in tallies])
    out = Run()
    tim = (C.c_double * TUNE_CANDIDATES)()
    _check("mcbte_autotune", lib().mcbte_autotune(th, k, npart, ids, tp,
                                                  C.c_void_p(queue.data_ptr()) if queue is not None else None,
                                                  C.byref(base), int(n_probe), int(reps), C.byref(out), tim,
                                                  TUNE_CANDIDATES, _stream(stream)))
    return out, np.array(tim[:])


def tune(w, precision: int = 32, n_probe: int = 1 << 18, reps: int = 3, tables=None, device: int = 0,
         segments: bool = False) -> dict:
    """Autotune the launch shape for a workload (dict) or a sweep (list of dicts, batched form)."""
    import torch
    ws = w if isinstance(w, list) else [w]
    tabs = tables or [Tables(x, device) for x in ws]
    tabs = tabs if isinstance(tabs, list) else [tabs]
    tallies = [t.new_tally() for t in tabs]
    queue = (torch.zeros(batch_queue_bytes(len(ws)), dtype=torch.uint8, device=f"cuda:{device}")
             if len(ws) > 1 else None)
    base = make_run(int(ws[0]["seed"]), precision, segments=segments)
    run_, tim = autotune(tabs, [x["problem"]["N"] for x in ws], [int(x.get("instance", 0)) for x in ws], tallies,
                         queue, base, n_probe, reps)
    return {"block": run_.block, "refill": run_.refill, "timings_ms": tim, "tables": tabs}


SENS_SCORE = 0
SENS_PATHWISE = 1
SENS_LOCAL = 2
ESTIMATORS = {"score": SENS_SCORE, "pathwise": SENS_PATHWISE, "local": SENS_LOCAL}


def adjoint(t: "Tables", run: Run, estimator: int, first_pid: int, n: int, particle_F, adj, stream=None,
            lambda_split: float = 0.0):
    _check("mcbte_adjoint", lib().mcbte_adjoint(t.h, C.byref(run), estimator, float(lambda_split), first_pid, n,
                                                C.c_void_p(particle_F.data_ptr()), C.c_void_p(adj.data_ptr()),
                                                _stream(stream)))


def adjoint_finalize(t: "Tables", adj, n_particles: int, stream=None) -> np.ndarray:
    nb = t.info["n_bins"]
    out = np.zeros(nb)
    _check("mcbte_adjoint_finalize", lib().mcbte_adjoint_finalize(
        t.h, C.c_void_p(adj.data_ptr()), n_particles, out.ctypes.data_as(C.POINTER(C.c_double)), nb, _stream(stream)))
    return out


def tally(t: "Tables", tally_buf, stream=None, with_arrays: bool = True) -> dict:
    res = Result()
    n = t.info["n_cells"] * t.info["n_cols"] * 4
    out = np.zeros(n) if with_arrays else None
    ptr = out.ctypes.data_as(C.POINTER(C.c_double)) if with_arrays else None
    _check("mcbte_tally", lib().mcbte_tally(t.h, C.c_void_p(tally_buf.data_ptr()), ptr, n if with_arrays else 0,
                                            C.byref(res), _stream(stream)))
    r = {k: getattr(res, k) for k, _ in Result._fields_ if k not in ("counts", "moments")}
    r["counts_raw"] = np.array(res.counts[:], dtype=np.uint64)
    r["counts"] = dict(zip(COUNT_NAMES, [int(x) for x in res.counts[:len(COUNT_NAMES)]]))
    r["moments"] = np.array(res.moments[:])
    if with_arrays:
        arr = out.reshape(t.info["n_cells"], t.info["n_cols"], 4)
        r["T"] = arr[..., 0]
        r["q"] = arr[..., 1:]
    return r


def _ptr_array(bufs):
    arr = (C.c_void_p * len(bufs))(*[b.data_ptr() for b in bufs])
    return C.cast(arr, C.POINTER(C.c_void_p)), arr


def _dptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double)) if a is not None else None


def tally_batches(t: "Tables", tallies, stream=None) -> dict:
    """Finalized T and q, particle-weighted over the tally buffers `tallies` (each its own particle
    group), with batch-mean standard errors (NaN for one buffer): arrays (n_cells, n_cols)."""
    n = t.info["n_cells"] * t.info["n_cols"] * 4
    mean, sig = np.zeros(n), np.zeros(n)
    pa, keep = _ptr_array(tallies)
    _check("mcbte_tally_batches", lib().mcbte_tally_batches(t.h, pa, len(tallies), _dptr(mean), _dptr(sig), n,
                                                            _stream(stream)))
    shape = (t.info["n_cells"], t.info["n_cols"], 4)
    mean, sig = mean.reshape(shape), sig.reshape(shape)
    return {"T": mean[..., 0], "q": mean[..., 1:], "T_sigma": sig[..., 0], "q_sigma": sig[..., 1:]}


def kappa_cumulative(t: "Tables", tallies, order: str = "mfp", stream=None) -> dict:
    """Cumulative kappa over table rows by ascending mean free path (order "mfp") or over frequency
    bins by ascending angular frequency ("omega"): keys, kappa_cum and its batch-mean standard error."""
    k = t.info["n_modes"] if order == "mfp" else t.info["n_bins"]
    keys, cum, sig = np.zeros(k), np.zeros(k), np.zeros(k)
    pa, keep = _ptr_array(tallies)
    _check("mcbte_kappa_cumulative", lib().mcbte_kappa_cumulative(
        t.h, pa, len(tallies), CUM_MFP if order == "mfp" else CUM_OMEGA, _dptr(keys), _dptr(cum), _dptr(sig), k,
        _stream(stream)))
    return {"keys": keys, "kappa_cum": cum, "kappa_cum_sigma": sig}


class Tables:
    """Owner of one mcbte_tables handle."""

    def __init__(self, w: dict, device: int = 0):
        self.w = w
        modes, G, D, P, keep = structs_from_workload(w)
        h = C.c_void_p()
        _check("mcbte_build_tables", lib().mcbte_build_tables(modes, len(modes), C.byref(G), C.byref(D), C.byref(P),
                                                              device, C.byref(h)))
        self.h = h
        self.device = device
        self.info = table_info(self)

    def free(self):
        if getattr(self, "h", None):
            lib().mcbte_free_tables(self.h)
            self.h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    def new_tally(self):
        import torch
        return torch.zeros(self.info["tally_bytes"], dtype=torch.uint8, device=f"cuda:{self.device}")

    def raw(self, tally_buf) -> np.ndarray:
        """Raw sums of a tally buffer (n_cells, n_cols, 4), copied to the host."""
        import torch
        nbytes = self.info["n_cells"] * self.info["n_cols"] * 4 * 8
        b = tally_buf[TALLY_HEADER_BYTES:TALLY_HEADER_BYTES + nbytes].view(torch.float64).cpu().numpy()
        return b.reshape(self.info["n_cells"], self.info["n_cols"], 4)


def run(w: dict, n: int | None = None, first_pid: int = 0, precision: int = 32, device: int = 0,
        n_log: int = 0, log_stride: int = 64, emit_first: bool = False, tables: Tables | None = None,
        **launch) -> dict:
    """Build (or reuse) tables, trace particles [first_pid, first_pid + n) and finalize."""
    import torch
    t = tables or Tables(w, device)
    n = w["problem"]["N"] if n is None else int(n)
    tl = t.new_tally()
    log = torch.zeros(max(n_log, 1) * log_stride, dtype=torch.int32, device=f"cuda:{device}") if n_log else None
    r = make_run(int(w["seed"]), precision, int(w.get("instance", 0)), event_log=log, n_log=n_log,
                 log_stride=log_stride, **launch)
    state = None
    if emit_first:
        state = torch.zeros(state_bytes(precision, n), dtype=torch.uint8, device=f"cuda:{device}")
        emit(t, r, first_pid, n, state, n)
    trace(t, r, first_pid, n, state, tl)
    out = tally(t, tl)
    out["raw"] = t.raw(tl)
    out["tables"] = t
    if n_log:
        out["log"] = log.view(n_log, log_stride).cpu().numpy().view(np.uint32)
    return out


def sensitivities(w: dict, n: int | None = None, first_pid: int = 0, precision: int = 32, device: int = 0,
                  tables: Tables | None = None, estimator: str = "local", lambda_split: float = 0.0,
                  **launch) -> dict:
    """Forward trace (recording each particle's flux score) then the replay that accumulates the
    sensitivity sums of `estimator` ("score", "pathwise" or "local"; lambda_split <= 0: the
    library's default split for "local"): kappa and dkappa / dln tau_i per frequency bin."""
    import torch
    t = tables or Tables(w, device)
    n = w["problem"]["N"] if n is None else int(n)
    dev = f"cuda:{device}"
    F = torch.zeros(n, dtype=torch.float64, device=dev)
    tl = t.new_tally()
    if estimator == "pathwise":
        # the pathwise replay carries its tangents through every transfer of the forward trace
        launch.setdefault("segments", True)
    r = make_run(int(w["seed"]), precision, int(w.get("instance", 0)), particle_F=F, **launch)
    trace(t, r, first_pid, n, None, tl)
    adj = torch.zeros(t.info["adj_doubles"], dtype=torch.float64, device=dev)
    r2 = make_run(int(w["seed"]), precision, int(w.get("instance", 0)), **launch)
    adjoint(t, r2, ESTIMATORS[estimator], first_pid, n, F, adj, lambda_split=lambda_split)
    out = tally(t, tl, with_arrays=False)
    out["dkappa_dlntau"] = adjoint_finalize(t, adj, n)
    out["F"] = F.cpu().numpy()
    out["adj_raw"] = adj.cpu().numpy()
    out["tables"] = t
    return out
