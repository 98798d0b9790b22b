"""ctypes binding of libmdeos (the C ABI declared in include/mdeos.h).

The functions carry the C entry-point names and only marshal arguments:
every step of lift, advance and restrict runs in the HIP kernels of
libmdeos.so. Loading fails loudly when the library has not been built; there
is no CPU fallback. Streams may be given as a raw hipStream_t (int), an
object with a ``cuda_stream`` attribute (a torch stream on ROCm), or None
(the context's own stream).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmdeos.so")

OK, INVALID_ARG, OUT_OF_MEMORY, DEVICE_ERROR, NOT_READY, ADMISSION_FULL, NO_DEVICE = 0, -1, -2, -3, -4, -5, -6
CELL_NONFINITE, CELL_ENERGY_BELOW_COLD, CELL_DRIFT, CELL_OVERFLOW, CELL_COLD_RELIFT = 1, 2, 4, 8, 16
PREC_FP64, PREC_KAHAN = 0, 1
NVE_REPIN, NVT_LANGEVIN = 0, 1
POT_LJTS, POT_EAM = 0, 1
MAX_RESCALE = 8


class CellSpec(C.Structure):
    _fields_ = [("rho", C.c_double), ("e", C.c_double), ("n_c", C.c_int), ("rc", C.c_float), ("dt", C.c_double),
                ("seed", C.c_ulonglong), ("cell_id", C.c_longlong)]


class Schedule(C.Structure):
    _fields_ = [("n_steps", C.c_int), ("n_avg", C.c_int), ("n_blocks", C.c_int), ("n_rescale", C.c_int),
                ("rescale_steps", C.c_int * MAX_RESCALE), ("energy_every", C.c_int), ("drift_tol", C.c_double),
                ("ensemble", C.c_int), ("gamma", C.c_double)]


class Result(C.Structure):
    _fields_ = [("P", C.c_double), ("P_se", C.c_double), ("P_rms", C.c_double), ("T", C.c_double),
                ("T_se", C.c_double), ("Epot_mean", C.c_double), ("Ecold", C.c_double), ("drift", C.c_double),
                ("pairs", C.c_double), ("n_samples", C.c_int), ("status", C.c_int), ("n_builds", C.c_int),
                ("max_list", C.c_int), ("max_ext", C.c_int), ("reserved", C.c_int), ("stress", C.c_double * 6)]


class Config(C.Structure):
    _fields_ = [("device", C.c_int), ("hbm_budget", C.c_size_t), ("skin", C.c_float), ("autotune", C.c_int),
                ("tune_cache", C.c_char_p),
                ("precision", C.c_int), ("potential", C.c_int), ("eam_c", C.c_double), ("prune_skin", C.c_float)]


class PlanInfo(C.Structure):
    _fields_ = [("N", C.c_int), ("L", C.c_float), ("rl", C.c_float), ("ext_cap", C.c_int), ("list_cap", C.c_int),
                ("ncell", C.c_int), ("lds_bytes", C.c_int), ("list_in_lds", C.c_int), ("multi_image", C.c_int)]


class ServeConfig(C.Structure):
    _fields_ = [("cold", Schedule), ("warm", Schedule), ("rc", C.c_float), ("dt", C.c_double),
                ("seed", C.c_ulonglong), ("chunk_steps", C.c_int), ("max_slots", C.c_int)]


class ServeStats(C.Structure):
    _fields_ = [("submitted", C.c_longlong), ("completed", C.c_longlong), ("cold", C.c_longlong),
                ("warm", C.c_longlong), ("relifts", C.c_longlong), ("evictions", C.c_longlong),
                ("chunks", C.c_longlong), ("queued", C.c_longlong), ("active", C.c_longlong),
                ("resident", C.c_longlong), ("resident_bytes", C.c_size_t), ("atom_steps", C.c_double)]


RESULT_DTYPE = np.dtype([("P", "f8"), ("P_se", "f8"), ("P_rms", "f8"), ("T", "f8"), ("T_se", "f8"),
                         ("Epot_mean", "f8"), ("Ecold", "f8"), ("drift", "f8"), ("pairs", "f8"),
                         ("n_samples", "i4"), ("status", "i4"), ("n_builds", "i4"), ("max_list", "i4"),
                         ("max_ext", "i4"), ("reserved", "i4"), ("stress", "f8", (6,))])
assert RESULT_DTYPE.itemsize == C.sizeof(Result)

EXPORTED = [
    "mdeos_strerror", "mdeos_last_error", "mdeos_version", "mdeos_validate", "mdeos_plan", "mdeos_cell_bytes",
    "mdeos_device_count", "mdeos_create", "mdeos_destroy", "mdeos_lift", "mdeos_lift_from_state",
    "mdeos_warm_start", "mdeos_advance", "mdeos_restrict", "mdeos_eval_batch", "mdeos_eval_plain",
    "mdeos_eval_batch_noalloc",
    "mdeos_release", "mdeos_last_advance_time", "mdeos_state_export", "mdeos_debug_forces", "mdeos_debug_trajectory", "mdeos_serve_start",
    "mdeos_serve_submit", "mdeos_serve_poll", "mdeos_serve_now", "mdeos_serve_stats_get", "mdeos_serve_stop",
]


class MdeosError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        lib = _lib
        msg = lib.mdeos_strerror(status).decode() if lib else str(status)
        detail = lib.mdeos_last_error().decode() if lib else ""
        super().__init__(f"{what}: {msg} ({status}) {detail}".strip())


_lib = None


def hip_runtimes() -> set:
    """Paths of the HIP runtime libraries (libamdhip64) mapped into this process."""
    paths = set()
    try:
        with open("/proc/self/maps") as f:
            for line in f:
                if "libamdhip64" in line:
                    paths.add(line.split()[-1])
    except OSError:
        pass
    return paths


def lib() -> C.CDLL:
    """Loads libmdeos.so; raises if it was not built (no fallback).

    One HIP runtime per process: PyTorch ships its own copy of the HIP runtime
    under the same soname as the system's. When torch is importable it is
    imported first, so the library binds to that copy and torch streams, torch
    memory and the library's work share one runtime. Loaded the other way
    round, the process maps both runtimes, each with its own device state and
    hardware queues, and a torch stream is foreign to the library."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2508_06012_amd.build`")
    try:
        import torch  # noqa: F401  (maps torch's HIP runtime before the library resolves its own)
    except ImportError:
        pass
    L = C.CDLL(LIB_PATH)
    P = C.POINTER
    vp = C.c_void_p
    dp = P(C.c_double)
    L.mdeos_strerror.argtypes = [C.c_int]
    L.mdeos_strerror.restype = C.c_char_p
    L.mdeos_last_error.restype = C.c_char_p
    L.mdeos_version.restype = C.c_char_p
    L.mdeos_validate.argtypes = [P(CellSpec), P(Schedule)]
    L.mdeos_plan.argtypes = [P(CellSpec), C.c_float, P(PlanInfo)]
    L.mdeos_cell_bytes.argtypes = [C.c_int]
    L.mdeos_cell_bytes.restype = C.c_size_t
    L.mdeos_create.argtypes = [P(Config), P(vp)]
    L.mdeos_destroy.argtypes = [vp]
    L.mdeos_lift.argtypes = [vp, C.c_int, P(CellSpec), P(Schedule), P(C.c_longlong), vp]
    L.mdeos_lift_from_state.argtypes = [vp, P(CellSpec), P(Schedule), dp, dp, P(C.c_longlong), vp]
    L.mdeos_warm_start.argtypes = [vp, C.c_int, P(C.c_longlong), dp, dp, P(Schedule), vp]
    L.mdeos_advance.argtypes = [vp, C.c_int, P(C.c_longlong), C.c_int, vp]
    L.mdeos_restrict.argtypes = [vp, C.c_int, P(C.c_longlong), P(Result), vp]
    L.mdeos_eval_batch.argtypes = [vp, C.c_int, P(CellSpec), P(Schedule), P(Result), vp]
    L.mdeos_eval_plain.argtypes = [vp, C.c_int, P(CellSpec), P(Schedule), P(Result), vp]
    L.mdeos_eval_batch_noalloc.argtypes = [vp, C.c_int, P(CellSpec), P(Schedule), P(Result), vp]
    L.mdeos_release.argtypes = [vp, C.c_int, P(C.c_longlong)]
    L.mdeos_last_advance_time.argtypes = [vp, dp, P(C.c_int)]
    L.mdeos_state_export.argtypes = [vp, C.c_longlong, dp, dp, P(C.c_int)]
    L.mdeos_debug_forces.argtypes = [vp, P(CellSpec), dp, dp, dp, dp]
    L.mdeos_debug_trajectory.argtypes = [vp, C.c_longlong, C.c_int, dp, dp, dp, dp]
    L.mdeos_serve_start.argtypes = [vp, P(ServeConfig)]
    L.mdeos_serve_submit.argtypes = [vp, C.c_longlong, C.c_double, C.c_double, C.c_int, C.c_double,
                                     P(C.c_longlong)]
    L.mdeos_serve_poll.argtypes = [vp, C.c_int, P(C.c_longlong), P(Result), dp, P(C.c_int)]
    L.mdeos_serve_now.argtypes = [vp]
    L.mdeos_serve_now.restype = C.c_double
    L.mdeos_serve_stats_get.argtypes = [vp, P(ServeStats)]
    L.mdeos_serve_stop.argtypes = [vp, C.c_int]
    _lib = L
    return L


def _check(st: int, what: str) -> None:
    if st != OK:
        raise MdeosError(st, what)


def _stream(stream) -> C.c_void_p:
    if stream is None:
        return None
    if hasattr(stream, "cuda_stream"):
        rt = hip_runtimes()
        if len(rt) > 1:
            raise MdeosError(INVALID_ARG, "a torch stream with two HIP runtimes mapped (" + ", ".join(sorted(rt)) +
                             "): import torch before loading libmdeos.so, so both use one runtime")
        return C.c_void_p(int(stream.cuda_stream))
    return C.c_void_p(int(stream))


def _spec_array(specs):
    if isinstance(specs, CellSpec):
        specs = [specs]
    if isinstance(specs, C.Array):
        return specs
    return (CellSpec * len(specs))(*specs)


def _dp(a: np.ndarray | None):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(C.POINTER(C.c_double))


# --- builders ---------------------------------------------------------------

def make_schedule(n_steps: int, n_avg: int, rescale_steps=(), n_blocks: int = 10, energy_every: int = 10,
                  drift_tol: float = 0.05, ensemble: int = 0, gamma: float = 0.0) -> Schedule:
    s = Schedule()
    s.n_steps, s.n_avg, s.n_blocks = n_steps, n_avg, n_blocks
    s.n_rescale = len(rescale_steps)
    for i, k in enumerate(rescale_steps):
        s.rescale_steps[i] = int(k)
    s.energy_every, s.drift_tol = energy_every, drift_tol
    s.ensemble, s.gamma = ensemble, gamma
    return s


def make_specs(rho, e, n_c, rc, dt, seed, cell_id) -> C.Array:
    """Array of cell specs; every argument is a scalar or has one entry per cell."""
    rho = np.atleast_1d(np.asarray(rho, dtype=float))
    n = rho.size
    seeds = np.broadcast_to(np.asarray(seed, dtype=object), (n,))
    e = np.broadcast_to(np.asarray(e, dtype=float), (n,))
    n_c = np.broadcast_to(np.asarray(n_c, dtype=int), (n,))
    rc = np.broadcast_to(np.asarray(rc, dtype=float), (n,))
    dt = np.broadcast_to(np.asarray(dt, dtype=float), (n,))
    cid = np.broadcast_to(np.asarray(cell_id, dtype=np.int64), (n,))
    arr = (CellSpec * n)()
    for i in range(n):
        arr[i] = CellSpec(float(rho[i]), float(e[i]), int(n_c[i]), float(rc[i]), float(dt[i]),
                          int(seeds[i]) & (2 ** 64 - 1), int(cid[i]))
    return arr


def specs_from_workload(w) -> tuple[C.Array, Schedule]:
    s = w.sched
    return (make_specs(w.rho, w.e, w.n_c, w.rc, w.dt, w.seed, w.cell_id),
            make_schedule(s.n_steps, s.n_avg, s.rescale_steps, s.n_blocks, s.energy_every, s.drift_tol))


def results_to_numpy(res) -> np.ndarray:
    return np.frombuffer(bytes(res), dtype=RESULT_DTYPE).copy()


# --- entry points (C-ABI names) ----------------------------------------------

def mdeos_version() -> str:
    return lib().mdeos_version().decode()


def mdeos_device_count() -> int:
    return lib().mdeos_device_count()


def mdeos_validate(spec: CellSpec, sched: Schedule | None = None) -> int:
    return lib().mdeos_validate(C.byref(spec), C.byref(sched) if sched is not None else None)


def mdeos_plan(spec: CellSpec, skin: float = 0.0) -> PlanInfo:
    info = PlanInfo()
    _check(lib().mdeos_plan(C.byref(spec), skin, C.byref(info)), "mdeos_plan")
    return info


def mdeos_cell_bytes(n_c: int) -> int:
    return lib().mdeos_cell_bytes(n_c)


def mdeos_create(device: int = 0, hbm_budget: int = 0, skin: float = 0.0, autotune: int = 0,
                 tune_cache: str | None = None, precision: int = 0, potential: int = 0,
                 eam_c: float = 0.0, prune_skin: float = 0.0) -> C.c_void_p:
    cfg = Config(device, hbm_budget, skin, autotune, tune_cache.encode() if tune_cache else None, precision,
                 potential, eam_c, prune_skin)
    ctx = C.c_void_p()
    _check(lib().mdeos_create(C.byref(cfg), C.byref(ctx)), "mdeos_create")
    return ctx


def mdeos_destroy(ctx) -> None:
    _check(lib().mdeos_destroy(ctx), "mdeos_destroy")


def mdeos_lift(ctx, specs, sched: Schedule, stream=None) -> np.ndarray:
    specs = _spec_array(specs)
    n = len(specs)
    h = (C.c_longlong * n)()
    _check(lib().mdeos_lift(ctx, n, specs, C.byref(sched), h, _stream(stream)), "mdeos_lift")
    return np.array(list(h), dtype=np.int64)


def mdeos_lift_from_state(ctx, spec: CellSpec, sched: Schedule, xyz: np.ndarray, v: np.ndarray, stream=None) -> int:
    xyz = np.ascontiguousarray(xyz, dtype=np.float64)
    v = np.ascontiguousarray(v, dtype=np.float64)
    h = C.c_longlong()
    _check(lib().mdeos_lift_from_state(ctx, C.byref(spec), C.byref(sched), _dp(xyz), _dp(v), C.byref(h),
                                       _stream(stream)), "mdeos_lift_from_state")
    return h.value


def _handles(h) -> C.Array:
    h = np.atleast_1d(np.asarray(h, dtype=np.int64))
    return (C.c_longlong * h.size)(*[int(x) for x in h])


def mdeos_warm_start(ctx, handles, rho, e, sched: Schedule, stream=None) -> None:
    hh = _handles(handles)
    n = len(hh)
    r = np.ascontiguousarray(np.broadcast_to(np.asarray(rho, dtype=float), (n,)))
    ee = np.ascontiguousarray(np.broadcast_to(np.asarray(e, dtype=float), (n,)))
    _check(lib().mdeos_warm_start(ctx, n, hh, _dp(r), _dp(ee), C.byref(sched), _stream(stream)), "mdeos_warm_start")


def mdeos_advance(ctx, handles, n_steps: int, stream=None) -> None:
    hh = _handles(handles)
    _check(lib().mdeos_advance(ctx, len(hh), hh, n_steps, _stream(stream)), "mdeos_advance")


def mdeos_restrict(ctx, handles, stream=None, allow_not_ready: bool = False) -> np.ndarray:
    hh = _handles(handles)
    out = (Result * len(hh))()
    st = lib().mdeos_restrict(ctx, len(hh), hh, out, _stream(stream))
    if not (allow_not_ready and st == NOT_READY):
        _check(st, "mdeos_restrict")
    return results_to_numpy(out)


def mdeos_eval_batch(ctx, specs, sched: Schedule, stream=None) -> np.ndarray:
    specs = _spec_array(specs)
    out = (Result * len(specs))()
    _check(lib().mdeos_eval_batch(ctx, len(specs), specs, C.byref(sched), out, _stream(stream)), "mdeos_eval_batch")
    return results_to_numpy(out)


def mdeos_eval_batch_noalloc(ctx, specs, sched: Schedule, stream=None) -> np.ndarray:
    specs = _spec_array(specs)
    out = (Result * len(specs))()
    _check(lib().mdeos_eval_batch_noalloc(ctx, len(specs), specs, C.byref(sched), out, _stream(stream)),
           "mdeos_eval_batch_noalloc")
    return results_to_numpy(out)


def mdeos_eval_plain(ctx, specs, sched: Schedule, stream=None) -> np.ndarray:
    specs = _spec_array(specs)
    out = (Result * len(specs))()
    _check(lib().mdeos_eval_plain(ctx, len(specs), specs, C.byref(sched), out, _stream(stream)), "mdeos_eval_plain")
    return results_to_numpy(out)


def mdeos_release(ctx, handles) -> None:
    hh = _handles(handles)
    _check(lib().mdeos_release(ctx, len(hh), hh), "mdeos_release")


def mdeos_last_advance_time(ctx) -> tuple[float, int]:
    ms = C.c_double()
    n = C.c_int()
    _check(lib().mdeos_last_advance_time(ctx, C.byref(ms), C.byref(n)), "mdeos_last_advance_time")
    return ms.value, n.value


def mdeos_state_export(ctx, handle: int, N: int):
    xyz = np.zeros((N, 3))
    v = np.zeros((N, 3))
    step = C.c_int()
    _check(lib().mdeos_state_export(ctx, int(handle), _dp(xyz), _dp(v), C.byref(step)), "mdeos_state_export")
    return xyz, v, step.value


def mdeos_debug_forces(ctx, spec: CellSpec, xyz: np.ndarray):
    xyz = np.ascontiguousarray(xyz, dtype=np.float64)
    F = np.zeros_like(xyz)
    U = C.c_double()
    W = C.c_double()
    _check(lib().mdeos_debug_forces(ctx, C.byref(spec), _dp(xyz), _dp(F), C.byref(U), C.byref(W)),
           "mdeos_debug_forces")
    return F, U.value, W.value


def mdeos_debug_trajectory(ctx, handle: int, n_steps: int, N: int, forces: bool = True):
    F = np.zeros((n_steps + 1, N, 3)) if forces else None
    K, U, W = (np.zeros(n_steps + 1) for _ in range(3))
    _check(lib().mdeos_debug_trajectory(ctx, int(handle), n_steps, _dp(F), _dp(K), _dp(U), _dp(W)),
           "mdeos_debug_trajectory")
    return F, K, U, W


def mdeos_serve_start(ctx, cold: Schedule, warm: Schedule, rc: float, dt: float, seed: int, chunk_steps: int,
                      max_slots: int = 0) -> None:
    cfg = ServeConfig(cold, warm, rc, dt, int(seed) & (2 ** 64 - 1), chunk_steps, max_slots)
    _check(lib().mdeos_serve_start(ctx, C.byref(cfg)), "mdeos_serve_start")


def mdeos_serve_submit(ctx, cell_id: int, rho: float, e: float, n_c: int, t_arrival: float) -> int:
    t = C.c_longlong()
    _check(lib().mdeos_serve_submit(ctx, int(cell_id), float(rho), float(e), int(n_c), float(t_arrival),
                                    C.byref(t)), "mdeos_serve_submit")
    return t.value


def mdeos_serve_poll(ctx, max_n: int = 4096):
    tickets = (C.c_longlong * max_n)()
    out = (Result * max_n)()
    td = np.zeros(max_n)
    n = C.c_int()
    _check(lib().mdeos_serve_poll(ctx, max_n, tickets, out, _dp(td), C.byref(n)), "mdeos_serve_poll")
    k = n.value
    return np.array(list(tickets)[:k], dtype=np.int64), results_to_numpy(out)[:k], td[:k].copy()


def mdeos_serve_now(ctx) -> float:
    return lib().mdeos_serve_now(ctx)


def mdeos_serve_stats_get(ctx) -> dict:
    s = ServeStats()
    _check(lib().mdeos_serve_stats_get(ctx, C.byref(s)), "mdeos_serve_stats_get")
    return {f[0]: getattr(s, f[0]) for f in ServeStats._fields_}


def mdeos_serve_stop(ctx, drain: bool = True) -> None:
    _check(lib().mdeos_serve_stop(ctx, 1 if drain else 0), "mdeos_serve_stop")
