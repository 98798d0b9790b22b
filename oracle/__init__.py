"""FP64 CPU oracle for the in-line MD equation of state (test infrastructure).

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package. The product path never does, and the
oracle imports nothing from the product package.

The arithmetic lives in ``mdeos_oracle.c`` (plain C, FP64, all pairs); this
module compiles it with gcc on demand and wraps it with ctypes. Each wrapped
routine names the passage of the paper it follows (arXiv 2508.06012,
Sec. III lifting/restricting operators, Sec. II.B microscopic model).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mdeos_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

NONFINITE = 1
BELOW_COLD = 2
DRIFT = 4


def build(force: bool = False) -> str:
    """Compile the oracle into ``oracle/liboracle.so`` with gcc."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"]
        )
        os.replace(tmp, _LIB)
    return _LIB


class _Cell(C.Structure):
    _fields_ = [
        ("rho", C.c_double),
        ("e", C.c_double),
        ("n_c", C.c_int),
        ("rc", C.c_double),
        ("dt", C.c_double),
        ("seed", C.c_uint64),
        ("cell_id", C.c_int64),
        ("query", C.c_int64),
        ("potential", C.c_int),
        ("eam_c", C.c_double),
    ]


class _Sched(C.Structure):
    _fields_ = [
        ("n_steps", C.c_int),
        ("n_avg", C.c_int),
        ("n_blocks", C.c_int),
        ("n_rescale", C.c_int),
        ("rescale_steps", C.c_int * 8),
        ("energy_every", C.c_int),
        ("drift_tol", C.c_double),
        ("eps", C.c_double),
        ("ensemble", C.c_int),
        ("gamma", C.c_double),
    ]


class _Result(C.Structure):
    _fields_ = [
        ("P", C.c_double),
        ("P_se", C.c_double),
        ("P_rms", C.c_double),
        ("T", C.c_double),
        ("T_se", C.c_double),
        ("Epot_mean", C.c_double),
        ("Ecold", C.c_double),
        ("drift", C.c_double),
        ("stress", C.c_double * 6),
        ("n_samples", C.c_int),
        ("status", C.c_int),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = C.CDLL(build())
        dp = C.POINTER(C.c_double)
        _lib.orc_philox4x64_10.argtypes = [C.POINTER(C.c_uint64)] * 3
        _lib.orc_gauss.argtypes = [C.c_uint64, C.c_int64, C.c_int64, C.c_int]
        _lib.orc_gauss.restype = C.c_double
        _lib.orc_noise3.argtypes = [C.c_uint64, C.c_int64, C.c_int64, C.c_int64, C.c_int64, dp]
        _lib.orc_lattice_param.argtypes = [C.c_double]
        _lib.orc_lattice_param.restype = C.c_double
        _lib.orc_box_length.argtypes = [C.c_int, C.c_double]
        _lib.orc_box_length.restype = C.c_double
        _lib.orc_lattice.argtypes = [C.c_int, C.c_double, dp]
        _lib.orc_forces.argtypes = [C.c_int, C.c_double, C.c_double, C.c_double, dp, dp, dp, dp]
        _lib.orc_forces_tensor.argtypes = [C.c_int, C.c_double, C.c_double, C.c_double, dp, dp, dp, dp, dp]
        _lib.orc_forces_celllist.argtypes = [C.c_int, C.c_double, C.c_double, C.c_double, dp, dp, dp, dp]
        _lib.orc_forces_celllist.restype = C.c_int
        _lib.orc_ecold.argtypes = [C.c_int, C.c_double, C.c_double, C.c_double]
        _lib.orc_ecold.restype = C.c_double
        _lib.orc_ecold_cell.argtypes = [C.POINTER(_Cell), C.c_double]
        _lib.orc_ecold_cell.restype = C.c_double
        _lib.orc_forces_eam.argtypes = [C.c_int, C.c_double, C.c_double, C.c_double, dp, dp, dp, dp, dp, dp]
        _lib.orc_lift.argtypes = [C.POINTER(_Cell), C.c_double, dp, dp]
        _lib.orc_lift.restype = C.c_double
        _lib.orc_block_stats.argtypes = [C.c_int, dp, C.c_int, dp, dp]
        _lib.orc_run.argtypes = [
            C.POINTER(_Cell), C.POINTER(_Sched), C.c_double, dp, dp,
            dp, dp, dp, dp, dp, C.c_int, dp, C.POINTER(_Result),
        ]
    return _lib


def _dp(a: np.ndarray | None):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(C.POINTER(C.c_double))


@dataclass
class Cell:
    """One continuum cell's EOS query: (rho*, e*) plus the box and run knobs."""

    rho: float
    e: float
    n_c: int
    rc: float = 2.5
    dt: float = 0.005
    seed: int = 20250806
    cell_id: int = 0
    query: int = 0  # index of this query of the cell (thermostat noise counter word 3)
    potential: int = 0  # 0: LJTS; 1: embedded-atom form of Eq. Etot (Sutton-Chen (9, 6) stand-in)
    eam_c: float = 39.432  # embedding strength c of the embedded-atom form

    @property
    def N(self) -> int:
        return 4 * self.n_c ** 3

    def _c(self) -> _Cell:
        return _Cell(self.rho, self.e, self.n_c, self.rc, self.dt, self.seed & (2**64 - 1), self.cell_id, self.query,
                     self.potential, self.eam_c)


@dataclass
class Schedule:
    n_steps: int
    n_avg: int
    n_blocks: int = 10
    rescale_steps: tuple = ()
    energy_every: int = 10
    drift_tol: float = 0.05
    eps: float = 1.0
    ensemble: int = 0  # 0: velocity Verlet + energy re-pins; 1: GJF Langevin + temperature updates
    gamma: float = 0.0  # Langevin friction (ensemble 1)

    def _c(self) -> _Sched:
        s = _Sched()
        s.n_steps, s.n_avg, s.n_blocks = self.n_steps, self.n_avg, self.n_blocks
        s.n_rescale = len(self.rescale_steps)
        for i, k in enumerate(self.rescale_steps):
            s.rescale_steps[i] = k
        s.energy_every, s.drift_tol, s.eps = self.energy_every, self.drift_tol, self.eps
        s.ensemble, s.gamma = self.ensemble, self.gamma
        return s


@dataclass
class Result:
    P: float
    P_se: float
    P_rms: float
    T: float
    T_se: float
    Epot_mean: float
    Ecold: float
    drift: float
    stress: tuple  # <sigma> (xx, yy, zz, xy, xz, yz), Eq. stress, over the sampled window steps
    n_samples: int
    status: int


@dataclass
class Run:
    """Everything orc_run returns: the final state, per-step series and the result."""

    x: np.ndarray
    v: np.ndarray
    K: np.ndarray
    U: np.ndarray
    W: np.ndarray
    P: np.ndarray
    T: np.ndarray
    F: np.ndarray
    result: Result
    Ecold_total: float = 0.0
    extra: dict = field(default_factory=dict)


def philox4x64_10(key, ctr) -> np.ndarray:
    k = (C.c_uint64 * 2)(*[int(v) & (2**64 - 1) for v in key])
    c = (C.c_uint64 * 4)(*[int(v) & (2**64 - 1) for v in ctr])
    o = (C.c_uint64 * 4)()
    lib().orc_philox4x64_10(k, c, o)
    return np.array(list(o), dtype=np.uint64)


def gauss(seed: int, cell_id: int, atom: int, comp: int) -> float:
    return lib().orc_gauss(seed & (2**64 - 1), cell_id, atom, comp)


def noise3(seed: int, cell_id: int, atom: int, step: int, query: int = 0) -> np.ndarray:
    """Thermostat noise of one atom at one step of a query: three standard normals."""
    z = np.zeros(3)
    lib().orc_noise3(seed & (2**64 - 1), cell_id, atom, step, query, z.ctypes.data_as(C.POINTER(C.c_double)))
    return z


def lattice_param(rho: float) -> float:
    return lib().orc_lattice_param(rho)


def box_length(n_c: int, rho: float) -> float:
    return lib().orc_box_length(n_c, rho)


def lattice(n_c: int, rho: float) -> np.ndarray:
    x = np.zeros((4 * n_c ** 3, 3))
    lib().orc_lattice(n_c, rho, _dp(x))
    return x


def forces(x: np.ndarray, L: float, rc: float, eps: float = 1.0):
    """All-pairs forces, potential energy and pair virial sum W = sum r.f."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    F = np.zeros_like(x)
    U = C.c_double()
    W = C.c_double()
    lib().orc_forces(x.shape[0], L, rc, eps, _dp(x), _dp(F), C.byref(U), C.byref(W))
    return F, U.value, W.value


def virial_tensor(x: np.ndarray, L: float, rc: float, eps: float = 1.0) -> np.ndarray:
    """Pair virial tensor sum over pairs of d_a f_b, as (xx, yy, zz, xy, xz, yz)."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    F = np.zeros_like(x)
    U = C.c_double()
    W = C.c_double()
    S = np.zeros(6)
    lib().orc_forces_tensor(x.shape[0], L, rc, eps, _dp(x), _dp(F), C.byref(U), C.byref(W), _dp(S))
    return S


def forces_celllist(x: np.ndarray, L: float, rc: float, eps: float = 1.0):
    x = np.ascontiguousarray(x, dtype=np.float64)
    F = np.zeros_like(x)
    U = C.c_double()
    W = C.c_double()
    rc_ = lib().orc_forces_celllist(x.shape[0], L, rc, eps, _dp(x), _dp(F), C.byref(U), C.byref(W))
    if rc_ != 0:
        raise ValueError("box too small for a 3-cell-per-side list")
    return F, U.value, W.value


def forces_eam(x: np.ndarray, L: float, rc: float, c: float):
    """Embedded-atom form (Eq. Etot): forces, E_pot, W, virial tensor and the
    host densities rhobar."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    F = np.zeros_like(x)
    U = C.c_double()
    W = C.c_double()
    S = np.zeros(6)
    rb = np.zeros(x.shape[0])
    lib().orc_forces_eam(x.shape[0], L, rc, c, _dp(x), _dp(F), C.byref(U), C.byref(W), _dp(S), _dp(rb))
    return F, U.value, W.value, S, rb


def cell_forces(cell: "Cell", x: np.ndarray, eps: float = 1.0):
    """Forces, E_pot and W of the cell's material at positions x."""
    L = box_length(cell.n_c, cell.rho)
    if cell.potential == 1:
        F, U, W, _, _ = forces_eam(x, L, cell.rc, cell.eam_c)
        return F, U, W
    return forces(x, L, cell.rc, eps)


def ecold_cell(cell: "Cell", eps: float = 1.0) -> float:
    """Total cold energy of the cell's static lattice, for its material."""
    c = cell._c()
    return lib().orc_ecold_cell(C.byref(c), eps)


def ecold(n_c: int, rho: float, rc: float, eps: float = 1.0) -> float:
    """Total cold energy of the static lattice (not per atom)."""
    return lib().orc_ecold(n_c, rho, rc, eps)


def lift(cell: Cell, eps: float = 1.0):
    """Lifting operator: returns (x, v, E_cold total)."""
    x = np.zeros((cell.N, 3))
    v = np.zeros((cell.N, 3))
    c = cell._c()
    Ec = lib().orc_lift(C.byref(c), eps, _dp(x), _dp(v))
    return x, v, Ec


def block_stats(series: np.ndarray, B: int):
    s = np.ascontiguousarray(series, dtype=np.float64)
    m = C.c_double()
    se = C.c_double()
    lib().orc_block_stats(s.shape[0], _dp(s), B, C.byref(m), C.byref(se))
    return m.value, se.value


def run(cell: Cell, sched: Schedule, x=None, v=None, Ecold_total=None, n_recF: int = 0) -> Run:
    """Lift (unless a state is given) and advance; returns per-step records and the result."""
    if x is None:
        x, v, Ecold_total = lift(cell, sched.eps)
    else:
        x = np.array(x, dtype=np.float64, order="C", copy=True)
        v = np.array(v, dtype=np.float64, order="C", copy=True)
        if Ecold_total is None:
            Ecold_total = ecold_cell(cell, sched.eps)
    n = sched.n_steps
    K, U, W, P, T = (np.zeros(n + 1) for _ in range(5))
    F = np.zeros((max(n_recF, 0), cell.N, 3))
    res = _Result()
    c = cell._c()
    s = sched._c()
    lib().orc_run(
        C.byref(c), C.byref(s), Ecold_total, _dp(x), _dp(v),
        _dp(K), _dp(U), _dp(W), _dp(P), _dp(T), n_recF, _dp(F) if n_recF > 0 else None, C.byref(res),
    )
    r = Result(*((tuple(getattr(res, f[0])) if f[0] == "stress" else getattr(res, f[0])) for f in _Result._fields_))
    return Run(x, v, K, U, W, P, T, F, r, Ecold_total)


def warm_start_state(x: np.ndarray, n_c: int, rho_old: float, rho_new: float) -> np.ndarray:
    """Warm start: dilate the resident configuration to the new density,
    x <- x L'/L (the lattice-parameter relation of Eq. numdens at rho')."""
    return np.asarray(x, dtype=np.float64) * (box_length(n_c, rho_new) / box_length(n_c, rho_old))
