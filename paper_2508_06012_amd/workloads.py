"""Seeded synthetic workloads (input generators only).

This module is shared by the HIP path's tests and benchmark and by the oracle
tests. It produces the per-cell inputs of an EOS query (density, target
energy, box size, cutoff, time step, RNG key) and the run schedule; it holds
none of the method's arithmetic and imports nothing from the rest of the
package.

The paper's own workloads (copper EAM, deuterium ML potential, LEOS tables)
are not available; these stand-ins follow the shapes the paper describes:
independent boxes of O(10^2..10^3) atoms, one per continuum quadrature point
(Sec. III, Sec. VI, App. C), over density/temperature ranges like the EOS
sweep of App. B.

Temperatures are turned into the method's input e* (energy per atom above the
cold lattice) by inverting the lifting operator's first guess T = 2E/N_DOF
with E = N e* and N_DOF = 3N - 3, so the initial Maxwell-Boltzmann
temperature equals the requested T*.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

DEFAULT_SEED = 20250806
FCC_SIZES = (108, 256, 500, 864, 1372, 2048, 4000)  # 4 n_c^3 for n_c = 3..8, 10


def n_c_of(N: int) -> int:
    n = round((N / 4) ** (1 / 3))
    assert 4 * n ** 3 == N, N
    return n


def e_from_T(T, N):
    """Input recipe: e* = N_DOF T* / (2N) with N_DOF = 3N - 3."""
    return 1.5 * np.asarray(T, dtype=float) * (1.0 - 1.0 / np.asarray(N, dtype=float))


@dataclass
class Schedule:
    n_steps: int
    n_avg: int
    rescale_steps: tuple
    n_blocks: int = 10
    energy_every: int = 10
    drift_tol: float = 0.05


@dataclass
class Workload:
    name: str
    rho: np.ndarray
    e: np.ndarray
    n_c: np.ndarray
    rc: np.ndarray
    dt: np.ndarray
    seed: int
    cell_id: np.ndarray
    sched: Schedule
    T: np.ndarray = None
    meta: dict = field(default_factory=dict)
    potential: int = 0  # 0: LJTS; 1: the embedded-atom form (Sutton-Chen (9, 6) stand-in)

    @property
    def n(self) -> int:
        return int(self.rho.shape[0])

    @property
    def N(self) -> np.ndarray:
        return 4 * self.n_c.astype(np.int64) ** 3

    def atom_steps(self) -> int:
        return int(self.N.sum()) * self.sched.n_steps

    def subset(self, idx) -> "Workload":
        idx = np.asarray(idx)
        return Workload(
            self.name + "[sub]", self.rho[idx], self.e[idx], self.n_c[idx], self.rc[idx], self.dt[idx],
            self.seed, self.cell_id[idx], self.sched, None if self.T is None else self.T[idx], dict(self.meta),
            self.potential,
        )


def smooth_field(n: int, rng: np.random.Generator, nmodes: int = 4):
    """Min-max normalised sum of 4 random plane waves on an n x n periodic mesh."""
    i, j = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    f = np.zeros((n, n))
    modes = []
    while len(modes) < nmodes:
        p, q = (int(v) for v in rng.integers(-3, 4, size=2))
        if p == 0 and q == 0:
            continue
        a = rng.uniform(0.5, 1.0)
        ph = rng.uniform(0.0, 2 * math.pi)
        modes.append((p, q, a, ph))
    for p, q, a, ph in modes:
        f += a * np.sin(2 * math.pi * (p * i + q * j) / n + ph)
    f = (f - f.min()) / (f.max() - f.min())
    return f, modes


def advected_field(n: int, modes, t: float, speed: float = 0.5):
    """The plane-wave field of ``smooth_field`` advected along i by speed*t."""
    i, j = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    f = np.zeros((n, n))
    for p, q, a, ph in modes:
        f += a * np.sin(2 * math.pi * (p * (i - speed * t) + q * j) / n + ph)
    return f


def cfg1(seed: int = DEFAULT_SEED) -> Workload:
    """Plain method, one cell: 256 atoms, rho* = 0.8442, T* = 0.722, rc = 2.5,
    dt = 0.005, 1000 steps, re-pins at 250 and 500, average over the last 500."""
    N = 256
    return Workload(
        "cfg1-single-256", np.array([0.8442]), e_from_T([0.722], [N]), np.array([4]), np.array([2.5]),
        np.array([0.005]), seed, np.array([0]), Schedule(1000, 500, (250, 500)), np.array([0.722]),
    )


def cfg2(seed: int = DEFAULT_SEED, mesh: int = 64) -> Workload:
    """Uniform batch: 64 x 64 mesh of 500-atom boxes, rho* in [0.3, 1.1] from a
    smooth field, T* ~ U[0.8, 3.0], rc = 2.5, dt = 0.004, 2000 steps, re-pins at
    500 and 1000, average over the last 1000."""
    rng = np.random.default_rng(seed)
    f, modes = smooth_field(mesh, rng)
    rho = 0.3 + 0.8 * f.ravel()
    n = rho.size
    T = rng.uniform(0.8, 3.0, size=n)
    N = np.full(n, 500)
    return Workload(
        "cfg2-uniform-4096x500" if mesh == 64 else f"cfg2-uniform-{n}x500", rho, e_from_T(T, N),
        np.full(n, 5), np.full(n, 2.5), np.full(n, 0.004), seed, np.arange(n),
        Schedule(2000, 1000, (500, 1000)), T, {"modes": modes},
    )


def draw_sizes_log_uniform(rng: np.random.Generator, n: int) -> np.ndarray:
    """u ~ U[ln 108, ln 4000], then the member of FCC_SIZES nearest in ln N."""
    u = rng.uniform(math.log(FCC_SIZES[0]), math.log(FCC_SIZES[-1]), size=n)
    lg = np.log(np.array(FCC_SIZES, dtype=float))
    idx = np.abs(u[:, None] - lg[None, :]).argmin(axis=1)
    return np.array(FCC_SIZES)[idx]


def cfg3(seed: int = DEFAULT_SEED, n: int = 10_000) -> Workload:
    """Uneven sizes: N log-uniform over {108..4000}, rho* ~ U[0.2, 1.2],
    T* ~ U[0.7, 5.0], rc in {2.5, 3.0}, dt = 0.004, 1500 steps, re-pins at 375
    and 750, average over the last 750."""
    rng = np.random.default_rng(seed + 3)
    N = draw_sizes_log_uniform(rng, n)
    rho = rng.uniform(0.2, 1.2, size=n)
    T = rng.uniform(0.7, 5.0, size=n)
    rc = np.where(rng.uniform(size=n) < 0.5, 2.5, 3.0)
    n_c = np.array([n_c_of(int(v)) for v in N])
    return Workload(
        f"cfg3-uneven-{n}", rho, e_from_T(T, N), n_c, rc, np.full(n, 0.004), seed, np.arange(n),
        Schedule(1500, 750, (375, 750)), T,
    )


def cfg5(seed: int = DEFAULT_SEED, n: int = 65_536) -> Workload:
    """Large batch: 864-atom boxes, rho* ~ U[0.5, 1.2], T* ~ U[1, 10], rc = 4.0,
    dt = 0.002, 1000 steps, re-pins at 250 and 500, average over the last 500."""
    rng = np.random.default_rng(seed + 5)
    rho = rng.uniform(0.5, 1.2, size=n)
    T = rng.uniform(1.0, 10.0, size=n)
    N = np.full(n, 864)
    return Workload(
        f"cfg5-large-{n}x864", rho, e_from_T(T, N), np.full(n, 6), np.full(n, 4.0), np.full(n, 0.002), seed,
        np.arange(n), Schedule(1000, 500, (250, 500)), T,
    )


def eam_cu(seed: int = DEFAULT_SEED, mesh: int = 64) -> Workload:
    """Many-body batch: the embedded-atom form with the Sutton-Chen (9, 6)
    functions standing in for the paper's copper potential (App. A). A 64 x 64
    mesh of 500-atom boxes, rho ~ [4.0, 6.0] atoms per a^3 from a smooth field
    (the fitted lattice up to 1.5x compression, about 150 GPa in copper units),
    T ~ U[7, 35] (about 1000-5000 K), rc = 1.5 a, dt = 0.001 (2.6 fs), 2000
    steps, re-pins at 500 and 1000, average over the last 1000."""
    rng = np.random.default_rng(seed + 7)
    f, modes = smooth_field(mesh, rng)
    rho = 4.0 + 2.0 * f.ravel()
    n = rho.size
    T = rng.uniform(7.0, 35.0, size=n)
    N = np.full(n, 500)
    return Workload(
        f"eam-cu-{n}x500", rho, e_from_T(T, N), np.full(n, 5), np.full(n, 1.5), np.full(n, 0.001), seed,
        np.arange(n), Schedule(2000, 1000, (500, 1000)), T, {"modes": modes}, potential=1,
    )


def stratified_sample(w: Workload, n_rho: int = 8, n_T: int = 8) -> np.ndarray:
    """Indices of a fixed stratified subsample: the lowest-index cell in each
    of n_rho x n_T equal bins over the workload's density and temperature
    ranges (bins with no cell are skipped)."""
    lo_r, hi_r = w.rho.min(), w.rho.max()
    lo_t, hi_t = w.T.min(), w.T.max()
    br = np.minimum(((w.rho - lo_r) / (hi_r - lo_r) * n_rho).astype(int), n_rho - 1)
    bt = np.minimum(((w.T - lo_t) / (hi_t - lo_t) * n_T).astype(int), n_T - 1)
    out = []
    for i in range(n_rho):
        for j in range(n_T):
            idx = np.nonzero((br == i) & (bt == j))[0]
            if idx.size:
                out.append(int(idx[0]))
    return np.array(out, dtype=int)


@dataclass
class Query:
    t_arrival: float
    cell: int
    step: int
    rho: float
    e: float
    n_c: int


def cfg4_queries(rate: float, seed: int = DEFAULT_SEED, mesh: int = 128, n_t: int = 100,
                 t_max: int | None = None) -> tuple[list[Query], dict]:
    """Serving stream: every cell of a mesh x mesh grid emits one query per
    continuum step t (shuffled within t); arrivals form a Poisson process of the
    given rate. Density and temperature are advected plane-wave fields mapped to
    [0.3, 1.1] and [0.8, 3.0]; each cell keeps one size from {256, 500, 864}."""
    rng = np.random.default_rng(seed + 4)
    ncell = mesh * mesh
    sizes = rng.choice(np.array([256, 500, 864]), size=ncell)
    _, modes_r = smooth_field(mesh, rng)
    _, modes_t = smooth_field(mesh, rng)
    steps = n_t if t_max is None else min(n_t, t_max)
    # normalisation bounds of the advected fields from the t = 0 snapshot
    f0r = advected_field(mesh, modes_r, 0.0)
    f0t = advected_field(mesh, modes_t, 0.0)
    rlo, rhi = f0r.min(), f0r.max()
    tlo, thi = f0t.min(), f0t.max()
    out: list[Query] = []
    t_now = 0.0
    for t in range(steps):
        fr = np.clip((advected_field(mesh, modes_r, t) - rlo) / (rhi - rlo), 0.0, 1.0).ravel()
        ft = np.clip((advected_field(mesh, modes_t, t) - tlo) / (thi - tlo), 0.0, 1.0).ravel()
        rho = 0.3 + 0.8 * fr
        T = 0.8 + 2.2 * ft
        e = e_from_T(T, sizes)
        order = rng.permutation(ncell)
        gaps = rng.exponential(1.0 / rate, size=ncell)
        for k, c in enumerate(order):
            t_now += gaps[k]
            out.append(Query(t_now, int(c), t, float(rho[c]), float(e[c]), n_c_of(int(sizes[c]))))
    meta = {
        "cold": Schedule(2000, 1000, (500, 1000)),
        "warm": Schedule(500, 250, (0, 125)),
        "rc": 2.5,
        "dt": 0.004,
        "sizes": sizes,
    }
    return out, meta
