"""A toy continuum driver: 1-D planar Lagrangian hydrodynamics whose equation
of state is either analytic (Mie-Grueneisen, Eq. MieGrun) or the in-line MD
evaluation of this library, called for every zone at every step (Sec. III,
Sec. IV) through the C ABI.

Euler equations in Lagrangian form (Eqs. EulerMass, EulerMom, EulerE) on a
staggered mesh: node positions x and velocities u (both at whole steps), zone
masses m, specific volume v = (x_{j+1} - x_j) / m, specific internal energy e,
pressure from the EOS (Eq. EOS). Shocks are captured with a quadratic plus
linear artificial viscosity active in compression (the Wilkins form the paper
cites, Sec. II.A). A step is a predictor-corrector with velocity averaging,
an explicit energy-conserving time step like the paper's continuum solver
uses (Sec. II.A), with nodal forces
F_i = (p + q)_{i-1} - (p + q)_i and, for a stage of length h from state n,
    u' = u^n + h F(p + q) / M,   ubar = (u^n + u') / 2,   x' = x^n + h ubar
    e' = e^n - h (p + q) (ubar_{j+1} - ubar_j) / m_j,     p' = EOS(1 / v', e')
The predictor takes h = dt / 2 with (p + q)^n; the corrector takes h = dt from
state n with the predictor's (p + q). Since the same forces move the nodes
and do work on the zones with the same averaged velocities, the kinetic plus
internal energy changes only by the work of the walls (to rounding). The
right wall is rigid; the left may move at a prescribed speed (a piston), and
the work it does is kept in wall_work. The EOS is called twice per step.

Units: those of the EOS. With the MD EOS they are the reduced units of the
context's potential (LJTS: sigma and eps; embedded-atom form: the lattice
parameter a and eps) with unit atomic mass, so the mass density is the number
density. The hydro's e has a fixed zero; by default the MD adapter hands the
lift the energy above the cold lattice at each zone's own density (the
lifting operator's energy zero, Sec. III).
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field
from typing import Callable

import numpy as np


class MieGruneisen:
    """P = P_ref(rho) + Gamma rho (e - e_ref(rho)) (Eq. MieGrun per unit mass).
    With zero reference curves this is the gamma-law gas, Gamma = gamma - 1."""

    def __init__(self, gamma_g: float, p_ref: Callable | None = None, e_ref: Callable | None = None):
        self.Gamma = gamma_g
        self.p_ref = p_ref or (lambda rho: np.zeros_like(rho))
        self.e_ref = e_ref or (lambda rho: np.zeros_like(rho))
        self.calls = 0
        self.seconds = 0.0

    def __call__(self, rho: np.ndarray, e: np.ndarray) -> np.ndarray:
        t0 = time.perf_counter()
        p = self.p_ref(rho) + self.Gamma * rho * (e - self.e_ref(rho))
        self.calls += rho.size
        self.seconds += time.perf_counter() - t0
        return p

    def sound_speed(self, rho: np.ndarray, e: np.ndarray, p: np.ndarray) -> np.ndarray:
        # gamma-law estimate (exact for zero reference curves)
        return np.sqrt(np.maximum((1.0 + self.Gamma) * p / rho, 1e-12))


class MDEOS:
    """The in-line MD equation of state, one box per zone (Sec. III, Sec. IV).

    mode "warm": the first call lifts every zone cold; later calls warm-start
    each resident box at the zone's new (rho, e), advance and restrict.
    mode "cold": every call lifts, advances and restricts an independent box
    per zone, as the paper does at every quadrature point and step.

    Energy zero. The lifting operator takes e above the cold lattice at the
    zone's density (Eq. Tcontribution), while the continuum energy equation
    needs a fixed zero. With energy_zero "absolute" (default) the hydro
    carries e_abs = e + E_cold(rho) / N and every call first asks the device
    for E_cold(rho) / N (a lattice pass plus two steps per zone, the same pass
    the lift makes) and hands e_abs - E_cold / N to the lift. With "cold" the
    hydro's e is passed through unchanged.

    Values at or below the cold lattice are raised to e_floor and counted in
    `floored`; cells whose status reports a non-finite state or a list
    overflow are counted in `failed`."""

    PROBE = 0.01  # relative density step of the cold-curve stiffness estimate

    def __init__(self, n_zones: int, n_c: int = 4, rc: float = 2.5, dt: float = 0.004, seed: int = 1,
                 cold=(1000, 500, (250, 500)), warm=(300, 150, (0, 75)), mode: str = "warm",
                 energy_zero: str = "absolute", e_floor: float = 1e-3, ctx=None):
        from . import mdeos as m
        if mode not in ("warm", "cold") or energy_zero not in ("absolute", "cold"):
            raise ValueError("mode is warm or cold, energy_zero is absolute or cold")
        self.m = m
        self.ctx = ctx if ctx is not None else m.mdeos_create()
        self.own_ctx = ctx is None
        self.n, self.n_c, self.rc, self.dt, self.seed = n_zones, n_c, rc, dt, seed
        self.mode, self.energy_zero = mode, energy_zero
        self.cold = m.make_schedule(cold[0], cold[1], cold[2])
        self.warm = m.make_schedule(warm[0], warm[1], warm[2])
        self.probe_schedule = m.make_schedule(2, 2, (), 2)
        self.e_floor = e_floor
        self.h = None
        self.step = 0
        self.calls = 0
        self.seconds = 0.0
        self.floored = 0
        self.failed = 0
        self.last = None
        self.c2_cold = np.zeros(n_zones)
        self.p_cold = np.zeros(n_zones)

    def cold_curve(self, rho: np.ndarray) -> np.ndarray:
        """E_cold / N of the static lattice at each density, from the device."""
        m = self.m
        rho = np.asarray(rho, dtype=float)
        specs = m.make_specs(rho, 1.0, self.n_c, self.rc, self.dt, self.seed, np.arange(rho.size))
        return m.mdeos_eval_batch(self.ctx, specs, self.probe_schedule)["Ecold"].copy()

    def _cold_terms(self, rho: np.ndarray) -> np.ndarray:
        # E_c at rho (1 - d), rho, rho (1 + d) in one batch; the cold pressure
        # is p_c = rho^2 dE_c/drho and its stiffness dp_c/drho bounds the
        # sound speed of the dense states from below
        d = self.PROBE
        E = self.cold_curve(np.concatenate([rho * (1 - d), rho, rho * (1 + d)])).reshape(3, -1)
        h = rho * d
        dE = (E[2] - E[0]) / (2 * h)
        d2E = (E[2] - 2 * E[1] + E[0]) / (h * h)
        self.p_cold = rho * rho * dE
        self.c2_cold = np.maximum(2 * rho * dE + rho * rho * d2E, 0.0)
        return E[1]

    def __call__(self, rho: np.ndarray, e: np.ndarray) -> np.ndarray:
        m = self.m
        t0 = time.perf_counter()
        rho = np.asarray(rho, dtype=float)
        Ec = self._cold_terms(rho)
        e_md = e - Ec if self.energy_zero == "absolute" else np.asarray(e, dtype=float)
        self.floored += int((e_md < self.e_floor).sum())
        e_md = np.maximum(e_md, self.e_floor)
        if self.mode == "cold" or self.h is None:
            if self.h is not None:
                m.mdeos_release(self.ctx, self.h)
            # a new seed per step keeps independent lifts independent
            specs = m.make_specs(rho, e_md, self.n_c, self.rc, self.dt, self.seed + self.step, np.arange(self.n))
            self.h = m.mdeos_lift(self.ctx, specs, self.cold)
        else:
            m.mdeos_warm_start(self.ctx, self.h, rho, e_md, self.warm)
        m.mdeos_advance(self.ctx, self.h, 10 ** 9)
        res = m.mdeos_restrict(self.ctx, self.h)
        self.failed += int(((res["status"] & (m.CELL_NONFINITE | m.CELL_OVERFLOW)) != 0).sum())
        self.last = res
        self.e_md = e_md
        self.step += 1
        self.calls += self.n
        self.seconds += time.perf_counter() - t0
        return res["P"].copy()

    def sound_speed(self, rho: np.ndarray, e: np.ndarray, p: np.ndarray) -> np.ndarray:
        # stability estimate for the CFL step, not a thermodynamic derivative:
        # the cold-curve stiffness plus a thermal part with Gruneisen gamma 1
        return np.sqrt(self.c2_cold + 2.0 * np.maximum(p - self.p_cold, 0.0) / rho + 1e-12)

    def close(self):
        if self.h is not None:
            self.m.mdeos_release(self.ctx, self.h)
            self.h = None
        if self.own_ctx:
            self.m.mdeos_destroy(self.ctx)


@dataclass
class Lagrangian1D:
    """State of the 1-D Lagrangian mesh: a rigid wall on the right, a wall
    moving at u_left (a piston, or at rest) on the left."""

    x: np.ndarray          # node positions (n + 1)
    u: np.ndarray          # node velocities (n + 1)
    m: np.ndarray          # zone masses (n)
    e: np.ndarray          # zone specific internal energies (n)
    eos: Callable
    cq: float = 1.0        # quadratic artificial-viscosity coefficient
    cl: float = 0.2        # linear artificial-viscosity coefficient
    cfl: float = 0.3
    t: float = 0.0
    p: np.ndarray = field(default=None)
    q: np.ndarray = field(default=None)
    u_left: float = 0.0    # velocity of the left wall (a piston when > 0)
    wall_work: float = 0.0 # work done on the fluid by the left wall

    @classmethod
    def tube(cls, n: int, length: float, left: tuple, right: tuple, eos, split: float = 0.5, **kw):
        """Shock tube: zones left of split at (rho, e) = left, the rest at right."""
        x = np.linspace(0.0, length, n + 1)
        xc = 0.5 * (x[1:] + x[:-1])
        rho = np.where(xc < split * length, left[0], right[0]).astype(float)
        e = np.where(xc < split * length, left[1], right[1]).astype(float)
        s = cls(x=x, u=np.zeros(n + 1), m=rho * np.diff(x), e=e, eos=eos, **kw)
        s.u[0] = s.u_left
        s.p = eos(rho, e)
        s.q = np.zeros(n)
        return s

    @property
    def rho(self) -> np.ndarray:
        return self.m / np.diff(self.x)

    def node_mass(self) -> np.ndarray:
        M = np.zeros(self.x.size)
        M[:-1] += 0.5 * self.m
        M[1:] += 0.5 * self.m
        return M

    def total_energy(self) -> float:
        return float(np.sum(self.m * self.e) + 0.5 * np.sum(self.node_mass() * self.u ** 2))

    def stable_dt(self) -> float:
        rho = self.rho
        c = self.eos.sound_speed(rho, self.e, self.p)
        dx = np.diff(self.x)
        du = np.abs(np.diff(self.u))
        return float(self.cfl * np.min(dx / (c + 2.0 * self.cq * du + 1e-30)))

    def _viscosity(self, x: np.ndarray, u: np.ndarray, p: np.ndarray, e: np.ndarray) -> np.ndarray:
        rho = self.m / np.diff(x)
        du = np.diff(u)
        c = self.eos.sound_speed(rho, e, p)
        return np.where(du < 0, rho * (self.cq * du ** 2 + self.cl * c * np.abs(du)), 0.0)

    def _stage(self, h: float, pq: np.ndarray):
        F = np.zeros(self.x.size)
        F[1:-1] = pq[:-1] - pq[1:]
        u1 = self.u + h * F / self.node_mass()
        u1[0], u1[-1] = self.u_left, 0.0          # the walls move as prescribed
        ubar = 0.5 * (self.u + u1)
        x1 = self.x + h * ubar
        if np.any(np.diff(x1) <= 0):
            raise FloatingPointError("tangled mesh: reduce the time step")
        e1 = self.e - h * pq * np.diff(ubar) / self.m
        return x1, u1, e1

    def step(self, dt: float | None = None) -> float:
        dt = self.stable_dt() if dt is None else dt
        pq0 = self.p + self._viscosity(self.x, self.u, self.p, self.e)
        xh, uh, eh = self._stage(0.5 * dt, pq0)
        ph = self.eos(self.m / np.diff(xh), eh)
        qh = self._viscosity(xh, uh, ph, eh)
        x1, u1, e1 = self._stage(dt, ph + qh)
        self.wall_work += dt * self.u_left * (ph[0] + qh[0])
        self.x, self.u, self.e, self.q = x1, u1, e1, qh
        self.p = self.eos(self.rho, self.e)
        self.t += dt
        return dt
