"""The toy continuum driver (1-D Lagrangian hydro, Eqs. EulerMass / EulerMom /
EulerE with artificial viscosity) against the exact solution of the Sod
shock tube for a gamma-law gas, the Mie-Grueneisen EOS (Eq. MieGrun) with
zero reference curves and Gamma = gamma - 1."""
import numpy as np
import pytest

from paper_2508_06012_amd.hydro import Lagrangian1D, MieGruneisen

def sod_exact(x: np.ndarray, t: float, left=(1.0, 0.0, 1.0), right=(0.125, 0.0, 0.1), gamma: float = 1.4,
              x0: float = 0.5) -> tuple[np.ndarray, np.ndarray, np.ndarray]:
    """Exact solution of the Riemann problem of a gamma-law gas, states given
    as (rho, u, p): pressure of the star region by Newton iteration on the
    sum of the two wave functions (shock: Rankine-Hugoniot, rarefaction:
    isentropic), then sampling of the self-similar fan at x / t."""
    rl, ul, pl = left
    rr, ur, pr = right
    cl, cr = np.sqrt(gamma * pl / rl), np.sqrt(gamma * pr / rr)

    def f(p, rk, pk, ck):
        if p > pk:  # shock
            A, B = 2.0 / ((gamma + 1) * rk), (gamma - 1) / (gamma + 1) * pk
            s = np.sqrt(A / (p + B))
            return (p - pk) * s, s * (1 - 0.5 * (p - pk) / (p + B))
        r = p / pk  # rarefaction
        return 2 * ck / (gamma - 1) * (r ** ((gamma - 1) / (2 * gamma)) - 1), 1 / (rk * ck) * r ** (-(gamma + 1) / (2 * gamma))

    p = 0.5 * (pl + pr)
    for _ in range(100):
        fl, dl = f(p, rl, pl, cl)
        fr, dr = f(p, rr, pr, cr)
        dp = (fl + fr + ur - ul) / (dl + dr)
        p = max(p - dp, 1e-12)
        if abs(dp) < 1e-14 * p:
            break
    us = 0.5 * (ul + ur) + 0.5 * (f(p, rr, pr, cr)[0] - f(p, rl, pl, cl)[0])
    g1, g2 = (gamma - 1) / (gamma + 1), (gamma - 1) / (2 * gamma)
    rho, u, pp = np.empty_like(x), np.empty_like(x), np.empty_like(x)
    for i, xi in enumerate(x):
        s = (xi - x0) / t
        if s < us:  # left of the contact
            if p > pl:
                sl = ul - cl * np.sqrt((gamma + 1) / (2 * gamma) * p / pl + g2)
                val = (rl * (p / pl + g1) / (g1 * p / pl + 1), us, p) if s > sl else (rl, ul, pl)
            else:
                cs = cl * (p / pl) ** g2
                if s < ul - cl:
                    val = (rl, ul, pl)
                elif s > us - cs:
                    val = (rl * (p / pl) ** (1 / gamma), us, p)
                else:
                    uu = 2 / (gamma + 1) * (cl + (gamma - 1) / 2 * ul + s)
                    cc = 2 / (gamma + 1) * (cl + (gamma - 1) / 2 * (ul - s))
                    val = (rl * (cc / cl) ** (2 / (gamma - 1)), uu, pl * (cc / cl) ** (2 * gamma / (gamma - 1)))
        else:  # right of the contact
            if p > pr:
                sr = ur + cr * np.sqrt((gamma + 1) / (2 * gamma) * p / pr + g2)
                val = (rr * (p / pr + g1) / (g1 * p / pr + 1), us, p) if s < sr else (rr, ur, pr)
            else:
                cs = cr * (p / pr) ** g2
                if s > ur + cr:
                    val = (rr, ur, pr)
                elif s < us + cs:
                    val = (rr * (p / pr) ** (1 / gamma), us, p)
                else:
                    uu = 2 / (gamma + 1) * (-cr + (gamma - 1) / 2 * ur + s)
                    cc = 2 / (gamma + 1) * (cr - (gamma - 1) / 2 * (ur - s))
                    val = (rr * (cc / cr) ** (2 / (gamma - 1)), uu, pr * (cc / cr) ** (2 * gamma / (gamma - 1)))
        rho[i], u[i], pp[i] = val
    return rho, u, pp


def _run_sod(n):
    gamma = 1.4
    eos = MieGruneisen(gamma - 1)
    s = Lagrangian1D.tube(n, 1.0, (1.0, 1.0 / (0.4 * 1.0)), (0.125, 0.1 / (0.4 * 0.125)), eos)
    E0 = s.total_energy()
    while s.t < 0.2:
        s.step(min(s.stable_dt(), 0.2 - s.t))
    xc = 0.5 * (s.x[1:] + s.x[:-1])
    rho_ex, _, p_ex = sod_exact(xc, s.t)
    return s, np.mean(np.abs(s.rho - rho_ex)), np.mean(np.abs(s.p - p_ex)), abs(s.total_energy() - E0) / E0


def test_exact_riemann_solution_fixed_points():
    # the star state of the Sod problem (textbook values, 4-5 digits), either
    # side of the contact at x = 0.5 + u* t = 0.685
    rho, u, p = sod_exact(np.array([0.6, 0.8]), 0.2)
    assert p[0] == pytest.approx(0.30313, rel=1e-4) and u[0] == pytest.approx(0.92745, rel=1e-4)
    assert rho[0] == pytest.approx(0.42632, rel=1e-4) and rho[1] == pytest.approx(0.26557, rel=1e-4)


def test_sod_shock_tube_converges_to_the_exact_solution():
    _, e1, p1, de1 = _run_sod(200)
    s, e2, p2, de2 = _run_sod(800)
    assert e2 < 1e-3 and p2 < 1e-3, (e2, p2)
    assert e2 < 0.3 * e1 and p2 < 0.3 * p1, (e1, e2, p1, p2)  # first order at the discontinuities
    assert de1 < 1e-12 and de2 < 1e-12, (de1, de2)  # rigid walls do no work
    assert np.all(np.diff(s.x) > 0)


def test_piston_shock_matches_the_exact_hugoniot():
    """A piston driven at u_p into a gamma-law gas at rest: the shocked state
    is uniform with u = u_p, and the shock speed has the closed form
    U_s = (gamma + 1) u_p / 4 + sqrt(((gamma + 1) u_p / 4)^2 + c_1^2); mass and
    momentum jumps give rho_2 = rho_1 U_s / (U_s - u_p), p_2 = p_1 + rho_1 U_s u_p,
    and the energy jump is e_2 - e_1 = (p_1 + p_2) (1 / rho_1 - 1 / rho_2) / 2."""
    gamma, rho1, p1, up = 1.4, 1.0, 1.0, 1.0
    e1 = p1 / ((gamma - 1) * rho1)
    s = Lagrangian1D.tube(400, 1.0, (rho1, e1), (rho1, e1), MieGruneisen(gamma - 1), u_left=up)
    E0 = s.total_energy()
    c1 = np.sqrt(gamma * p1 / rho1)
    a = (gamma + 1) * up / 4
    Us = a + np.sqrt(a * a + c1 * c1)
    rho2, p2 = rho1 * Us / (Us - up), p1 + rho1 * Us * up
    t_end = 0.8 / Us
    while s.t < t_end:
        s.step(min(s.stable_dt(), t_end - s.t))
    xc = 0.5 * (s.x[1:] + s.x[:-1])
    behind = (xc > s.x[0] + 0.1) & (xc < Us * s.t - 0.05)
    assert behind.sum() > 100
    assert np.mean(s.rho[behind]) == pytest.approx(rho2, rel=1e-4)
    assert np.mean(s.p[behind]) == pytest.approx(p2, rel=1e-4)
    assert np.mean(s.e[behind]) - e1 == pytest.approx(0.5 * (p1 + p2) * (1 / rho1 - 1 / rho2), rel=1e-4)
    assert np.abs(s.u[1:-1][behind[1:]] / up - 1).max() < 1e-3
    # the shock front (half-way density) sits where the exact speed puts it
    k = np.argmax(s.rho < 0.5 * (rho1 + rho2))
    assert abs(xc[k] - Us * s.t) < 4.0 / 400
    # the piston's work is the only energy source
    assert abs(s.total_energy() - E0 - s.wall_work) < 1e-12 * s.wall_work


class _FakeLibrary:
    """Stands in for the device library on the CPU, to test the adapter's host
    logic. Its 'MD' EOS is P = p_c(rho) + rho (e_md - 0) with the cold curve
    E_c(rho) = 2 rho^4 - 4 rho^2 per atom, p_c = rho^2 dE_c/drho; e_md is the
    energy above the cold lattice, as the lifting operator takes it."""

    def __init__(self):
        self.boxes = {}
        self.lifts = self.warm_starts = 0

    @staticmethod
    def Ec(rho):
        return 2 * rho ** 4 - 4 * rho ** 2

    @staticmethod
    def pc(rho):
        return rho * rho * (8 * rho ** 3 - 8 * rho)

    def install(self, monkeypatch, m):
        for name in ("mdeos_create", "mdeos_destroy", "mdeos_lift", "mdeos_warm_start", "mdeos_advance",
                     "mdeos_restrict", "mdeos_release", "mdeos_eval_batch"):
            monkeypatch.setattr(m, name, getattr(self, name))

    def mdeos_create(self, *a, **k):
        return "ctx"

    def mdeos_destroy(self, ctx):
        pass

    def _result(self, rho, e):
        from paper_2508_06012_amd import mdeos as m
        r = np.zeros(rho.size, m.RESULT_DTYPE)
        r["P"], r["Ecold"] = self.pc(rho) + rho * e, self.Ec(rho)
        return r

    def mdeos_eval_batch(self, ctx, specs, sch):
        return self._result(np.array([s.rho for s in specs]), np.array([s.e for s in specs]))

    def mdeos_lift(self, ctx, specs, sch):
        self.lifts += 1
        h = np.arange(len(self.boxes), len(self.boxes) + len(specs))
        for k, s in zip(h, specs):
            self.boxes[int(k)] = (s.rho, s.e)
        return h

    def mdeos_warm_start(self, ctx, h, rho, e, sch):
        self.warm_starts += 1
        for k, r, x in zip(h, rho, e):
            assert int(k) in self.boxes
            self.boxes[int(k)] = (r, x)

    def mdeos_advance(self, ctx, h, n):
        pass

    def mdeos_restrict(self, ctx, h):
        st = np.array([self.boxes[int(k)] for k in h])
        return self._result(st[:, 0], st[:, 1])

    def mdeos_release(self, ctx, h):
        for k in h:
            del self.boxes[int(k)]


@pytest.mark.parametrize("mode", ["warm", "cold"])
def test_md_adapter_hands_the_lift_the_energy_above_the_cold_curve(monkeypatch, mode):
    """With the absolute energy zero, the adapter around the fake library is
    the Mie-Grueneisen EOS with reference curves (E_c, p_c) and Gamma = 1: the
    same shock tube run with either gives the same states to rounding."""
    from paper_2508_06012_amd import mdeos as m
    from paper_2508_06012_amd.hydro import MDEOS
    fake = _FakeLibrary()
    fake.install(monkeypatch, m)
    n = 64
    md = MDEOS(n, mode=mode)
    mg = MieGruneisen(1.0, p_ref=fake.pc, e_ref=fake.Ec)
    left, right = (0.9, fake.Ec(0.9) + 2.0), (0.6, fake.Ec(0.6) + 0.5)
    # no linear viscosity: it scales with each EOS's own sound-speed estimate
    a = Lagrangian1D.tube(n, 1.0, left, right, md, u_left=0.3, cl=0.0)
    b = Lagrangian1D.tube(n, 1.0, left, right, mg, u_left=0.3, cl=0.0)
    for _ in range(60):
        dt = 0.5 * min(a.stable_dt(), b.stable_dt())
        a.step(dt)
        b.step(dt)
    for f in ("x", "u", "e", "p"):
        assert np.allclose(getattr(a, f), getattr(b, f), rtol=1e-12, atol=1e-12), f
    assert md.floored == 0 and md.failed == 0 and md.calls == 121 * n
    assert (fake.lifts, fake.warm_starts) == ((1, 120) if mode == "warm" else (121, 0))
    assert len(fake.boxes) == n  # cold mode releases the previous boxes
    # the stiffness estimate: dp_c/drho by central differences of the cold curve
    rho = a.rho
    assert np.allclose(md.c2_cold, np.maximum(2 * rho * (8 * rho ** 3 - 8 * rho) + rho * rho * (24 * rho ** 2 - 8), 0),
                       rtol=1e-3, atol=1e-2)
    md.close()


def test_md_adapter_floors_energies_below_the_cold_lattice(monkeypatch):
    from paper_2508_06012_amd import mdeos as m
    from paper_2508_06012_amd.hydro import MDEOS
    fake = _FakeLibrary()
    fake.install(monkeypatch, m)
    md = MDEOS(3, e_floor=1e-3)
    rho = np.array([0.8, 0.8, 0.8])
    p = md(rho, fake.Ec(rho) + np.array([-0.1, 0.0, 0.2]))
    assert md.floored == 2
    assert np.allclose(p, fake.pc(rho) + rho * np.array([1e-3, 1e-3, 0.2]))
    with pytest.raises(ValueError):
        MDEOS(3, mode="lazy")
