"""The toy continuum driver on the device EOS: a piston driven into a
Lennard-Jones fluid, and into the embedded-atom stand-in for copper, every
zone's pressure from its own MD box at every stage of every step (the EOS is
called at every point and step, Sec. IV).

Checks, each fixed by the continuum equations rather than by the oracle:
  - no cell fails and no zone's energy falls to the cold lattice;
  - kinetic plus internal energy grows by exactly the piston's work (the
    scheme conserves energy for any pressure, noisy or not);
  - the shocked plateau and the shock speed measured from the front's path
    satisfy the Rankine-Hugoniot jumps: mass rho2 (Us - up) = rho1 Us,
    momentum p2 - p1 = rho1 Us up, energy e2 - e1 = (p1 + p2)(v1 - v2) / 2;
  - the plateau's pressure, produced by boxes warm-started at every call,
    agrees with independent fresh lifts at the plateau's (rho, e).
It also prints the cost per zone call of the MD EOS (warm-started, and with
an independent lift per call as the paper does) next to the analytic
Mie-Grueneisen comparator, the comparison of the paper's runtime figure.
"""
import time

import numpy as np
import pytest

import oracle
from _stats import check_stats, oracle_many
from paper_2508_06012_amd import mdeos as m
from paper_2508_06012_amd.hydro import MDEOS, Lagrangian1D, MieGruneisen

pytestmark = pytest.mark.gpu

N_ZONES, LENGTH = 48, 48.0
RHO1, E_MD1, UP = 0.7, 2.5, 1.0


def _front(x, rho, level):
    """Position of the first crossing of `level` from the right (the shock)."""
    xc = 0.5 * (x[1:] + x[:-1])
    k = len(rho) - 1
    while k > 0 and rho[k] < level:
        k -= 1
    if k == len(rho) - 1:
        return xc[-1]
    f = (rho[k] - level) / (rho[k] - rho[k + 1])
    return xc[k] + f * (xc[k + 1] - xc[k])


def _run_piston(eos, rho1, e1, up, label):
    """Drives the piston until the front (5 % density rise) passes 3/4 of the
    tube; returns the final state, the (t, x, rho) history, p1, E0 and the
    wall time."""
    s = Lagrangian1D.tube(N_ZONES, LENGTH, (rho1, e1), (rho1, e1), eos, u_left=up)
    p1 = float(np.mean(s.p))
    E0 = s.total_energy()
    hist = []
    t0 = time.perf_counter()
    while True:
        s.step()
        hist.append((s.t, s.x.copy(), s.rho.copy()))
        xf = _front(s.x, s.rho, rho1 * 1.05)
        if len(hist) % 25 == 0:
            print(f"  {label} step {len(hist)} t {s.t:.4f} front {xf:.2f}", flush=True)
        if xf > 0.75 * LENGTH or len(hist) >= 600:
            break
    return s, hist, p1, E0, time.perf_counter() - t0


def _check_piston(eos, s, hist, rho1, e1, p1, E0, up, ctx, fresh_kw, tol=(0.03, 0.05, 0.05)):
    """Energy = piston work; Rankine-Hugoniot jumps with the fitted shock
    speed; plateau pressure = fresh lifts at the plateau state."""
    assert eos.failed == 0 and eos.floored == 0
    assert not (eos.last["status"] & m.CELL_COLD_RELIFT).any()
    dE = s.total_energy() - E0
    print(f"energy: gained {dE:.6f}, piston work {s.wall_work:.6f}", flush=True)
    assert abs(dE - s.wall_work) < 1e-9 * abs(s.wall_work)
    xc = 0.5 * (s.x[1:] + s.x[:-1])
    xf = _front(s.x, s.rho, rho1 * 1.05)
    plat = (xc > s.x[0] + 4.0) & (xc < xf - 4.0)
    assert plat.sum() >= 10
    rho2, p2, e2 = s.rho[plat].mean(), s.p[plat].mean(), s.e[plat].mean()
    u2 = 0.5 * (s.u[1:] + s.u[:-1])[plat].mean()
    level = 0.5 * (rho1 + rho2)
    ts = np.array([h[0] for h in hist])
    xs = np.array([_front(h[1], h[2], level) for h in hist])
    late = ts > 0.5 * ts[-1]
    Us = np.polyfit(ts[late], xs[late], 1)[0]
    mass = rho2 * (Us - up) / (rho1 * Us) - 1
    mom = (p2 - p1) / (rho1 * Us * up) - 1
    ene = (e2 - e1) / (0.5 * (p1 + p2) * (1 / rho1 - 1 / rho2)) - 1
    print(f"plateau: rho2 {rho2:.4f} p2 {p2:.4f} (p1 {p1:.4f}) e2-e1 {e2 - e1:.4f} u2 {u2:.4f}; "
          f"Us {Us:.4f}; RH residuals mass {mass:+.4f} momentum {mom:+.4f} energy {ene:+.4f}", flush=True)
    assert abs(u2 / up - 1) < 0.02
    assert abs(mass) < tol[0] and abs(mom) < tol[1] and abs(ene) < tol[2]
    ec2 = eos.cold_curve([rho2])[0]
    R = 16
    specs = m.make_specs(np.full(R, rho2), np.full(R, e2 - ec2), fresh_kw["n_c"], fresh_kw["rc"], fresh_kw["dt"],
                         np.arange(100, 100 + R), 0)
    fresh = m.mdeos_eval_batch(ctx, specs, eos.cold)
    pf, pf_se = fresh["P"].mean(), fresh["P"].std(ddof=1) / np.sqrt(R)
    p_sd = s.p[plat].std(ddof=1)
    bar = 3 * np.hypot(pf_se, p_sd / np.sqrt(plat.sum())) + 0.02 * abs(p2)
    print(f"fresh lifts at the plateau state: P {pf:.4f} +- {pf_se:.4f}; plateau {p2:.4f} (zone sd {p_sd:.4f}); "
          f"bar {bar:.4f}", flush=True)
    assert abs(pf - p2) < bar


@pytest.fixture(scope="module")
def ctx():
    c = m.mdeos_create()
    yield c
    m.mdeos_destroy(c)


def test_driver_device_calls_match_the_oracle(ctx):
    """The cold curve E_cold/N per zone (the energy-zero conversion of every
    call, C25) against the oracle's static-lattice energy to the energy bar;
    the first call's fresh lifts (lift, 1000-step schedule with re-pins,
    restriction) against oracle runs of the same specs (same Philox key per
    zone, same energy above cold) by the statistical bar."""
    nz = 8
    eos = MDEOS(nz, n_c=4, rc=2.5, dt=0.004, seed=3, ctx=ctx)
    rho = np.linspace(0.55, 1.05, nz)
    print(f"driver vs oracle: cold curve and first lifts of {nz} zones", flush=True)
    ec = eos.cold_curve(rho)
    want = np.array([oracle.ecold(4, float(r), 2.5) / 256 for r in rho])
    assert np.all(np.abs(ec - want) <= 1e-6 * np.abs(want)), (ec, want)
    p = eos(rho, want + np.linspace(1.0, 3.0, nz))
    assert eos.failed == 0 and np.array_equal(p, eos.last["P"])
    cells = [oracle.Cell(rho=float(rho[i]), e=float(eos.e_md[i]), n_c=4, rc=2.5, dt=0.004, seed=3, cell_id=i)
             for i in range(nz)]
    o = oracle_many(cells, 1000, 500, (250, 500))
    check_stats(list(eos.last), o, "driver first lifts", [f"zone {i} rho {rho[i]:.3f}" for i in range(nz)])
    eos.close()


def test_piston_into_lj_fluid_with_the_md_eos(ctx):
    print(f"piston into LJ fluid: {N_ZONES} zones, rho1 {RHO1}, e1 {E_MD1} above cold, up {UP}", flush=True)
    eos = MDEOS(N_ZONES, n_c=4, rc=2.5, dt=0.004, seed=3, ctx=ctx)
    e1 = E_MD1 + eos.cold_curve([RHO1])[0]
    s, hist, p1, E0, wall = _run_piston(eos, RHO1, e1, UP, "lj")
    _check_piston(eos, s, hist, RHO1, e1, p1, E0, UP, ctx, dict(n_c=4, rc=2.5, dt=0.004))

    # cost per zone call (a call is one EOS evaluation of one zone)
    steps = len(hist)
    md_warm = eos.seconds / eos.calls
    mg = MieGruneisen(0.4)
    g = Lagrangian1D.tube(N_ZONES, LENGTH, (1.0, 2.5), (0.125, 2.0), mg)
    for _ in range(steps):
        g.step()
    cold = MDEOS(N_ZONES, n_c=4, rc=2.5, dt=0.004, seed=5, mode="cold", ctx=ctx)
    c = Lagrangian1D.tube(N_ZONES, LENGTH, (RHO1, e1), (RHO1, e1), cold, u_left=UP)
    for _ in range(5):
        c.step()
    assert cold.failed == 0
    md_cold = cold.seconds / cold.calls
    cold.close()
    print(f"cost per zone call: Mie-Grueneisen {mg.seconds / mg.calls:.3e} s; MD warm start "
          f"(300 steps, 256 atoms) {md_warm:.3e} s; MD fresh lift (1000 steps) {md_cold:.3e} s; "
          f"{steps} hydro steps, {2 * steps + 1} EOS calls of {N_ZONES} zones in {wall:.2f} s", flush=True)
    assert md_warm < md_cold
    eos.close()


def test_piston_into_eam_copper():
    """The same problem in the embedded-atom stand-in for the paper's
    application material: the fitted lattice (rho 4.0 per a^3), e 3.0 above
    the cold lattice, a piston at 7.3 a/tau."""
    rho1, e_md1, up = 4.0, 3.0, 7.3
    ctx = m.mdeos_create(potential=m.POT_EAM)
    try:
        print(f"piston into EAM copper: {N_ZONES} zones, rho1 {rho1}, e1 {e_md1} above cold, up {up}", flush=True)
        eos = MDEOS(N_ZONES, n_c=4, rc=1.5, dt=0.001, seed=4, ctx=ctx)
        e1 = e_md1 + eos.cold_curve([rho1])[0]
        s, hist, p1, E0, wall = _run_piston(eos, rho1, e1, up, "eam")
        print(f"  {len(hist)} steps in {wall:.2f} s", flush=True)
        _check_piston(eos, s, hist, rho1, e1, p1, E0, up, ctx, dict(n_c=4, rc=1.5, dt=0.001))
        eos.close()
    finally:
        m.mdeos_destroy(ctx)
