"""The restricting operator on the GPU (Sec. III, Eq. stress; the RMS of
Sec. IV) against the oracle's per-step records, and the per-cell status bits
of a restriction: a partial window, the drift flag, a cell whose forces are
not finite, and the batch paths' capacity retry.

From identical starting bits the device trajectory equals the oracle's to
~1e-7 over these few dozen steps, so pressure-like fields meet the force bar
(1e-5 of max(|<P>|, rho <T>)) and energy-like fields the energy bar (1e-6).
"""
import math
import os

import numpy as np
import pytest

import oracle
from paper_2508_06012_amd import mdeos as m
from paper_2508_06012_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = m.mdeos_create()
    yield c
    m.mdeos_destroy(c)


def _spec(cell):
    return m.make_specs(cell.rho, cell.e, cell.n_c, cell.rc, cell.dt, cell.seed, cell.cell_id)[0]


CELL = oracle.Cell(rho=0.8442, e=wl.e_from_T(1.2, 256).item(), n_c=4, rc=2.5, dt=0.005, seed=7, cell_id=11)


def test_partial_window_restriction(ctx):
    """Restrict after 5, 35 and 45 of 60 steps (window 21..60, 4 blocks of
    10): averages over the samples recorded so far, block errors over the
    completed blocks only, NaN drift, and MDEOS_NOT_READY as the call status."""
    n, na, B = 60, 40, 4
    x0, v0, Ec = oracle.lift(CELL)
    ref = oracle.run(CELL, oracle.Schedule(n, na, n_blocks=B, rescale_steps=(10,), energy_every=1), x=x0, v=v0,
                     Ecold_total=Ec)
    sch = m.make_schedule(n, na, (10,), B, 1)
    print("partial restriction, 256 atoms", flush=True)
    h = m.mdeos_lift_from_state(ctx, _spec(CELL), sch, x0, v0)
    lib = m.lib()
    w0 = n - na
    pscale = max(abs(ref.result.P), CELL.rho * ref.result.T)
    done_steps = 0
    for stop in (5, 35, 45):
        m.mdeos_advance(ctx, [h], stop - done_steps)
        done_steps = stop
        hh = m._handles([h])
        out = (m.Result * 1)()
        st = lib.mdeos_restrict(ctx, 1, hh, out, None)
        assert st == m.NOT_READY, st
        g = m.results_to_numpy(out)[0]
        k = max(0, stop - w0)
        assert g["n_samples"] == k
        assert math.isnan(g["drift"])
        if k == 0:
            assert math.isnan(g["P"]) and math.isnan(g["T"]) and math.isnan(g["P_se"])
            continue
        w = np.arange(w0 + 1, stop + 1)
        P, T = ref.P[w], ref.T[w]
        assert abs(g["P"] - P.mean()) <= 1e-5 * pscale, (g["P"], P.mean())
        assert abs(g["T"] - T.mean()) <= 1e-6 * T.mean()
        assert abs(g["P_rms"] - math.sqrt(((P - P.mean()) ** 2).mean())) <= 1e-5 * pscale
        assert abs(g["Epot_mean"] - ref.U[w].mean() / CELL.N) <= 1e-6 * abs(ref.U[w].mean() / CELL.N)
        bl = na // B
        nb = k // bl
        if nb < 2:
            assert math.isnan(g["P_se"]) and math.isnan(g["T_se"])
        else:
            mb = P[: nb * bl].reshape(nb, bl).mean(axis=1)
            se = math.sqrt(((mb - mb.mean()) ** 2).sum() / (nb * (nb - 1)))
            assert abs(g["P_se"] - se) <= 1e-5 * pscale, (g["P_se"], se)
    m.mdeos_advance(ctx, [h], n)
    g = m.mdeos_restrict(ctx, [h])[0]
    m.mdeos_release(ctx, [h])
    assert g["n_samples"] == na and math.isfinite(g["drift"]) and math.isfinite(g["P_se"])


def test_drift_flag_matches_the_oracle(ctx):
    """From identical bits the drift agrees to the energy bar, so a tolerance
    half or twice the oracle's |drift| sets the flag on both sides alike."""
    cell = oracle.Cell(rho=0.9, e=wl.e_from_T(2.5, 256).item(), n_c=4, rc=2.5, dt=0.008, seed=2, cell_id=1)
    n, na = 60, 30
    x0, v0, Ec = oracle.lift(cell)
    base = oracle.run(cell, oracle.Schedule(n, na, n_blocks=3, rescale_steps=(10,), drift_tol=1e9), x=x0, v=v0,
                      Ecold_total=Ec).result
    d = abs(base.drift)
    print(f"drift flag: oracle drift {base.drift:.3e}", flush=True)
    assert d > 1e-5
    for tol, flagged in ((0.5 * d, True), (2.0 * d, False)):
        o = oracle.run(cell, oracle.Schedule(n, na, n_blocks=3, rescale_steps=(10,), drift_tol=tol), x=x0, v=v0,
                       Ecold_total=Ec).result
        h = m.mdeos_lift_from_state(ctx, _spec(cell), m.make_schedule(n, na, (10,), 3, 10, drift_tol=tol), x0, v0)
        m.mdeos_advance(ctx, [h], n)
        g = m.mdeos_restrict(ctx, [h])[0]
        m.mdeos_release(ctx, [h])
        assert abs(g["drift"] - base.drift) <= 1e-6 * max(abs(base.Epot_mean), base.T) * 2
        assert bool(o.status & oracle.DRIFT) == flagged
        assert bool(g["status"] & m.CELL_DRIFT) == flagged, (tol, g["drift"])


def test_coincident_atoms_are_flagged_nonfinite(ctx):
    """Two atoms at one point in a ghost-image box: the pair term is infinite,
    the forces of the first step are NaN on both sides, the cell stops and is
    flagged, and its averages are NaN."""
    cell = oracle.Cell(rho=0.8, e=1.0, n_c=4, rc=2.5, dt=0.005, seed=3, cell_id=2)
    x, v, Ec = oracle.lift(cell)
    x[5] = x[9]
    o = oracle.run(cell, oracle.Schedule(50, 20, n_blocks=2), x=x, v=v, Ecold_total=Ec).result
    assert o.status & oracle.NONFINITE
    plan = m.mdeos_plan(_spec(cell), 0.4)
    assert plan.ext_cap in (2047, 3071, 4095, 8175)  # ghost images (minimum image: 4087 usable slots)
    sch = m.make_schedule(50, 20, (), 2, 10)
    print("nonfinite: coincident atoms", flush=True)
    h = m.mdeos_lift_from_state(ctx, _spec(cell), sch, x, v)
    m.mdeos_advance(ctx, [h], 50)
    g = m.mdeos_restrict(ctx, [h])[0]
    m.mdeos_release(ctx, [h])
    assert g["status"] & m.CELL_NONFINITE
    for f in ("P", "P_se", "P_rms", "T", "T_se", "Epot_mean", "drift"):
        assert math.isnan(g[f]), f
    assert g["Ecold"] == pytest.approx(o.Ecold, rel=1e-6)


def test_capacity_retry_gives_the_same_bits():
    """MDEOS_SHRINK_CAPS plans every cell with an 8-entry list, so each cell
    overflows at its first list build and eval re-runs it from the lift with
    capacities from the overflow's measured sizes. Capacities never change a
    cell's arithmetic: the retried results equal an unforced run bit for bit,
    on both batch paths."""
    rng = np.random.default_rng(5)
    n = 24
    nc = rng.choice([3, 4, 5, 6], size=n)
    rho = rng.uniform(0.3, 1.1, size=n)
    T = rng.uniform(0.8, 3.0, size=n)
    specs = m.make_specs(rho, wl.e_from_T(T, 4 * nc ** 3), nc, 2.5, 0.004, 9, np.arange(n))
    sch = m.make_schedule(400, 200, (50, 100), 10, 10)
    c0 = m.mdeos_create()
    try:
        print("capacity retry: reference", flush=True)
        want = m.mdeos_eval_batch(c0, specs, sch)
    finally:
        m.mdeos_destroy(c0)
    os.environ["MDEOS_SHRINK_CAPS"] = "1"
    try:
        c1 = m.mdeos_create()
    finally:
        del os.environ["MDEOS_SHRINK_CAPS"]
    try:
        print("capacity retry: shrunk capacities", flush=True)
        got = m.mdeos_eval_batch(c1, specs, sch)
        got_plain = m.mdeos_eval_plain(c1, m.make_specs(rho[:4], wl.e_from_T(T[:4], 4 * nc[:4] ** 3), nc[:4], 2.5,
                                                        0.004, 9, np.arange(4)), sch)
    finally:
        m.mdeos_destroy(c1)
    print(f"  status batch {got['status'].tolist()} plain {got_plain['status'].tolist()}", flush=True)
    assert not (want["status"] & m.CELL_OVERFLOW).any()
    assert not (got["status"] & m.CELL_OVERFLOW).any()
    assert not (got_plain["status"] & m.CELL_OVERFLOW).any()
    assert got.tobytes() == want.tobytes()
    assert got_plain.tobytes() == want[:4].tobytes()
