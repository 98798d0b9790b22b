"""Thermostatted lifting and canonical production on the GPU (GJF Langevin
with temperature updates, Sec. II.B / III) against the FP64 oracle.

The device draws the same Philox uniforms as the oracle and forms the
Gaussian numbers in FP32 (hardware transcendentals), the oracle in FP64; the
noise agrees to about 1e-7 relative, well inside the per-step bars:
  - forces, norm-wise per step: <= 1e-5 (denominator as in test_gpu_parity)
  - E_pot, K and E_tot per step: <= 1e-6 of max(|E_pot|, K)
The 50 steps include a temperature update (step 30), so the window average,
Eq. Tcontribution and the velocity scaling are checked step by step.
Bitwise checks: alone vs in a batch, whole vs chunked (the noise is keyed by
atom, step and query, never by launch or chunk).
"""
import numpy as np
import pytest

import oracle
from paper_2508_06012_amd import mdeos as m
from paper_2508_06012_amd import workloads as wl

pytestmark = pytest.mark.gpu

F_TOL = 1e-5
E_TOL = 1e-6
GAMMA = 1.0


@pytest.fixture(scope="module")
def ctx():
    c = m.mdeos_create()
    yield c
    m.mdeos_destroy(c)


CELLS = [
    oracle.Cell(rho=0.8442, e=wl.e_from_T(1.5, 256).item(), n_c=4, rc=2.5, dt=0.005, seed=7, cell_id=1),
    oracle.Cell(rho=0.5, e=wl.e_from_T(2.0, 500).item(), n_c=5, rc=2.5, dt=0.004, seed=7, cell_id=3),
]


@pytest.mark.parametrize("cell", CELLS, ids=["dense-256", "medium-500"])
def test_first_50_steps_with_a_temperature_update(ctx, cell):
    n = 50
    x0, v0, Ec = oracle.lift(cell)
    ref = oracle.run(cell, oracle.Schedule(n_steps=n, n_avg=10, n_blocks=2, rescale_steps=(30,), energy_every=5,
                                           ensemble=1, gamma=GAMMA), x=x0, v=v0, Ecold_total=Ec, n_recF=n + 1)
    spec = m.make_specs(cell.rho, cell.e, cell.n_c, cell.rc, cell.dt, cell.seed, cell.cell_id)[0]
    sch = m.make_schedule(200, 100, (30,), 10, 5, ensemble=m.NVT_LANGEVIN, gamma=GAMMA)
    print(f"langevin trajectory {cell}", flush=True)
    h = m.mdeos_lift_from_state(ctx, spec, sch, x0, v0)
    F, K, U, W = m.mdeos_debug_trajectory(ctx, h, n, cell.N)
    m.mdeos_release(ctx, [h])
    fn = np.array([np.linalg.norm(ref.F[k]) for k in range(n + 1)])
    ferr = np.array([np.linalg.norm(F[k] - ref.F[k]) / max(fn[k], fn[-1]) for k in range(n + 1)])
    den = np.maximum(np.abs(ref.U), ref.K)
    uerr, kerr = np.abs(U - ref.U) / den, np.abs(K - ref.K) / den
    eerr = np.abs((K + U) - (ref.K + ref.U)) / den
    print(f"max rel err: F {ferr.max():.2e} U {uerr.max():.2e} K {kerr.max():.2e} E {eerr.max():.2e}; "
          f"K jump at the update {ref.K[30] / ref.K[29]:.3f}", flush=True)
    assert ferr.max() <= F_TOL, (ferr.argmax(), ferr.max())
    assert uerr.max() <= E_TOL, (uerr.argmax(), uerr.max())
    assert kerr.max() <= E_TOL, (kerr.argmax(), kerr.max())
    assert eerr.max() <= E_TOL, (eerr.argmax(), eerr.max())


def _specs(n, seed=11):
    rng = np.random.default_rng(seed)
    rho = rng.uniform(0.3, 1.1, size=n)
    T = rng.uniform(0.8, 3.0, size=n)
    nc = rng.choice([3, 4, 5], size=n)
    return m.make_specs(rho, wl.e_from_T(T, 4 * nc ** 3), nc, 2.5, 0.004, 99, np.arange(n))


def test_alone_batch_and_chunked_are_bitwise_equal(ctx):
    sch = m.make_schedule(400, 200, (100, 200), ensemble=m.NVT_LANGEVIN, gamma=GAMMA)
    specs = _specs(24)
    print("langevin batch of 24", flush=True)
    batch = m.mdeos_eval_batch(ctx, specs, sch)
    assert not (batch["status"] & (m.CELL_NONFINITE | m.CELL_OVERFLOW)).any()
    assert not (batch["status"] & m.CELL_DRIFT).any()  # no drift status under a thermostat
    for i in (0, 13, 23):
        alone = m.mdeos_eval_batch(ctx, (m.CellSpec * 1)(specs[i]), sch)[0]
        assert alone.tobytes() == batch[i].tobytes(), i
    h = m.mdeos_lift(ctx, specs, sch)
    for k in (1, 7, 50, 93, 1000):
        m.mdeos_advance(ctx, h, k)
    chunked = m.mdeos_restrict(ctx, h)
    m.mdeos_release(ctx, h)
    assert chunked.tobytes() == batch.tobytes()


def test_warm_start_draws_new_noise(ctx):
    """A warm-started query of a cell uses its own noise stream: the same
    target twice in a row gives different (not bitwise equal) trajectories."""
    cold = m.make_schedule(300, 100, (100, 200), ensemble=m.NVT_LANGEVIN, gamma=GAMMA)
    warm = m.make_schedule(200, 100, (0, 50), ensemble=m.NVT_LANGEVIN, gamma=GAMMA)
    h = m.mdeos_lift(ctx, m.make_specs(0.8, 2.0, 4, 2.5, 0.004, 5, 9), cold)
    m.mdeos_advance(ctx, h, 10 ** 6)
    m.mdeos_warm_start(ctx, h, 0.8, 2.0, warm)
    m.mdeos_advance(ctx, h, 10 ** 6)
    r1 = m.mdeos_restrict(ctx, h)[0]
    m.mdeos_warm_start(ctx, h, 0.8, 2.0, warm)
    m.mdeos_advance(ctx, h, 10 ** 6)
    r2 = m.mdeos_restrict(ctx, h)[0]
    m.mdeos_release(ctx, h)
    assert r1["status"] & (m.CELL_NONFINITE | m.CELL_OVERFLOW) == 0
    assert r1["P"] != r2["P"]
