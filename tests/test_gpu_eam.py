"""The embedded-atom form (Eq. Etot, the Sutton-Chen (9, 6) stand-in in
shifted-force truncation) on the GPU, through the C ABI, against the FP64
oracle.

The bars are those of the LJTS path:
  - forces, norm-wise per step: ||F_gpu - F_orc|| / ||F_orc|| <= 1e-5
  - E_pot and E_tot per step: |dE| / max(|E_pot|, K) <= 1e-6; W per step to
    1e-5 of max(|W|, |E_pot|) (it carries the force rounding)
Covered: ghost-image boxes (lists in LDS and in device memory), a box whose
cutoff exceeds half its edge (several images of one atom in range), a larger
cutoff, and a minimum-image box of 4000 atoms; the lift; 50 free-running
steps with an energy re-pin; bitwise alone vs batch vs chunked; a context
of each potential side by side; the Langevin shapes (50 GJF steps with a
temperature update, per step, and batch vs alone). Replica ensembles of two
states are in test_gpu_ensembles.py.
"""
import numpy as np
import pytest

import oracle
from paper_2508_06012_amd import mdeos as m
from paper_2508_06012_amd import workloads as wl

pytestmark = pytest.mark.gpu

F_TOL = 1e-5
E_TOL = 1e-6
W_TOL = 1e-5
C_SC = 39.432


@pytest.fixture(scope="module")
def ctx():
    c = m.mdeos_create(potential=m.POT_EAM)
    yield c
    m.mdeos_destroy(c)


def gspec(cell: oracle.Cell):
    return m.make_specs(cell.rho, cell.e, cell.n_c, cell.rc, cell.dt, cell.seed, cell.cell_id)[0]


def relnorm(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def ecell(rho, T, n_c, rc=1.5, cell_id=1):
    return oracle.Cell(rho=rho, e=wl.e_from_T(T, 4 * n_c ** 3).item(), n_c=n_c, rc=rc, dt=0.001, seed=7,
                       cell_id=cell_id, potential=1, eam_c=C_SC)


CELLS = [ecell(4.4, 14.0, 4, cell_id=1), ecell(5.5, 30.0, 5, cell_id=2), ecell(4.4, 10.0, 3, cell_id=3),
         ecell(3.6, 7.0, 6, rc=1.8, cell_id=4)]
IDS = ["eam-256", "eam-500-hot", "eam-multi-image-108", "eam-rc1.8-864"]


@pytest.mark.parametrize("cell", CELLS, ids=IDS)
def test_forces_on_oracle_positions(ctx, cell):
    r = oracle.run(cell, oracle.Schedule(n_steps=60, n_avg=20, n_blocks=2, rescale_steps=(20,)))
    L = oracle.box_length(cell.n_c, cell.rho)
    x = r.x.astype(np.float32).astype(np.float64)
    F0, U0, W0, _, _ = oracle.forces_eam(x, L, cell.rc, C_SC)
    print(f"eam debug_forces {cell}", flush=True)
    F, U, W = m.mdeos_debug_forces(ctx, gspec(cell), x)
    print(f"  rel F {relnorm(F, F0):.2e} U {abs(U - U0) / abs(U0):.2e} W {abs(W - W0) / max(abs(W0), abs(U0)):.2e}",
          flush=True)
    assert relnorm(F, F0) <= F_TOL
    assert abs(U - U0) <= E_TOL * abs(U0)
    assert abs(W - W0) <= W_TOL * max(abs(W0), abs(U0))


def test_forces_minimum_image_4000(ctx):
    """A box too large for ghost images in LDS: the minimum-image variant."""
    cell = ecell(4.0, 20.0, 10, cell_id=5)
    plan = m.mdeos_plan(gspec(cell), 0.3)  # the default embedded-atom skin above 1000 atoms
    assert plan.ext_cap == 4087  # the minimum-image plan: real atoms only
    rng = np.random.default_rng(3)
    L = oracle.box_length(cell.n_c, cell.rho)
    x = (oracle.lattice(cell.n_c, cell.rho) + rng.uniform(-0.08, 0.08, size=(cell.N, 3))) % L
    x = x.astype(np.float32).astype(np.float64)
    F0, U0, W0, _, _ = oracle.forces_eam(x, L, cell.rc, C_SC)
    print(f"eam debug_forces minimum image {cell}", flush=True)
    F, U, W = m.mdeos_debug_forces(ctx, gspec(cell), x)
    print(f"  rel F {relnorm(F, F0):.2e} U {abs(U - U0) / abs(U0):.2e}", flush=True)
    assert relnorm(F, F0) <= F_TOL
    assert abs(U - U0) <= E_TOL * abs(U0)
    assert abs(W - W0) <= W_TOL * max(abs(W0), abs(U0))


@pytest.mark.parametrize("cell", CELLS, ids=IDS)
def test_lift_matches_oracle(ctx, cell):
    sch = m.make_schedule(10, 10, (), 2)
    x0, v0, Ec = oracle.lift(cell)
    print(f"eam lift {cell}", flush=True)
    h = m.mdeos_lift(ctx, [gspec(cell)], sch)[0]
    xyz, v, step = m.mdeos_state_export(ctx, h, cell.N)
    m.mdeos_advance(ctx, [h], 10 ** 6)
    r = m.mdeos_restrict(ctx, [h])[0]
    m.mdeos_release(ctx, [h])
    assert step == 0
    assert np.array_equal(xyz, x0)
    assert np.abs(v - v0).max() <= 2.4e-7 * np.abs(v0).max()
    assert r["Ecold"] * cell.N == pytest.approx(Ec, rel=E_TOL)


@pytest.mark.parametrize("cell", CELLS[:3], ids=IDS[:3])
def test_first_50_steps(ctx, cell):
    n = 50
    x0, v0, Ec = oracle.lift(cell)
    ref = oracle.run(cell, oracle.Schedule(n_steps=n, n_avg=10, n_blocks=2, rescale_steps=(20,), energy_every=5),
                     x=x0, v=v0, Ecold_total=Ec, n_recF=n + 1)
    sch = m.make_schedule(200, 100, (20,), 10, 5)
    print(f"eam trajectory {cell}", flush=True)
    h = m.mdeos_lift_from_state(ctx, gspec(cell), sch, x0, v0)
    F, K, U, W = m.mdeos_debug_trajectory(ctx, h, n, cell.N)
    m.mdeos_release(ctx, [h])
    fn = np.array([np.linalg.norm(ref.F[k]) for k in range(n + 1)])
    ferr = np.array([np.linalg.norm(F[k] - ref.F[k]) / max(fn[k], fn[-1]) for k in range(n + 1)])
    den = np.maximum(np.abs(ref.U), ref.K)
    uerr, kerr = np.abs(U - ref.U) / den, np.abs(K - ref.K) / den
    eerr = np.abs((K + U) - (ref.K + ref.U)) / den
    werr = np.abs(W - ref.W) / np.maximum(np.abs(ref.W), np.abs(ref.U))
    print(f"  max rel err: F {ferr.max():.2e} U {uerr.max():.2e} K {kerr.max():.2e} E {eerr.max():.2e} "
          f"W {werr.max():.2e}", flush=True)
    assert ferr.max() <= F_TOL, (ferr.argmax(), ferr.max())
    assert uerr.max() <= E_TOL and kerr.max() <= E_TOL and eerr.max() <= E_TOL
    assert werr.max() <= W_TOL


def test_kahan_mode_first_50_steps():
    """The compensated-FP32 accumulation of the embedded-atom walk, per step
    against the oracle (same bars as the FP64 mode)."""
    cell = CELLS[0]
    n = 50
    x0, v0, Ec = oracle.lift(cell)
    ref = oracle.run(cell, oracle.Schedule(n_steps=n, n_avg=10, n_blocks=2, rescale_steps=(20,), energy_every=5),
                     x=x0, v=v0, Ecold_total=Ec, n_recF=n + 1)
    kctx = m.mdeos_create(potential=m.POT_EAM, precision=m.PREC_KAHAN)
    try:
        print(f"eam kahan trajectory {cell}", flush=True)
        h = m.mdeos_lift_from_state(kctx, gspec(cell), m.make_schedule(200, 100, (20,), 10, 5), x0, v0)
        F, K, U, W = m.mdeos_debug_trajectory(kctx, h, n, cell.N)
        m.mdeos_release(kctx, [h])
    finally:
        m.mdeos_destroy(kctx)
    fn = np.array([np.linalg.norm(ref.F[k]) for k in range(n + 1)])
    ferr = np.array([np.linalg.norm(F[k] - ref.F[k]) / max(fn[k], fn[-1]) for k in range(n + 1)])
    den = np.maximum(np.abs(ref.U), ref.K)
    uerr, kerr = np.abs(U - ref.U) / den, np.abs(K - ref.K) / den
    werr = np.abs(W - ref.W) / np.maximum(np.abs(ref.W), np.abs(ref.U))
    print(f"  max rel err: F {ferr.max():.2e} U {uerr.max():.2e} K {kerr.max():.2e} W {werr.max():.2e}", flush=True)
    assert ferr.max() <= F_TOL and uerr.max() <= E_TOL and kerr.max() <= E_TOL and werr.max() <= W_TOL


def test_alone_batch_and_chunked_are_bitwise_equal(ctx):
    w = wl.eam_cu().subset(np.arange(0, 4096, 128))
    specs, sch = m.specs_from_workload(w)
    sch = m.make_schedule(400, 200, (100, 200))
    print(f"eam batch of {w.n}", flush=True)
    batch = m.mdeos_eval_batch(ctx, specs, sch)
    assert not (batch["status"] & (m.CELL_NONFINITE | m.CELL_OVERFLOW)).any()
    for i in (0, 17, w.n - 1):
        alone = m.mdeos_eval_batch(ctx, (m.CellSpec * 1)(specs[i]), sch)[0]
        assert alone.tobytes() == batch[i].tobytes(), i
    h = m.mdeos_lift(ctx, specs, sch)
    for k in (1, 9, 50, 77, 1000):
        m.mdeos_advance(ctx, h, k)
    chunked = m.mdeos_restrict(ctx, h)
    m.mdeos_release(ctx, h)
    assert chunked.tobytes() == batch.tobytes()
    assert batch["Ecold"].max() < -100.0  # cohesive energies of the many-body crystal


def test_each_context_runs_its_own_potential(ctx):
    """One spec valid for both materials (a dilute state in either unit
    system), evaluated by an LJTS and an embedded-atom context side by side:
    each E_cold is its own potential's, as the oracle computes it."""
    kw = dict(rho=1.0, e=1.5, n_c=4, rc=1.5, dt=0.001, seed=3, cell_id=0)
    sch = m.make_schedule(20, 10, (), 2)
    spec = m.make_specs(kw["rho"], kw["e"], kw["n_c"], kw["rc"], kw["dt"], kw["seed"], kw["cell_id"])
    lj = m.mdeos_create()
    try:
        r_lj = m.mdeos_eval_batch(lj, spec, sch)[0]
    finally:
        m.mdeos_destroy(lj)
    r_eam = m.mdeos_eval_batch(ctx, spec, sch)[0]
    N = 4 * kw["n_c"] ** 3
    e_lj = oracle.ecold_cell(oracle.Cell(**kw)) / N
    e_eam = oracle.ecold_cell(oracle.Cell(**kw, potential=1, eam_c=C_SC)) / N
    print(f"E_cold/N: LJTS {r_lj['Ecold']:.6f} (oracle {e_lj:.6f}), EAM {r_eam['Ecold']:.6f} (oracle {e_eam:.6f})",
          flush=True)
    assert r_lj["Ecold"] == pytest.approx(e_lj, rel=E_TOL)
    assert r_eam["Ecold"] == pytest.approx(e_eam, rel=E_TOL)


def test_langevin_first_50_steps_with_a_temperature_update(ctx):
    """The embedded-atom Langevin shapes: 50 GJF steps with a temperature
    update at step 30 against the oracle, per step (noise as in
    test_gpu_nvt.py: the same Philox words, Gaussians in FP32 on the device)."""
    cell = ecell(4.4, 14.0, 4, cell_id=6)
    n = 50
    x0, v0, Ec = oracle.lift(cell)
    ref = oracle.run(cell, oracle.Schedule(n_steps=n, n_avg=10, n_blocks=2, rescale_steps=(30,), energy_every=5,
                                           ensemble=1, gamma=1.0), x=x0, v=v0, Ecold_total=Ec, n_recF=n + 1)
    sch = m.make_schedule(200, 100, (30,), 10, 5, ensemble=m.NVT_LANGEVIN, gamma=1.0)
    print(f"eam langevin trajectory {cell}", flush=True)
    h = m.mdeos_lift_from_state(ctx, gspec(cell), sch, x0, v0)
    F, K, U, W = m.mdeos_debug_trajectory(ctx, h, n, cell.N)
    m.mdeos_release(ctx, [h])
    fn = np.array([np.linalg.norm(ref.F[k]) for k in range(n + 1)])
    ferr = np.array([np.linalg.norm(F[k] - ref.F[k]) / max(fn[k], fn[-1]) for k in range(n + 1)])
    den = np.maximum(np.abs(ref.U), ref.K)
    uerr, kerr = np.abs(U - ref.U) / den, np.abs(K - ref.K) / den
    print(f"  max rel err: F {ferr.max():.2e} U {uerr.max():.2e} K {kerr.max():.2e}; "
          f"K jump at the update {ref.K[30] / ref.K[29]:.3f}", flush=True)
    assert ferr.max() <= F_TOL, (ferr.argmax(), ferr.max())
    assert uerr.max() <= E_TOL and kerr.max() <= E_TOL


def test_langevin_batch_is_bitwise_equal_to_alone(ctx):
    w = wl.eam_cu().subset(np.arange(5, 4096, 256))
    specs, _ = m.specs_from_workload(w)
    sch = m.make_schedule(300, 100, (100, 200), ensemble=m.NVT_LANGEVIN, gamma=1.0)
    print(f"eam langevin batch of {w.n}", flush=True)
    batch = m.mdeos_eval_batch(ctx, specs, sch)
    assert not (batch["status"] & (m.CELL_NONFINITE | m.CELL_OVERFLOW)).any()
    for i in (0, w.n - 1):
        alone = m.mdeos_eval_batch(ctx, (m.CellSpec * 1)(specs[i]), sch)[0]
        assert alone.tobytes() == batch[i].tobytes(), i


def test_langevin_minimum_image_4000_first_20_steps(ctx):
    """The Langevin shape for embedded-atom boxes too large for ghost images
    (4000 atoms, minimum image): 20 GJF steps with a temperature update at
    step 10, per step against the oracle."""
    cell = ecell(4.0, 14.0, 10, cell_id=9)
    assert m.mdeos_plan(gspec(cell), 0.3).ext_cap == 4087
    n = 20
    x0, v0, Ec = oracle.lift(cell)
    ref = oracle.run(cell, oracle.Schedule(n_steps=n, n_avg=10, n_blocks=2, rescale_steps=(10,), energy_every=5,
                                           ensemble=1, gamma=1.0), x=x0, v=v0, Ecold_total=Ec, n_recF=n + 1)
    sch = m.make_schedule(200, 100, (10,), 10, 5, ensemble=m.NVT_LANGEVIN, gamma=1.0)
    print(f"eam langevin minimum image {cell}", flush=True)
    h = m.mdeos_lift_from_state(ctx, gspec(cell), sch, x0, v0)
    F, K, U, W = m.mdeos_debug_trajectory(ctx, h, n, cell.N)
    m.mdeos_release(ctx, [h])
    fn = np.array([np.linalg.norm(ref.F[k]) for k in range(n + 1)])
    ferr = np.array([np.linalg.norm(F[k] - ref.F[k]) / max(fn[k], fn[-1]) for k in range(n + 1)])
    den = np.maximum(np.abs(ref.U), ref.K)
    uerr, kerr = np.abs(U - ref.U) / den, np.abs(K - ref.K) / den
    print(f"  max rel err: F {ferr.max():.2e} U {uerr.max():.2e} K {kerr.max():.2e}", flush=True)
    assert ferr.max() <= F_TOL and uerr.max() <= E_TOL and kerr.max() <= E_TOL


def test_eam_batch_full_size():
    """The embedded-atom batch at full size (4096 cells of 500 atoms, 2000
    steps) in the launch configuration the bench times (autotuned shapes,
    skin 0.5, inner lists at rc + 0.12): the oracle on the stratified sample
    of up to 64 cells at the statistical bar, and eight of those cells run
    again as a batch of their own, bitwise equal to their full-batch results."""
    from _stats import check_stats, oracle_many
    w = wl.eam_cu()
    specs, sch = m.specs_from_workload(w)
    tctx = m.mdeos_create(autotune=1, potential=m.POT_EAM, skin=0.5, prune_skin=0.12)
    try:
        print("eam batch of 4096", flush=True)
        res = m.mdeos_eval_batch(tctx, specs, sch)
        bad = (res["status"] & (m.CELL_NONFINITE | m.CELL_OVERFLOW)) != 0
        assert not bad.any(), np.nonzero(bad)
        assert (res["n_samples"] == w.sched.n_avg).all()
        pick = wl.stratified_sample(w)
        assert len(pick) >= 48, len(pick)
        sub = pick[:: max(1, len(pick) // 8)][:8]
        s2, _ = m.specs_from_workload(w.subset(sub))
        again = m.mdeos_eval_batch(tctx, s2, sch)
        for k, i in enumerate(sub):
            assert again[k].tobytes() == res[i].tobytes(), i
    finally:
        m.mdeos_destroy(tctx)
    cells = [oracle.Cell(rho=float(w.rho[i]), e=float(w.e[i]), n_c=5, rc=1.5, dt=0.001, seed=int(w.seed),
                         cell_id=int(w.cell_id[i]), potential=1, eam_c=C_SC) for i in pick]
    s = w.sched
    o = oracle_many(cells, s.n_steps, s.n_avg, s.rescale_steps)
    # E_cold of a compressed lattice is a large repulsive pair sum less a large
    # embedding term (at rho 5.9: +452 and -595 per atom, net -143). FP32 pair
    # terms carry a relative error of order 1e-7 each, and on a lattice the
    # pairs of one shell share it, so the bar is 1e-6 of the two magnitudes.
    bar = []
    for c in cells:
        x = oracle.lattice(c.n_c, c.rho)
        _, U, _, _, rb = oracle.forces_eam(x, oracle.box_length(c.n_c, c.rho), c.rc, c.eam_c)
        emb = -c.eam_c * np.sqrt(rb).sum()
        bar.append(1e-6 * (abs(U - emb) + abs(emb)) / len(x))
    check_stats([res[i] for i in pick], o, "eam", [f"cell {i} rho {w.rho[i]:.3f} T {w.T[i]:.1f}" for i in pick],
                ecold_abs=bar)
