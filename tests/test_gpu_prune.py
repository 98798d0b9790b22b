"""Inner (pruned) neighbour lists give the same bits.

Between list builds the embedded-atom force walks may use, instead of each
atom's list at rc + skin, the entries within rc + s_in at the last prune, in
list order. A prune follows whenever an atom has moved s_in / 2 since the
previous one, so every pair that comes within rc is still walked, in the same
order. Every entry dropped lies outside rc, where its terms are exact zeros.
So a run with inner lists must equal, bit for bit, the run without them:
every field of every result, for ghost-image and minimum-image boxes and both
integrators. Each case forces a launch shape whose lists live in device
memory (inner lists exist only there) and compares pruning off, the default
s_in and a small s_in that prunes nearly every step. The skins mix the
default (one or few outer lists per run) with a smaller one (many).
"""
import os

import numpy as np
import pytest

from paper_2508_06012_amd import mdeos as m

pytestmark = pytest.mark.gpu


def run(shape, potential, skin, prune_skin, specs, sch):
    os.environ["MDEOS_FORCE_VARIANT"] = ",".join(str(v) for v in shape)
    try:
        ctx = m.mdeos_create(potential=potential, skin=skin, prune_skin=prune_skin)
    finally:
        del os.environ["MDEOS_FORCE_VARIANT"]
    try:
        return m.mdeos_eval_batch(ctx, specs, sch)
    finally:
        m.mdeos_destroy(ctx)


# (name, shape, potential, n_c, rho range, e range, rc, dt, ensemble, skin, inner skins)
CASES = [
    ("eam-ghost", (512, 1, 4096, 0, 2, 0, 0, 1), 1, 5, (4.0, 6.0), (7.0, 35.0), 1.5, 0.001, 0, 0.5, (0.12, 0.02)),
    ("eam-ghost-langevin", (512, 1, 4096, 0, 2, 0, 1, 1), 1, 5, (4.0, 6.0), (7.0, 35.0), 1.5, 0.001, 1, 0.3,
     (0.12, 0.02)),
    ("eam-ghost-small-skin", (512, 1, 4096, 0, 2, 0, 0, 1), 1, 5, (4.0, 6.0), (7.0, 35.0), 1.5, 0.001, 0, 0.3,
     (0.12, 0.02)),
    ("eam-minimum-image", (512, 8, 4088, 0, 1, 1, 0, 1), 1, 10, (4.0, 4.0), (10.0, 20.0), 1.5, 0.001, 0, 0.5,
     (0.12, 0.02)),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_inner_lists_give_the_same_bits(case):
    name, shape, potential, n_c, rho, e, rc, dt, ensemble, skin, inner = case
    n = 6
    rng = np.random.default_rng(11)
    specs = m.make_specs(rng.uniform(*rho, n), rng.uniform(*e, n), n_c, rc, dt, np.arange(20, 20 + n), np.arange(n))
    # every cell fits the forced shape, so no cell falls back to a shape with its list in LDS
    for sp in specs:
        plan = m.mdeos_plan(sp, skin)
        assert plan.ext_cap <= shape[2] - 1 and plan.N <= shape[0] * shape[1], (name, plan.ext_cap)
        if shape[5]:
            assert plan.ext_cap == 4087  # planned as a minimum-image box
    sch = m.make_schedule(400, 200, (100, 200), 10, 10, ensemble=ensemble, gamma=1.0)
    print(f"{name}: shape {shape}, {n} cells of {4 * n_c ** 3} atoms, skin {skin}, inner skins off / {inner}",
          flush=True)
    off = run(shape, potential, skin, -1.0, specs, sch)
    assert not (off["status"] & (m.CELL_NONFINITE | m.CELL_OVERFLOW)).any()
    print(f"  list builds per cell {off['n_builds'].tolist()}", flush=True)
    for ps in inner:
        got = run(shape, potential, skin, ps, specs, sch)
        assert got.tobytes() == off.tobytes(), (name, ps)


def test_mixed_sizes_at_the_default_skins():
    """The default embedded-atom skin is chosen per cell (0.5 up to 1000 atoms,
    0.3 above), so one batch holds buckets planned at different skins, all with
    inner lists. Every cell of such a batch is bitwise equal to itself run
    alone, and to the same cell run with inner lists off."""
    rng = np.random.default_rng(12)
    n_c = np.array([5, 8, 5, 8, 6, 5])
    n = len(n_c)
    specs = m.make_specs(rng.uniform(4.0, 6.0, n), rng.uniform(7.0, 35.0, n), n_c, 1.5, 0.001,
                         np.arange(40, 40 + n), np.arange(n))
    sch = m.make_schedule(300, 150, (75, 150), 10, 10)
    print(f"mixed embedded-atom batch: {(4 * n_c ** 3).tolist()} atoms at the default skins", flush=True)
    ctx = m.mdeos_create(potential=m.POT_EAM)
    off = m.mdeos_create(potential=m.POT_EAM, prune_skin=-1.0)
    try:
        batch = m.mdeos_eval_batch(ctx, specs, sch)
        assert not (batch["status"] & (m.CELL_NONFINITE | m.CELL_OVERFLOW)).any()
        assert batch.tobytes() == m.mdeos_eval_batch(off, specs, sch).tobytes()
        for i in range(n):
            alone = m.mdeos_eval_batch(ctx, (m.CellSpec * 1)(specs[i]), sch)[0]
            assert alone.tobytes() == batch[i].tobytes(), i
    finally:
        m.mdeos_destroy(ctx)
        m.mdeos_destroy(off)
