"""The no-allocation entry point, mdeos_eval_batch_noalloc, against
mdeos_eval_batch on the same context: the same results bit for bit (a cell's
arithmetic does not depend on launch shapes, buckets or capacities), on two
calls in a row, the second with a smaller input over the workspace the first
left behind; and inputs beyond its stated limits refused with
MDEOS_INVALID_ARG before any device work.
"""
import numpy as np
import pytest

from paper_2508_06012_amd import mdeos as m
from paper_2508_06012_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _specs(n, seed, sizes, rho=(0.3, 1.1), T=(0.8, 3.0), rc=2.5, dt=0.004):
    rng = np.random.default_rng(seed)
    nc = rng.choice(sizes, size=n)
    r = rng.uniform(*rho, size=n)
    t = rng.uniform(*T, size=n)
    return m.make_specs(r, wl.e_from_T(t, 4 * nc ** 3), nc, rc, dt, seed, np.arange(n))


@pytest.mark.parametrize("potential,sizes,rc,dt,rho,T", [
    (m.POT_LJTS, [3, 4, 5, 6, 10], 2.5, 0.004, (0.3, 1.1), (0.8, 3.0)),
    (m.POT_EAM, [3, 4, 5], 1.5, 0.001, (4.0, 5.5), (7.0, 20.0)),
], ids=["ljts", "eam"])
def test_noalloc_equals_eval_batch_on_two_calls(potential, sizes, rc, dt, rho, T):
    ctx = m.mdeos_create(potential=potential)
    try:
        sch = m.make_schedule(300, 100, (50, 100), 10, 10)
        for n, seed in ((64, 1), (19, 2)):
            specs = _specs(n, seed, sizes, rho, T, rc, dt)
            print(f"no-alloc vs batch: potential {potential}, {n} cells", flush=True)
            want = m.mdeos_eval_batch(ctx, specs, sch)
            got = m.mdeos_eval_batch_noalloc(ctx, specs, sch)
            assert not (want["status"] & (m.CELL_NONFINITE | m.CELL_OVERFLOW)).any()
            assert got.tobytes() == want.tobytes()
    finally:
        m.mdeos_destroy(ctx)


def test_noalloc_refuses_inputs_beyond_its_limits():
    ctx = m.mdeos_create()
    try:
        sch = m.make_schedule(100, 50, (), 10, 10)
        too_many = _specs(4097, 3, [3])
        with pytest.raises(m.MdeosError) as e:
            m.mdeos_eval_batch_noalloc(ctx, too_many, sch)
        assert e.value.status == m.INVALID_ARG
        # 400 boxes of 4000 atoms: 115 MB of atom state against a 64 MiB workspace
        too_big = _specs(400, 4, [10])
        with pytest.raises(m.MdeosError) as e:
            m.mdeos_eval_batch_noalloc(ctx, too_big, sch)
        assert e.value.status == m.INVALID_ARG and "workspace" in str(e.value)
        # the context still works afterwards
        small = _specs(8, 5, [4])
        assert m.mdeos_eval_batch_noalloc(ctx, small, sch).tobytes() == m.mdeos_eval_batch(ctx, small, sch).tobytes()
    finally:
        m.mdeos_destroy(ctx)
