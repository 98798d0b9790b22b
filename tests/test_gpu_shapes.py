"""Every launch shape gives the same bits.

A cell's arithmetic is fixed by its spec and plan: reductions run over groups
of 64 consecutive atoms in a fixed order and lists are built in a fixed order,
so the threads per box, atoms per thread, position stride, list location and
register budget of the launch must not change a single bit. Each test forces,
one context at a time, every shape of the library's table that can hold the
box (MDEOS_FORCE_VARIANT, read when a context is created) and compares the
restricted results of a small batch bitwise. A forced shape that does not fit
the plan (for instance a list in LDS that does not fit there) falls back to
the static choice, which the comparison covers as well.
"""
import os
import re

import numpy as np
import pytest

from paper_2508_06012_amd import mdeos as m

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
VARIANTS_H = os.path.join(ROOT, "paper_2508_06012_amd", "csrc", "variants.h")


def shape_table():
    s = open(VARIANTS_H).read()
    found = re.findall(r"X\((\d+), (\d+), (\d+), (\d), (\d), (\d), (\d), (\d)\)", s)
    return sorted(set(tuple(int(v) for v in t) for t in found))


def run_forced(shape, potential, specs, sch, skin):
    os.environ["MDEOS_FORCE_VARIANT"] = ",".join(str(v) for v in shape)
    try:
        ctx = m.mdeos_create(potential=potential, skin=skin)
    finally:
        del os.environ["MDEOS_FORCE_VARIANT"]
    try:
        return m.mdeos_eval_batch(ctx, specs, sch)
    finally:
        m.mdeos_destroy(ctx)


CASES = [
    ("ljts", 0, 0, (0.8442, 1.2, 2.5, 0.005, 0.4)),
    ("ljts-langevin", 0, 1, (0.8442, 1.2, 2.5, 0.005, 0.4)),
    ("eam", 1, 0, (4.4, 20.0, 1.5, 0.001, 0.15)),
    ("eam-langevin", 1, 1, (4.4, 20.0, 1.5, 0.001, 0.15)),
]


@pytest.mark.parametrize("name,potential,ensemble,state", CASES, ids=[c[0] for c in CASES])
def test_every_launch_shape_gives_the_same_bits(name, potential, ensemble, state):
    rho, e, rc, dt, skin = state
    n_c = 4
    N = 4 * n_c ** 3
    specs = m.make_specs(np.full(3, rho), e, n_c, rc, dt, np.arange(3, 6), np.arange(3))
    plan = m.mdeos_plan(specs[0], skin)
    sch = m.make_schedule(200, 100, (50,), 10, 10, ensemble=ensemble, gamma=1.0)
    shapes = [v for v in shape_table()
              if v[5] == 0 and v[6] == ensemble and v[7] == potential and v[0] * v[1] >= N and v[2] - 1 >= plan.ext_cap]
    assert len(shapes) >= 3, shapes
    print(f"{name}: {len(shapes)} launch shapes", flush=True)
    ref = run_forced(shapes[0], potential, specs, sch, skin)
    assert not (ref["status"] & (m.CELL_NONFINITE | m.CELL_OVERFLOW)).any()
    for v in shapes[1:]:
        got = run_forced(v, potential, specs, sch, skin)
        assert got.tobytes() == ref.tobytes(), v


def test_every_minimum_image_shape_gives_the_same_bits():
    """The minimum-image shapes on 2048-atom boxes (dense, rc 3.0, which plan as
    minimum image): 2 to 8 atoms per thread, 512 or 1024 threads, forces in
    registers (2 atoms per thread) or in LDS (4 and more)."""
    n_c, rho, rc, skin = 8, 1.1, 3.0, 0.6
    specs = m.make_specs(np.full(3, rho), 1.5, n_c, rc, 0.004, np.arange(7, 10), np.arange(3))
    plan = m.mdeos_plan(specs[0], skin)
    assert plan.ext_cap == 4087  # minimum image
    sch = m.make_schedule(120, 60, (40,), 10, 10)
    shapes = [v for v in shape_table() if v[5] == 1 and v[6] == 0 and v[7] == 0 and v[0] * v[1] >= plan.N]
    assert len(shapes) >= 4, shapes
    print(f"minimum image: {len(shapes)} launch shapes", flush=True)
    ref = run_forced(shapes[0], 0, specs, sch, skin)
    assert not (ref["status"] & (m.CELL_NONFINITE | m.CELL_OVERFLOW)).any()
    for v in shapes[1:]:
        print(f"  shape {v}", flush=True)
        got = run_forced(v, 0, specs, sch, skin)
        assert got.tobytes() == ref.tobytes(), v
