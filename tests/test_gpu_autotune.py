"""Online launch-shape autotuning.

With autotune on, the first batch of a bucket times candidate launch shapes
on successive chunks of its own work and keeps the fastest in the tune
cache. A cell's results do not depend on the launch shape or on chunk
boundaries, so the tuned batch must equal, bit for bit, the same batch run
with the static choice, and a context that only reads the cache must too.
"""
import json

import numpy as np
import pytest

from paper_2508_06012_amd import mdeos as m
from paper_2508_06012_amd import workloads as wl

pytestmark = pytest.mark.gpu


def test_autotune_writes_cache_and_keeps_bits(tmp_path):
    w = wl.cfg2().subset(np.arange(0, 4096, 4))
    specs, sch = m.specs_from_workload(w)
    cache = str(tmp_path / "tune.json")
    print(f"autotuned batch of {w.n}", flush=True)
    ctx = m.mdeos_create(autotune=1, tune_cache=cache)
    try:
        tuned = m.mdeos_eval_batch(ctx, specs, sch)
    finally:
        m.mdeos_destroy(ctx)
    with open(cache) as f:
        entries = json.load(f)
    print("tune cache:", entries, flush=True)
    assert entries and all("/prec0" in k and len(v) == 8 for k, v in entries.items())

    ctx = m.mdeos_create()
    try:
        static = m.mdeos_eval_batch(ctx, specs, sch)
    finally:
        m.mdeos_destroy(ctx)
    ctx = m.mdeos_create(tune_cache=cache)
    try:
        cached = m.mdeos_eval_batch(ctx, specs, sch)
    finally:
        m.mdeos_destroy(ctx)
    assert not (tuned["status"] & (m.CELL_NONFINITE | m.CELL_OVERFLOW)).any()
    assert tuned.tobytes() == static.tobytes()
    assert cached.tobytes() == static.tobytes()
