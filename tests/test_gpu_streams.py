"""Caller streams: a PyTorch stream (a hipStream_t on ROCm) passed through
the binding. Work issued on it gives the same bits as on the context's own
stream, for a whole batch and for lift / advance / restrict; cached launch
graphs are keyed by stream, so none recorded on one stream is replayed on
the other.

PyTorch brings its own HIP runtime, so a process that uses both holds two.
The check runs in a child process of its own, where both start fresh, rather
than late in a long test session.
"""
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r"""
import sys
sys.path.insert(0, sys.argv[1])
import numpy as np
import torch
from paper_2508_06012_amd import mdeos as m

rng = np.random.default_rng(4)
n = 12
specs = m.make_specs(rng.uniform(0.4, 1.0, n), rng.uniform(1.2, 3.0, n), 4, 2.5, 0.004, 9, np.arange(n))
sch = m.make_schedule(300, 100, (50, 100))
ctx = m.mdeos_create()
try:
    ref = m.mdeos_eval_batch(ctx, specs, sch)
    s = torch.cuda.Stream()  # default priority
    got = m.mdeos_eval_batch(ctx, specs, sch, stream=s)
    assert got.tobytes() == ref.tobytes(), "batch on a torch stream"
    h = m.mdeos_lift(ctx, specs, sch, stream=s)
    m.mdeos_advance(ctx, h, 10 ** 6, stream=s)
    r = m.mdeos_restrict(ctx, h, stream=s)
    m.mdeos_release(ctx, h)
    assert r.tobytes() == ref.tobytes(), "lift / advance / restrict on a torch stream"
    torch.cuda.synchronize()
finally:
    m.mdeos_destroy(ctx)
print("torch stream: bitwise equal", flush=True)
"""


def test_torch_stream_gives_the_same_bits():
    pytest.importorskip("torch")
    print("batch and lift/advance/restrict on a torch stream (child process)", flush=True)
    r = subprocess.run([sys.executable, "-c", CHILD, ROOT], capture_output=True, text=True, timeout=240)
    print(r.stdout[-2000:], r.stderr[-2000:], flush=True)
    assert r.returncode == 0
    assert "bitwise equal" in r.stdout
