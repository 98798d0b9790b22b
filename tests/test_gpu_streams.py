"""Caller streams: a PyTorch stream (a hipStream_t on ROCm) passed through
the binding. Work issued on it gives the same bits as on the context's own
stream, for a whole batch and for lift / advance / restrict; cached launch
graphs are keyed by stream, so none recorded on one stream is replayed on
the other.

PyTorch ships its own HIP runtime under the system runtime's soname. The
binding imports torch before it loads the library, so the process maps one
runtime and a torch stream is a handle of the runtime the library uses. This
test runs in the suite's own process, after every test before it has created
and destroyed contexts.
"""
import numpy as np
import pytest

from paper_2508_06012_amd import mdeos as m

pytestmark = pytest.mark.gpu


def test_torch_stream_gives_the_same_bits():
    torch = pytest.importorskip("torch")
    m.lib()
    rt = m.hip_runtimes()
    print(f"HIP runtimes mapped: {sorted(rt)}", flush=True)
    assert len(rt) == 1, rt
    rng = np.random.default_rng(4)
    n = 12
    specs = m.make_specs(rng.uniform(0.4, 1.0, n), rng.uniform(1.2, 3.0, n), 4, 2.5, 0.004, 9, np.arange(n))
    sch = m.make_schedule(300, 100, (50, 100))
    ctx = m.mdeos_create()
    try:
        print("batch and lift/advance/restrict on a torch stream", flush=True)
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
