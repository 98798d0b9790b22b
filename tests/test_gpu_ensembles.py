"""Replica-ensemble parity: the mean of a time average over M independent
replicas (Philox seeds 1..M) of one state, device path against the oracle.

The oracle's per-replica averages are stored in golden/replica_ensembles.json
(written by golden/make_replica_ensembles.py, which calls only the oracle).
The bar: |mean_gpu - mean_oracle| <= 0.5 % of max(|<P>|, rho <T>) for P and of
<T> for T. M must be large enough that three combined standard errors of the
two means fit under that bar, or the comparison could not see a 0.5 % error;
the test checks that too, with the replica spreads it measures.
"""
import json
import math
import os

import numpy as np
import pytest

from paper_2508_06012_amd import mdeos as m

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "replica_ensembles.json")


def _states():
    with open(GOLDEN) as f:
        return {s["name"]: s for s in json.load(f)["states"]}


STATES = _states()
CASES = [(n, m.PREC_FP64) for n in STATES] + [("cfg1", m.PREC_KAHAN), ("rc4-864", m.PREC_KAHAN)]


@pytest.mark.parametrize("name,prec", CASES, ids=[f"{n}-{'kahan' if p else 'fp64'}" for n, p in CASES])
def test_replica_mean_matches_oracle(name, prec):
    s = STATES[name]
    M = s["M"]
    print(f"replicas {name} M {M} precision {prec}", flush=True)
    ctx = m.mdeos_create(precision=prec, potential=s.get("potential", 0))
    try:
        specs = m.make_specs(np.full(M, s["rho"]), np.full(M, s["e"]), s["n_c"], s["rc"], s["dt"],
                             np.arange(s["seed0"], s["seed0"] + M), s["cell_id"])
        sch = m.make_schedule(s["n_steps"], s["n_avg"], tuple(s["rescale_steps"]), s["n_blocks"], s["energy_every"],
                              ensemble=s.get("ensemble", 0), gamma=s.get("gamma", 0.0))
        res = m.mdeos_eval_batch(ctx, specs, sch)
    finally:
        m.mdeos_destroy(ctx)
    assert ((res["status"] & (m.CELL_NONFINITE | m.CELL_OVERFLOW)) == 0).all()
    Po, To = np.array(s["P"]), np.array(s["T"])
    Pg, Tg = res["P"], res["T"]
    scale_P = max(abs(Po.mean()), s["rho"] * To.mean())
    scale_T = To.mean()
    for what, g, o, scale in (("P", Pg, Po, scale_P), ("T", Tg, To, scale_T)):
        d = g.mean() - o.mean()
        se = math.sqrt(g.var(ddof=1) / M + o.var(ddof=1) / M)
        print(f"  {what}: gpu {g.mean():.5f} oracle {o.mean():.5f} diff {d:+.5f} ({d / scale * 100:+.3f} %), "
              f"3 SE {3 * se / scale * 100:.3f} %, sd gpu {g.std(ddof=1):.5f} oracle {o.std(ddof=1):.5f}", flush=True)
        assert 3 * se <= 0.005 * scale, f"{what}: too few replicas to resolve 0.5 %"
        assert abs(d) <= 0.005 * scale, what
