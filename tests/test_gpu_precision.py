"""Per-atom accumulation A/B on the large rc = 4 workload: FP64 sums against
Kahan-compensated FP32 sums of the pair energy and virial terms.

Both modes run the full batch of 65,536 boxes of 864 atoms. On the fixed
64-cell stratified subsample both are compared with the oracle:
* per step for steps 0..50 from identical starting bits (the oracle's lift):
  |dU| <= 1e-6 max(|U|, K) (the energy bar) and |dW| <= 1e-5 max(|W|, |U|, K)
  (the force bar: W = sum r.f is a force moment, and at hot dense states it
  is dominated by a few close pairs whose FP32 pair virial carries about
  12 times the relative rounding of their separation);
* <P> and <T> against golden/cfg5_sample.json (oracle full runs), through the
  statistical criterion of test_gpu_workloads.
"""
import json
import multiprocessing as mp
import os
import time

import numpy as np
import pytest

import oracle
from paper_2508_06012_amd import mdeos as m
from paper_2508_06012_amd import workloads as wl
from _stats import check_stats

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "cfg5_sample.json")
N_STEPS = 50
MODES = [(m.PREC_FP64, "fp64"), (m.PREC_KAHAN, "kahan")]


def ocell(w, i):
    return oracle.Cell(rho=float(w.rho[i]), e=float(w.e[i]), n_c=int(w.n_c[i]), rc=float(w.rc[i]),
                       dt=float(w.dt[i]), seed=int(w.seed), cell_id=int(w.cell_id[i]))


def _steps_job(cell):
    x0, v0, Ec = oracle.lift(cell)
    r = oracle.run(cell, oracle.Schedule(n_steps=N_STEPS, n_avg=10, n_blocks=2, energy_every=1), x=x0, v=v0,
                   Ecold_total=Ec)
    return x0, v0, Ec, r.K, r.U, r.W


@pytest.fixture(scope="module")
def sample():
    w = wl.cfg5()
    with open(GOLDEN) as f:
        g = json.load(f)
    pick = [c["index"] for c in g["cells"]]
    assert pick == list(wl.stratified_sample(w))
    with mp.get_context("fork").Pool(min(16, os.cpu_count() or 1)) as pool:
        steps = pool.map(_steps_job, [ocell(w, i) for i in pick], chunksize=1)
    return w, g["cells"], pick, steps


@pytest.mark.parametrize("prec,name", MODES, ids=[n for _, n in MODES])
def test_per_step_energy_and_virial(sample, prec, name):
    w, _, pick, steps = sample
    print(f"per-step W, U on {len(pick)} cells, {name}", flush=True)
    ctx = m.mdeos_create(precision=prec)
    worst_w = worst_u = 0.0
    try:
        sch = m.make_schedule(100, 50, (), 10, 1)
        for i, (x0, v0, Ec, K, U, W) in zip(pick, steps):
            spec = m.make_specs(w.rho[i], w.e[i], int(w.n_c[i]), w.rc[i], w.dt[i], w.seed, int(w.cell_id[i]))[0]
            h = m.mdeos_lift_from_state(ctx, spec, sch, x0, v0)
            _, Kg, Ug, Wg = m.mdeos_debug_trajectory(ctx, h, N_STEPS, int(w.N[i]), forces=False)
            m.mdeos_release(ctx, [h])
            den = np.maximum(np.abs(U), K)
            worst_w = max(worst_w, float(np.max(np.abs(Wg - W) / np.maximum(den, np.abs(W)))))
            worst_u = max(worst_u, float(np.max(np.abs(Ug - U) / den)))
    finally:
        m.mdeos_destroy(ctx)
    print(f"  {name}: max |dW| / max(|W|, |U|, K) {worst_w:.2e}, max |dU| / max(|U|, K) {worst_u:.2e}", flush=True)
    assert worst_w <= 1e-5 and worst_u <= 1e-6


@pytest.mark.parametrize("prec,name", MODES, ids=[n for _, n in MODES])
def test_full_batch_averages(sample, prec, name):
    w, cells, pick, _ = sample
    specs, sch = m.specs_from_workload(w)
    print(f"large batch of {w.n}, {name}", flush=True)
    ctx = m.mdeos_create(precision=prec)
    try:
        t0 = time.time()
        res = m.mdeos_eval_batch(ctx, specs, sch)
        wall = time.time() - t0
        kms, _ = m.mdeos_last_advance_time(ctx)
    finally:
        m.mdeos_destroy(ctx)
    print(f"  {name}: wall {wall:.2f} s, advance kernels {kms:.1f} ms", flush=True)
    bad = (res["status"] & (m.CELL_NONFINITE | m.CELL_OVERFLOW)) != 0
    assert not bad.any(), np.nonzero(bad)
    o = [(c["P"], c["P_se"], c["T"], c["T_se"], c["Ecold"]) for c in cells]
    check_stats([res[i] for i in pick], o, f"large {name}",
                [f"cell {i} rho {w.rho[i]:.3f} T {w.T[i]:.2f}" for i in pick])
