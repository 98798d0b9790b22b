"""Writes cfg5_sample.json: oracle results for the fixed 64-cell stratified
subsample of the large rc = 4 workload (65,536 boxes of 864 atoms,
rho* in [0.5, 1.2], T* in [1, 10], dt 0.002, 1000 steps, re-pins at 250
and 500, averages over the last 500).

For each sampled cell: <P>, its block SE, <T>, its block SE, E_cold / N and
the status, from the oracle's full run (lift, advance, restrict; Sec. III).
The device path's two accumulation modes (FP64 and Kahan-compensated FP32
per-atom sums) are compared with these values at full batch size.

Calls only the oracle. Run from the repository root:
    python tests/golden/make_cfg5_sample.py [--jobs J]
"""
import argparse
import json
import multiprocessing as mp
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2508_06012_amd import workloads as wl  # noqa: E402


def _job(a):
    rho, e, n_c, rc, dt, seed, cid, n, na, S = a
    c = oracle.Cell(rho=rho, e=e, n_c=n_c, rc=rc, dt=dt, seed=seed, cell_id=cid)
    r = oracle.run(c, oracle.Schedule(n, na, rescale_steps=tuple(S))).result
    return dict(P=r.P, P_se=r.P_se, T=r.T, T_se=r.T_se, Ecold=r.Ecold, status=r.status)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=os.cpu_count())
    ap.add_argument("--out", default=os.path.join(os.path.dirname(os.path.abspath(__file__)), "cfg5_sample.json"))
    args = ap.parse_args()
    oracle.build()
    w = wl.cfg5()
    pick = wl.stratified_sample(w)
    s = w.sched
    jobs = [(float(w.rho[i]), float(w.e[i]), int(w.n_c[i]), float(w.rc[i]), float(w.dt[i]), int(w.seed),
             int(w.cell_id[i]), s.n_steps, s.n_avg, list(s.rescale_steps)) for i in pick]
    t0 = time.time()
    with mp.get_context("fork").Pool(args.jobs) as pool:
        res = pool.map(_job, jobs, chunksize=1)
    print(f"{len(pick)} cells in {time.time() - t0:.0f} s", flush=True)
    cells = [dict(index=int(i), **r) for i, r in zip(pick, res)]
    with open(args.out, "w") as f:
        json.dump(dict(generator="tests/golden/make_cfg5_sample.py (oracle only)", workload=w.name,
                       seed=int(w.seed), cells=cells), f, indent=1)
        f.write("\n")


if __name__ == "__main__":
    main()
