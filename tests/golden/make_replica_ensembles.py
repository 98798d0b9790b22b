"""Writes replica_ensembles.json: oracle time averages over M independent
replicas (Philox seeds 1..M) of a few fixed states.

Time averages of a chaotic trajectory are random variables (the method's
restriction, Sec. III, averages one trajectory over a window). The mean over
M replicas of the same (rho*, e*) estimates the ensemble value with an error
that shrinks as 1/sqrt(M); the replica spread is the honest error bar, since
block standard errors of one run underestimate it when the blocks are
correlated. The device path's replica mean must agree with the oracle's to
0.5 % of max(|P|, rho T) (and of T), with M large enough that three combined
standard errors of the two means stay below that bar.

Calls only the oracle. Run from the repository root:
    python tests/golden/make_replica_ensembles.py [--jobs J]
"""
import argparse
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2508_06012_amd import workloads as wl  # noqa: E402

# name, rho*, T* (input recipe e* = N_DOF T*/(2N)), n_c, rc, dt, n_steps, n_avg, rescale steps, M
# [, ensemble, gamma[, potential]]: ensemble 1 is thermostatted lifting (GJF Langevin,
# temperature updates at the rescale steps) with canonical production; potential 1 is the
# embedded-atom form (Sutton-Chen (9, 6) stand-in, densities in atoms per a^3)
STATES = [
    ("cfg1", 0.8442, 0.722, 4, 2.5, 0.005, 1000, 500, (250, 500), 64),
    ("dense-500", 1.1, 3.0, 5, 2.5, 0.004, 2000, 1000, (500, 1000), 64),
    ("dilute-500", 0.3, 1.0, 5, 2.5, 0.004, 2000, 1000, (500, 1000), 1024),
    ("multi-image-108", 1.0, 2.0, 3, 3.0, 0.004, 1500, 750, (375, 750), 256),
    ("rc4-864", 0.9, 5.0, 6, 4.0, 0.002, 1000, 500, (250, 500), 64),
    ("minimum-image-4000", 0.8, 2.0, 10, 2.5, 0.004, 1500, 750, (375, 750), 32),
    ("cfg1-nvt", 0.8442, 0.722, 4, 2.5, 0.005, 1000, 500, (250, 500), 1280, 1, 1.0),
    ("dense-500-nvt", 1.1, 3.0, 5, 2.5, 0.004, 2000, 1000, (500, 1000), 384, 1, 1.0),
    ("eam-256", 4.4, 14.0, 4, 1.5, 0.001, 1000, 500, (250, 500), 256, 0, 0.0, 1),
    ("eam-500-hot", 5.5, 30.0, 5, 1.5, 0.001, 1000, 500, (250, 500), 128, 0, 0.0, 1),
]
SEED0 = 1
CELL_ID = 0


def _job(a):
    rho, e, n_c, rc, dt, n, na, S, seed, ens, gam, pot = a
    c = oracle.Cell(rho=rho, e=e, n_c=n_c, rc=rc, dt=dt, seed=seed, cell_id=CELL_ID, potential=pot)
    r = oracle.run(c, oracle.Schedule(n, na, rescale_steps=tuple(S), ensemble=ens, gamma=gam)).result
    return r.P, r.T, r.status


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=os.cpu_count())
    ap.add_argument("--only", default=None, help="comma-separated state names")
    ap.add_argument("--out", default=os.path.join(os.path.dirname(os.path.abspath(__file__)),
                                                  "replica_ensembles.json"))
    args = ap.parse_args()
    oracle.build()
    old = {}
    if os.path.exists(args.out):
        with open(args.out) as f:
            old = {s["name"]: s for s in json.load(f)["states"]}
    only = set(args.only.split(",")) if args.only else None
    out = []
    with mp.get_context("fork").Pool(args.jobs) as pool:
        for name, rho, T, n_c, rc, dt, n, na, S, M, *extra in STATES:
            ens, gam, pot = (list(extra) + [0, 0.0, 0][len(extra):])[:3]
            if only is not None and name not in only and name in old:
                out.append(old[name])
                continue
            N = 4 * n_c ** 3
            e = float(wl.e_from_T(T, N))
            t0 = time.time()
            jobs = [(rho, e, n_c, rc, dt, n, na, S, SEED0 + k, ens, gam, pot) for k in range(M)]
            res = pool.map(_job, jobs, chunksize=1)
            P = [r[0] for r in res]
            Tm = [r[1] for r in res]
            status = [r[2] for r in res]
            print(f"{name}: M {M} in {time.time() - t0:.0f} s, P {np.mean(P):.5f} sd {np.std(P, ddof=1):.5f}, "
                  f"T {np.mean(Tm):.5f} sd {np.std(Tm, ddof=1):.5f}", flush=True)
            out.append(dict(name=name, rho=rho, T_input=T, e=e, n_c=n_c, rc=rc, dt=dt, n_steps=n, n_avg=na,
                            rescale_steps=list(S), n_blocks=10, energy_every=10, seed0=SEED0, cell_id=CELL_ID,
                            ensemble=ens, gamma=gam, potential=pot, M=M, P=P, T=Tm, status=status))
    with open(args.out, "w") as f:
        json.dump(dict(generator="tests/golden/make_replica_ensembles.py (oracle only)", states=out), f, indent=1)
        f.write("\n")


if __name__ == "__main__":
    main()
