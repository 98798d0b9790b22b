#!/usr/bin/env python3
"""Benchmark of the batched in-line MD equation of state on one MI355X.

One bench step = one EOS evaluation of every cell of the uniform workload: a
64 x 64 continuum mesh of 500-atom LJTS boxes (rho* from a smooth field in
[0.3, 1.1], T* ~ U[0.8, 3.0], rc = 2.5, dt = 0.004, 2000 velocity-Verlet
steps with energy re-pins at 500 and 1000, averages over the last 1000),
lift + advance + restrict, inputs prepared on the host. Prints one JSON line.

Beside the headline (EOS evaluations per second of the batched path) it
reports atom-steps/s, the plain path (one cell per launch, cells one after
another) on a stratified sample, the force kernel against the FP32 roofline
(algorithmic FLOPs from the measured ordered in-range pair counts, kernel time
from HIP events on the launch stream), a short serving run with p50/p99 query
latency, and the FP64 oracle timed on this host's cores on a bounded sample,
whose results are also compared with the GPU's (statistical parity).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

METRIC = "EOS evals/s + atom-steps/s; p50/p99 query latency; batched vs plain at ⟨P⟩ tol"
PEAK_FP32 = 157.3          # TFLOP/s, MI355X FP32 vector (packed) spec
PEAK_FP32_NONPACKED = 78.6  # TFLOP/s, 256 CU x 4 SIMD x 16 lanes x 2 FLOP x 2.4 GHz
FLOP_PAIR = 23             # per ordered in-range pair: force + virial
FLOP_PAIR_ENERGY = 5       # extra on energy steps


def energy_steps(s) -> int:
    n, w0 = s.n_steps, s.n_steps - s.n_avg
    return sum(1 for k in range(1, n + 1)
               if k % s.energy_every == 0 or k == n or k == w0 or k in s.rescale_steps)


def _oracle_job(args):
    import oracle
    rho, e, n_c, rc, dt, seed, cid, n_steps, n_avg, resc = args
    cell = oracle.Cell(rho=rho, e=e, n_c=n_c, rc=rc, dt=dt, seed=seed, cell_id=cid)
    r = oracle.run(cell, oracle.Schedule(n_steps, n_avg, rescale_steps=tuple(resc))).result
    return r.P, r.P_se, r.T, r.T_se, r.status


def cpu_baseline(w, idx, gpu_res, workers):
    """The oracle as it stands on a stratified sample, parallel over cells."""
    import multiprocessing as mp

    import oracle
    oracle.build()
    s = w.sched
    jobs = [(float(w.rho[i]), float(w.e[i]), int(w.n_c[i]), float(w.rc[i]), float(w.dt[i]), int(w.seed),
             int(w.cell_id[i]), s.n_steps, s.n_avg, list(s.rescale_steps)) for i in idx]
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(workers) as pool:
        out = pool.map(_oracle_job, jobs, chunksize=1)
    wall = time.perf_counter() - t0
    within_p = within_t = 0
    for k, i in enumerate(idx):
        P, Pse, T, Tse, st = out[k]
        g = gpu_res[i]
        within_p += abs(g["P"] - P) <= 3 * math.hypot(g["P_se"], Pse)
        within_t += abs(g["T"] - T) <= 3 * math.hypot(g["T_se"], Tse)
    return wall, within_p, within_t


def serve_leg(m, wl, rate: float, mesh: int, t_steps: int, seconds_cap: float):
    """A short serving run: Poisson queries from a drifting field, cold then warm."""
    ctx = m.mdeos_create()
    queries, meta = wl.cfg4_queries(rate, mesh=mesh, t_max=t_steps)
    cold, warm = meta["cold"], meta["warm"]
    m.mdeos_serve_start(ctx, m.make_schedule(cold.n_steps, cold.n_avg, cold.rescale_steps),
                        m.make_schedule(warm.n_steps, warm.n_avg, warm.rescale_steps),
                        meta["rc"], meta["dt"], wl.DEFAULT_SEED, chunk_steps=100)
    arrival = {}
    kinds = {}
    t0 = m.mdeos_serve_now(ctx)
    seen = set()
    done = []
    for q in queries:
        t_target = t0 + q.t_arrival
        while m.mdeos_serve_now(ctx) < t_target:
            time.sleep(min(0.0005, max(0.0, t_target - m.mdeos_serve_now(ctx))))
        tk = m.mdeos_serve_submit(ctx, q.cell, q.rho, q.e, q.n_c, m.mdeos_serve_now(ctx))
        arrival[tk] = m.mdeos_serve_now(ctx)
        kinds[tk] = "warm" if q.cell in seen else "cold"
        seen.add(q.cell)
        if m.mdeos_serve_now(ctx) - t0 > seconds_cap:
            break
    m.mdeos_serve_stop(ctx, drain=True)
    tickets, res, td = m.mdeos_serve_poll(ctx, 1 << 20)
    stats = m.mdeos_serve_stats_get(ctx)
    wall = m.mdeos_serve_now(ctx) - t0
    m.mdeos_destroy(ctx)
    lat = {"cold": [], "warm": []}
    for tk, t in zip(tickets, td):
        lat[kinds[int(tk)]].append(t - arrival[int(tk)])
    out = {"rate_qps": rate, "queries": int(len(tickets)), "mesh": mesh, "continuum_steps": t_steps,
           "evals_per_s": len(tickets) / wall, "atom_steps_per_s": stats["atom_steps"] / wall,
           "relifts": stats["relifts"], "failed": int((res["status"] & (1 | 8)).astype(bool).sum())}
    for k in ("cold", "warm"):
        a = np.array(lat[k])
        if a.size:
            out[f"{k}_p50_ms"] = float(np.percentile(a, 50) * 1e3)
            out[f"{k}_p99_ms"] = float(np.percentile(a, 99) * 1e3)
    allv = np.array(lat["cold"] + lat["warm"])
    out["p50_ms"] = float(np.percentile(allv, 50) * 1e3)
    out["p99_ms"] = float(np.percentile(allv, 99) * 1e3)
    return out


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--plain-sample", type=int, default=16)
    ap.add_argument("--cpu-sample", type=int, default=64)
    ap.add_argument("--cpu-workers", type=int, default=0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--serve-rate", type=float, default=10000.0)
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(boxes are independent, so several GPUs would each take a share of them); run with --gpus 1", file=sys.stderr)
        return 2

    from paper_2508_06012_amd import mdeos as m
    from paper_2508_06012_amd import workloads as wl
    try:
        import torch
        sync = torch.cuda.synchronize if torch.cuda.is_available() else (lambda: None)
    except Exception:  # torch only provides the synchronisation bracket
        sync = lambda: None  # noqa: E731

    w = wl.cfg2()
    specs, sch = m.specs_from_workload(w)
    n = w.n
    ctx = m.mdeos_create()
    print(f"# workload {w.name}: {n} cells, {int(w.N[0])} atoms, {w.sched.n_steps} steps", file=sys.stderr, flush=True)
    for i in range(args.warmup):
        m.mdeos_eval_batch(ctx, specs, sch)
        print(f"# warmup {i + 1}/{args.warmup} done", file=sys.stderr, flush=True)
    kernel_ms = []
    sync()
    t0 = time.perf_counter()
    for i in range(args.steps):
        res = m.mdeos_eval_batch(ctx, specs, sch)
        ms, nl = m.mdeos_last_advance_time(ctx)
        kernel_ms.append(ms)
        print(f"# step {i + 1}/{args.steps}: advance {ms:.1f} ms in {nl} launch(es)", file=sys.stderr, flush=True)
    sync()
    wall = time.perf_counter() - t0
    ms_per_step = wall / args.steps * 1e3
    evals = n * args.steps / wall
    atom_steps = float(w.atom_steps()) * args.steps / wall
    failed = int(((res["status"] & (1 | 8)) != 0).sum())

    # roofline of the advance kernel: algorithmic FLOPs / event-timed duration
    ne = energy_steps(w.sched)
    flops = float(np.sum(res["pairs"] * (FLOP_PAIR * w.sched.n_steps + FLOP_PAIR_ENERGY * ne)))
    k_s = float(np.mean(kernel_ms)) / 1e3
    achieved = flops / k_s / 1e12
    roof = {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP32, "unit": "TFLOP/s",
            "frac": round(achieved / PEAK_FP32, 4), "traffic": None,
            "peak_nonpacked": PEAK_FP32_NONPACKED, "frac_nonpacked": round(achieved / PEAK_FP32_NONPACKED, 4),
            "kernel_ms": round(float(np.mean(kernel_ms)), 3), "flops_per_launch": flops,
            "flop_per_pair": FLOP_PAIR, "pairs_per_atom_step": float(np.mean(res["pairs"]) / w.N[0])}

    # plain path on a stratified sample (same kernels, one cell per launch)
    idx = np.linspace(0, n - 1, args.plain_sample).astype(int)
    sub = (m.CellSpec * len(idx))(*[specs[int(i)] for i in idx])
    t1 = time.perf_counter()
    plain = m.mdeos_eval_plain(ctx, sub, sch)
    t_plain = time.perf_counter() - t1
    plain_evals = len(idx) / t_plain
    bitwise = bool(plain.tobytes() == res[idx].tobytes())
    dP = np.abs(plain["P"] - res[idx]["P"]) / np.maximum(np.hypot(plain["P_se"], res[idx]["P_se"]), 1e-300)
    m.mdeos_destroy(ctx)

    out = {
        "metric": METRIC, "value": round(evals, 3), "unit": "EOS evals/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": w.name, "cells": n, "atoms_per_cell": int(w.N[0]), "md_steps": w.sched.n_steps,
                   "avg_window": w.sched.n_avg, "rc": 2.5, "dt": 0.004, "rho": [0.3, 1.1], "T": [0.8, 3.0],
                   "precision": "fp32 pair forces; fp64 state, energy/virial reductions and re-pin"},
        "atom_steps_per_s": atom_steps,
        "failed_cells": failed,
        "plain": {"sample": int(len(idx)), "evals_per_s": round(plain_evals, 3),
                  "batched_over_plain": round(evals / plain_evals, 2), "bitwise_equal_to_batched": bitwise,
                  "max_dP_over_combined_se": float(dP.max())},
        "roofline": roof,
    }
    if not args.no_serve:
        print("# serving leg", file=sys.stderr, flush=True)
        out["serving"] = serve_leg(m, wl, args.serve_rate, mesh=32, t_steps=6, seconds_cap=30.0)
    if not args.no_cpu:
        workers = args.cpu_workers or min(16, os.cpu_count() or 1)
        cidx = np.linspace(0, n - 1, args.cpu_sample).astype(int)
        print(f"# cpu baseline: oracle on {len(cidx)} cells with {workers} processes", file=sys.stderr, flush=True)
        cwall, wp, wt = cpu_baseline(w, cidx, res, workers)
        out["cpu_baseline"] = {"value": round(len(cidx) / cwall, 4), "unit": "EOS evals/s", "cores": workers,
                               "kind": "oracle",
                               "sample": f"{len(cidx)} stratified cells of {w.name}, full 2000-step schedule, "
                                         f"{cwall:.1f} s wall, one cell per process"}
        out["parity"] = {"cells": int(len(cidx)), "P_within_3_combined_se": int(wp), "T_within_3_combined_se": int(wt)}
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
