#!/usr/bin/env python3
"""Benchmark of the batched in-line MD equation of state on one MI355X.

One bench step = one EOS evaluation of every cell of the uniform workload: a
64 x 64 continuum mesh of 500-atom LJTS boxes (rho* from a smooth field in
[0.3, 1.1], T* ~ U[0.8, 3.0], rc = 2.5, dt = 0.004, 2000 velocity-Verlet
steps with energy re-pins at 500 and 1000, averages over the last 1000),
lift + advance + restrict, inputs prepared on the host. Prints one JSON line.

Beside the headline (EOS evaluations per second of the batched path) it
reports atom-steps/s, the plain path (one cell per launch, cells one after
another) on a stratified sample, the single-cell latency of the 256-atom
case, the force kernel against the FP32 roofline (algorithmic FLOPs from the
measured ordered in-range pair counts, kernel time from HIP events on the
launch stream, HBM traffic from a committed counter summary while the kernel
sources are unchanged), a short serving run with p50/p99 query latency, and
the FP64 oracle timed on this host's cores on a bounded sample, whose results
are also compared with the GPU's (statistical parity).

Launch shapes are autotuned during the warmup steps (results do not depend
on them). --workload cfg3 / cfg5 / eam and --precision kahan run the other
batch workloads (eam: the embedded-atom form, a many-body potential with a
density walk and a force walk per step) and the Kahan accumulation mode with
the same accounting.

Profile summaries (profiles/) are written from rocprofv3 output by
--trace-summary and --pmc-summary (see each summary for its commands).
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

METRIC = "EOS evals/s + atom-steps/s; p50/p99 query latency; batched vs plain at ⟨P⟩ tol"
PEAK_FP32 = 157.3          # TFLOP/s, MI355X FP32 vector spec (256 CUs, 2.4 GHz)
FLOP_PAIR = 23             # per ordered in-range pair: force + virial
FLOP_PAIR_ENERGY = 5       # extra on energy steps
FLOP_PAIR_EAM = 48         # embedded-atom form: density walk 17 + force and virial walk 31
FLOP_PAIR_EAM_ENERGY = 7   # extra on energy steps (the pair energy)
HERE = os.path.dirname(os.path.abspath(__file__))
ADVANCE = "k_advance"      # the dominant kernel (name prefix in traces)
SERVE_LEGS = ((2000.0, 2), (10000.0, 4), (50000.0, 10))  # (queries/s, continuum steps)
PROFILE_NAME = {"cfg2": "uniform_4096x500", "cfg3": "uneven_10000", "cfg5": "large_65536x864",
                "eam": "eam_4096x500"}


def kernel_sources_sha256() -> str:
    """Hash of every source that shapes the device work (kernels, host planning, ABI)."""
    h = hashlib.sha256()
    files = sorted(glob.glob(os.path.join(HERE, "paper_2508_06012_amd", "csrc", "*")))
    files.append(os.path.join(HERE, "include", "mdeos.h"))
    for f in files:
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def traffic_from_profile(workload: str, precision: str, profiles: str = os.path.join(HERE, "profiles")):
    """HBM bytes per advance launch from the committed counter summary, or
    None if there is none or the kernel sources changed since it was taken."""
    path = os.path.join(profiles, f"{ADVANCE}_{PROFILE_NAME.get(workload, workload)}_{precision}_traffic.md")
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as f:
        for line in f:
            if ":" in line and line.startswith("- `"):
                k, v = line[3:].split("`", 1)
                vals[k] = v.split(":", 1)[1].strip().strip("`")
    if vals.get("kernel_sources_sha256") != kernel_sources_sha256():
        return None
    return float(vals["traffic_bytes_per_launch"])


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


def _cfg1_job(_):
    import oracle
    from paper_2508_06012_amd import workloads as wl
    w = wl.cfg1()
    cell = oracle.Cell(rho=float(w.rho[0]), e=float(w.e[0]), n_c=int(w.n_c[0]), rc=float(w.rc[0]),
                       dt=float(w.dt[0]), seed=int(w.seed), cell_id=int(w.cell_id[0]))
    s = w.sched
    t0 = time.perf_counter()
    oracle.run(cell, oracle.Schedule(s.n_steps, s.n_avg, rescale_steps=tuple(s.rescale_steps)))
    return time.perf_counter() - t0


def cfg1_oracle_rates(wl, workers):
    """The single 256-atom cell (1000 steps) through the oracle: on one core,
    and as one copy per core on `workers` cores at once (evals/s)."""
    import multiprocessing as mp

    import oracle
    oracle.build()
    one = _cfg1_job(0)
    with mp.get_context("fork").Pool(workers) as pool:
        t0 = time.perf_counter()
        pool.map(_cfg1_job, range(workers), chunksize=1)
        wall = time.perf_counter() - t0
    return {"one_core_s_per_eval": round(one, 4), "one_core_evals_per_s": round(1.0 / one, 4),
            "all_cores_evals_per_s": round(workers / wall, 4), "all_cores": workers}


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
    """Serving run of the cfg4 stream: Poisson queries from a drifting field
    over a mesh x mesh grid of cells, the first visit of each cell a cold lift
    of 2000 steps and later visits warm starts of 500 steps, for the first
    t_steps continuum steps (submissions stop after seconds_cap; every
    submitted query is drained). Latency = result visible to poll - arrival."""
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
    max_queued = max_active = 0
    max_resident_bytes = 0
    for i, q in enumerate(queries):
        t_target = t0 + q.t_arrival
        while m.mdeos_serve_now(ctx) < t_target:
            time.sleep(min(0.0005, max(0.0, t_target - m.mdeos_serve_now(ctx))))
        tk = m.mdeos_serve_submit(ctx, q.cell, q.rho, q.e, q.n_c, m.mdeos_serve_now(ctx))
        arrival[tk] = m.mdeos_serve_now(ctx)
        kinds[tk] = "warm" if q.cell in seen else "cold"
        seen.add(q.cell)
        if i % 512 == 0:
            st = m.mdeos_serve_stats_get(ctx)
            max_queued = max(max_queued, st["queued"])
            max_active = max(max_active, st["active"])
            max_resident_bytes = max(max_resident_bytes, st["resident_bytes"])
        if m.mdeos_serve_now(ctx) - t0 > seconds_cap:
            break
    t_submit = m.mdeos_serve_now(ctx) - t0
    m.mdeos_serve_stop(ctx, drain=True)
    tickets, res, td = m.mdeos_serve_poll(ctx, 1 << 22)
    stats = m.mdeos_serve_stats_get(ctx)
    wall = m.mdeos_serve_now(ctx) - t0
    m.mdeos_destroy(ctx)
    lat = {"cold": [], "warm": []}
    for tk, t in zip(tickets, td):
        lat[kinds[int(tk)]].append(t - arrival[int(tk)])
    out = {"rate_qps": rate, "queries": int(len(tickets)), "mesh": mesh, "continuum_steps": t_steps,
           "submit_s": round(t_submit, 3), "wall_s": round(wall, 3),
           "evals_per_s": len(tickets) / wall, "atom_steps_per_s": stats["atom_steps"] / wall,
           "cold": int(stats["cold"]), "warm": int(stats["warm"]), "relifts": int(stats["relifts"]),
           "chunks": int(stats["chunks"]), "max_queue_depth": int(max_queued), "max_in_flight": int(max_active),
           "resident_bytes": int(max(max_resident_bytes, stats["resident_bytes"])),
           "failed": int((res["status"] & (1 | 8)).astype(bool).sum())}
    for k in ("cold", "warm"):
        a = np.array(lat[k])
        if a.size:
            out[f"{k}_p50_ms"] = round(float(np.percentile(a, 50) * 1e3), 3)
            out[f"{k}_p99_ms"] = round(float(np.percentile(a, 99) * 1e3), 3)
    allv = np.array(lat["cold"] + lat["warm"])
    out["p50_ms"] = round(float(np.percentile(allv, 50) * 1e3), 3)
    out["p99_ms"] = round(float(np.percentile(allv, 99) * 1e3), 3)
    return out


def serve_leg_child(rate: float, t_steps: int) -> dict:
    """One serving leg in a child process of its own, so that a leg that
    fails is reported in the JSON line (with its exit status) instead of ending
    the whole bench."""
    import subprocess
    cmd = [sys.executable, os.path.abspath(__file__), "--serve-leg", str(rate), str(t_steps)]
    try:
        r = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    except subprocess.TimeoutExpired:
        return {"rate_qps": rate, "continuum_steps": t_steps, "error": "timed out after 300 s"}
    lines = [ln for ln in r.stdout.splitlines() if ln.startswith("{")]
    if r.returncode == 0 and lines:
        return json.loads(lines[-1])
    tail = " | ".join(ln for ln in r.stderr.strip().splitlines()[-3:] if "amdgpu.ids" not in ln)
    why = f"signal {-r.returncode}" if r.returncode < 0 else f"exit status {r.returncode}"
    return {"rate_qps": rate, "continuum_steps": t_steps, "error": f"{why}: {tail}"}


def plain_latency(m, wl):
    """Per-eval latency of the plain path (one cell per launch) for the
    serving stream's cell sizes: a fresh lift + the cold schedule (2000
    steps), and a fresh lift + the warm schedule's 500 steps."""
    _, meta = wl.cfg4_queries(1000.0, mesh=2, t_max=1)
    cold, warm = meta["cold"], meta["warm"]
    ctx = m.mdeos_create()
    out = {}
    try:
        for N, n_c in ((256, 4), (500, 5), (864, 6)):
            spec = m.make_specs(0.8, float(wl.e_from_T(1.5, N)), n_c, meta["rc"], meta["dt"], wl.DEFAULT_SEED, 0)
            for name, s in (("cold", m.make_schedule(cold.n_steps, cold.n_avg, cold.rescale_steps)),
                            ("warm_steps", m.make_schedule(warm.n_steps, warm.n_avg, ()))):
                m.mdeos_eval_plain(ctx, spec, s)
                lat = []
                for _ in range(3):
                    t1 = time.perf_counter()
                    m.mdeos_eval_plain(ctx, spec, s)
                    lat.append(time.perf_counter() - t1)
                out[f"N{N}_{name}_ms"] = round(float(np.median(lat)) * 1e3, 3)
    finally:
        m.mdeos_destroy(ctx)
    return out


# --- profile summaries (rocprofv3 output -> profiles/*.md) -------------------

def _csv_rows(d: str, suffix: str):
    rows = []
    for f in sorted(glob.glob(os.path.join(d, "**", f"*{suffix}"), recursive=True)):
        with open(f, newline="") as fh:
            rows += list(csv.DictReader(fh))
    if not rows:
        raise SystemExit(f"no *{suffix} under {d}")
    return rows


def _bench_line(path: str) -> dict:
    with open(path) as f:
        lines = [ln for ln in f if ln.startswith("{")]
    return json.loads(lines[-1])


def _short(name: str) -> str:
    n = name[5:] if name.startswith("void ") else name
    n = n.replace("mdeos::(anonymous namespace)::", "")
    return n.split("(")[0] if not n.startswith("at::") else n.split("<")[0]


def _advance_steps(items, b):
    """The advance dispatches of the timed steps, grouped per step: `items` in
    dispatch order, each (kernel name, ...); the last steps x launches-per-step."""
    nl = int(b["roofline"].get("advance_launches_per_step", 1))
    adv = [it for it in items if f"{ADVANCE}<" in it[0]]
    adv = adv[-b["steps"] * nl:]
    return [adv[i * nl:(i + 1) * nl] for i in range(b["steps"])], nl


def trace_summary(trace_dir: str, bench_json: str, cmd: str) -> str:
    """Kernel-time summary of a `rocprofv3 --kernel-trace --stats` run of bench.py."""
    b = _bench_line(bench_json)
    stats = _csv_rows(trace_dir, "kernel_stats.csv")
    trace = _csv_rows(trace_dir, "kernel_trace.csv")
    stats.sort(key=lambda r: -float(r["TotalDurationNs"]))
    top = stats[0]["Name"]
    trace.sort(key=lambda r: int(r["Start_Timestamp"]))
    items = [(_short(r["Kernel_Name"]) + "<", int(r["Start_Timestamp"]), int(r["End_Timestamp"]), r["Kernel_Name"])
             for r in trace]
    steps, nl = _advance_steps(items, b)
    span = sum(max(e for _, _, e, _ in st) - min(s0 for _, s0, _, _ in st) for st in steps) / len(steps) / 1e6
    busy = sum(sum(e - s0 for _, s0, e, _ in st) for st in steps) / len(steps) / 1e6
    kms = b["roofline"]["kernel_ms"]
    out = [f"# {_short(top)} on {b['config']['workload']} ({b['config'].get('precision_mode', 'fp64')})", "",
           "Command (from the repository root, on the GPU host):", "", "```",
           "cd /tmp && export TMPDIR=/tmp && cd -", cmd, "```", "",
           "rocprofv3 kernel statistics (all dispatches of the run, warmup and its",
           "launch-shape tuning chunks included):", "",
           "| kernel | calls | average ms | total ms | % |", "|---|---|---|---|---|"]
    for r in stats[:6]:
        out.append(f"| `{_short(r['Name'])}` | {r['Calls']} | {float(r['AverageNs']) / 1e6:.3f} | "
                   f"{float(r['TotalDurationNs']) / 1e6:.1f} | {float(r['Percentage']):.1f} |")
    if nl == 1:
        out += ["", f"Timed dispatches of the dominant kernel (the last {len(steps)}): average "
                f"**{span:.3f} ms** per launch; bench.py's HIP-event time on the launch stream: "
                f"**{kms:.3f} ms** (difference {100 * (span - kms) / kms:+.2f} %).", ""]
    else:
        out += ["", f"Each timed step launches {nl} advance kernels (one per size bucket, on concurrent "
                f"streams). Over the last {len(steps)} steps: first start to last end **{span:.3f} ms** per "
                f"step (the sum of the {nl} launch durations, which overlap, is {busy:.1f} ms); bench.py's "
                f"HIP-event time of the step: **{kms:.3f} ms** (difference {100 * (span - kms) / kms:+.2f} %).",
                "", "Launches of the last timed step:", "", "| launch shape | ms |", "|---|---|"]
        for name, s0, e, full in sorted(steps[-1], key=lambda it: -(it[2] - it[1])):
            shape = full[full.index("<") + 1:full.index(">")] if "<" in full else full
            out.append(f"| `{shape}` | {(e - s0) / 1e6:.1f} |")
        out.append("")
    out += [f"Full name of the kernel with the most time: `{top}`", "",
            f"bench line: value {b['value']} {b['unit']}, roofline achieved {b['roofline']['achieved']} "
            f"{b['roofline']['unit']} (frac {b['roofline']['frac']} of {b['roofline']['peak']}).", ""]
    return "\n".join(out)


def _counters(d: str):
    """Per-dispatch counter sums of a `rocprofv3 --pmc ... --output-format csv` run,
    in dispatch order: [(kernel name, {counter: value})]."""
    by = {}
    for r in _csv_rows(d, "counter_collection.csv"):
        e = by.setdefault(int(r["Dispatch_Id"]), [r["Kernel_Name"], {}])
        e[1][r["Counter_Name"]] = e[1].get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    return [(by[i][0], by[i][1]) for i in sorted(by)]


def pmc_summary(fetch_dir: str, write_dir: str, bench_json: str, cmds: list[str]) -> str:
    """HBM traffic of the advance launches of a step from FETCH_SIZE and
    WRITE_SIZE passes, each scaled by the same counter's reading for a plain
    device copy of known size (the last dispatch of the run)."""
    b = _bench_line(bench_json)
    copy_bytes = b["copy_calibration"]["bytes"]
    per = {}
    for key, d, cname in (("fetch", fetch_dir, "FETCH_SIZE"), ("write", write_dir, "WRITE_SIZE")):
        disp = _counters(d)
        steps, nl = _advance_steps([(_short(n) + "<", c.get(cname, 0.0)) for n, c in disp], b)
        last = [(n, c.get(cname, 0.0)) for n, c in disp if "elementwise" in n][-1]
        per[key] = {"advance_kib": sum(sum(v for _, v in st) for st in steps) / len(steps), "copy_kib": last[1],
                    "copy_kernel": _short(last[0])}
    f_fetch = copy_bytes / (per["fetch"]["copy_kib"] * 1024.0)
    f_write = copy_bytes / (per["write"]["copy_kib"] * 1024.0)
    fetch_b = per["fetch"]["advance_kib"] * 1024.0 * f_fetch
    write_b = per["write"]["advance_kib"] * 1024.0 * f_write
    traffic = fetch_b + write_b
    kms = b["roofline"]["kernel_ms"]
    algo = b["roofline"].get("state_bytes_per_launch")
    unit = "launch" if nl == 1 else f"step ({nl} launches)"
    out = [f"# HBM traffic of {ADVANCE} on {b['config']['workload']} ({b['config'].get('precision_mode', 'fp64')})",
           "", "Commands (from the repository root, on the GPU host):", "", "```",
           "cd /tmp && export TMPDIR=/tmp && cd -", *cmds, "```", "",
           f"Calibration: the last dispatch of each run is a plain device copy (`{per['fetch']['copy_kernel']}`) "
           f"of {copy_bytes} bytes read and written; factors known bytes / counter bytes: "
           f"FETCH {f_fetch:.4f}, WRITE {f_write:.4f}.", "",
           f"Per {unit}, mean of the {b['steps']} timed steps:", "",
           "| counter | KiB | calibrated bytes | GB/s at the event-timed duration |",
           "|---|---|---|---|",
           f"| FETCH_SIZE | {per['fetch']['advance_kib']:.4g} | {fetch_b:.4g} | {fetch_b / kms / 1e6:.1f} |",
           f"| WRITE_SIZE | {per['write']['advance_kib']:.4g} | {write_b:.4g} | {write_b / kms / 1e6:.1f} |",
           "", f"Kernel duration (bench.py, HIP events): {kms:.3f} ms" +
           ("." if nl == 1 else " (under counter collection the launches of a step run one after another)."),
           f"Algorithmic bytes (every atom's state read once and written once): {algo:.4g}." if algo else "",
           "", "Read by bench.py (roofline.traffic) while the kernel sources are unchanged:", "",
           f"- `traffic_bytes_per_launch`: {traffic:.6e}",
           f"- `kernel_sources_sha256`: `{kernel_sources_sha256()}`", ""]
    return "\n".join(out)


VALU_PASSES = (
    ("SQ_INSTS_VALU", "SQ_INSTS_VALU_FMA_F32", "SQ_INSTS_VALU_MUL_F32", "SQ_INSTS_VALU_ADD_F32",
     "SQ_INSTS_VALU_TRANS_F32", "SQ_INSTS_VALU_FLOPS_FP32", "SQ_THREAD_CYCLES_VALU", "SQ_BUSY_CYCLES"),
    ("SQ_ACTIVE_INST_VALU", "SQ_INSTS_LDS", "SQ_LDS_BANK_CONFLICT", "SQ_ACTIVE_INST_LDS", "SQ_WAVE_CYCLES",
     "SQ_WAVES", "SQ_INSTS_VALU_FLOPS_FP64", "SQ_INSTS_SALU"),
)


def valu_summary(dirs: list[str], bench_json: str, cmds: list[str]) -> str:
    """VALU and LDS counters of the advance launches of a step (two --pmc
    passes of VALU_PASSES), with the executed FP32 FLOP rate next to the
    algorithmic one."""
    b = _bench_line(bench_json)
    tot = {}
    nl = 1
    for d in dirs:
        disp = _counters(d)
        steps, nl = _advance_steps([(_short(n) + "<", c) for n, c in disp], b)
        for st in steps:
            for _, c in st:
                for k, v in c.items():
                    tot[k] = tot.get(k, 0.0) + v / len(steps)
    kms = b["roofline"]["kernel_ms"]
    t = kms / 1e3
    cus, clk = 256, 2.4e9
    atom_steps = b["atom_steps_per_s"] * b["ms_per_step"] / 1e3
    iv = tot["SQ_INSTS_VALU"]
    flops32 = 64.0 * tot["SQ_INSTS_VALU_FLOPS_FP32"]
    lanes = tot["SQ_THREAD_CYCLES_VALU"] / iv
    unit = "launch" if nl == 1 else f"step ({nl} launches)"
    out = [f"# VALU and LDS counters of {ADVANCE} on {b['config']['workload']} "
           f"({b['config'].get('precision_mode', 'fp64')})", "",
           "Commands (from the repository root, on the GPU host):", "", "```",
           "cd /tmp && export TMPDIR=/tmp && cd -", *cmds, "```", "",
           f"Counters summed over the advance dispatches of one {unit}, mean of the {b['steps']} timed steps "
           "(instruction counters count wave-wide instructions):", "",
           "| counter | value |", "|---|---|"]
    for k in [c for p in VALU_PASSES for c in p]:
        if k in tot:
            out.append(f"| {k} | {tot[k]:.4g} |")
    out += ["", f"Derived, with the event-timed duration {kms:.3f} ms of the bench line given (a run without "
            f"counter collection), {cus} CUs at {clk / 1e9:.1f} GHz and "
            f"{atom_steps:.4g} atom-steps per step:", "",
            f"- VALU lane-instructions per atom-step: {64 * iv / atom_steps:.0f}",
            f"- VALU wave-instructions issued per CU and clock: {iv / (cus * clk * t):.3f} (a register-only "
            "v_fma_f32 loop reaches 1.57)",
            f"- active lanes per VALU instruction (SQ_THREAD_CYCLES_VALU / SQ_INSTS_VALU): {lanes:.1f} of 64",
            f"- FP32 instructions per VALU instruction: FMA {tot['SQ_INSTS_VALU_FMA_F32'] / iv:.3f}, "
            f"MUL {tot['SQ_INSTS_VALU_MUL_F32'] / iv:.3f}, ADD {tot['SQ_INSTS_VALU_ADD_F32'] / iv:.3f}, "
            f"TRANS {tot['SQ_INSTS_VALU_TRANS_F32'] / iv:.3f}",
            f"- executed FP32 FLOP/s (64 x SQ_INSTS_VALU_FLOPS_FP32 / duration): {flops32 / t / 1e12:.2f} TFLOP/s; "
            f"weighted by the active lanes: {flops32 * lanes / 64 / t / 1e12:.2f} TFLOP/s",
            f"- algorithmic FP32 FLOP/s (bench.py: {b['roofline']['flop_per_pair']} FLOP per in-range pair): "
            f"{b['roofline']['achieved']:.2f} TFLOP/s, frac {b['roofline']['frac']} of {b['roofline']['peak']}"]
    if "SQ_INSTS_LDS" in tot:
        out += [f"- LDS instructions per atom-step (wave-wide): {tot['SQ_INSTS_LDS'] / atom_steps:.3f}; "
                f"bank-conflict cycles per LDS instruction: {tot['SQ_LDS_BANK_CONFLICT'] / tot['SQ_INSTS_LDS']:.2f}; "
                f"bank-conflict cycles per CU over the duration: "
                f"{tot['SQ_LDS_BANK_CONFLICT'] / cus / (clk * t):.2f} of each cycle"]
    out.append("")
    return "\n".join(out)


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", choices=["cfg2", "cfg3", "cfg5", "eam"], default="cfg2",
                    help="cfg2: 4096 x 500 atoms (default); cfg3: 10,000 boxes of 108..4000 atoms; "
                         "cfg5: 65,536 x 864 atoms at rc 4; eam: 4096 x 500 atoms of the embedded-atom form")
    ap.add_argument("--precision", choices=["fp64", "kahan"], default="fp64",
                    help="per-atom energy/virial accumulation")
    ap.add_argument("--no-autotune", action="store_true", help="static launch-shape model only")
    ap.add_argument("--plain-sample", type=int, default=16)
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=64)
    ap.add_argument("--cpu-workers", type=int, default=0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--serve-leg", nargs=2, type=float, metavar=("RATE", "STEPS"),
                    help="run one serving leg of the default run and print its JSON line (the default run "
                         "starts each leg as a child process of its own)")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="end with one plain device copy of this many MiB (counter calibration)")
    ap.add_argument("--trace-summary", nargs=2, metavar=("TRACE_DIR", "BENCH_LOG"),
                    help="write a markdown summary of a rocprofv3 --kernel-trace --stats run and exit")
    ap.add_argument("--pmc-summary", nargs=3, metavar=("FETCH_DIR", "WRITE_DIR", "BENCH_LOG"),
                    help="write a markdown summary of FETCH_SIZE / WRITE_SIZE runs and exit")
    ap.add_argument("--valu-summary", nargs=3, metavar=("PASS1_DIR", "PASS2_DIR", "BENCH_LOG"),
                    help="write a markdown summary of the two VALU / LDS counter passes and exit")
    ap.add_argument("--valu-pass", type=int, default=0, choices=[1, 2],
                    help="print the --pmc counter list of that VALU pass and exit")
    ap.add_argument("--cmd", action="append", default=[], help="command lines recorded in a summary")
    ap.add_argument("--out", default=None, help="summary file (default: stdout)")
    args = ap.parse_args()

    if args.valu_pass:
        print(" ".join(VALU_PASSES[args.valu_pass - 1]))
        return 0
    if args.serve_leg:
        from paper_2508_06012_amd import mdeos as m
        from paper_2508_06012_amd import workloads as wl
        rate, t_steps = args.serve_leg
        print(json.dumps(serve_leg(m, wl, rate, mesh=128, t_steps=int(t_steps), seconds_cap=25.0)), flush=True)
        return 0
    if args.trace_summary or args.pmc_summary or args.valu_summary:
        if args.trace_summary:
            text = trace_summary(*args.trace_summary, " && ".join(args.cmd))
        elif args.pmc_summary:
            text = pmc_summary(*args.pmc_summary, args.cmd)
        else:
            text = valu_summary(args.valu_summary[:2], args.valu_summary[2], args.cmd)
        if args.out:
            with open(args.out, "w") as f:
                f.write(text)
        else:
            print(text)
        return 0

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(boxes are independent, so several GPUs would each take a share of them); run with --gpus 1",
              file=sys.stderr)
        return 2

    from paper_2508_06012_amd import mdeos as m
    from paper_2508_06012_amd import workloads as wl
    try:
        import torch
        sync = torch.cuda.synchronize if torch.cuda.is_available() else (lambda: None)
    except Exception:  # torch only provides the synchronisation bracket and the calibration copy
        torch = None
        sync = lambda: None  # noqa: E731

    w = {"cfg2": wl.cfg2, "cfg3": wl.cfg3, "cfg5": wl.cfg5, "eam": wl.eam_cu}[args.workload]()
    default = args.workload == "cfg2"
    prec = m.PREC_KAHAN if args.precision == "kahan" else m.PREC_FP64
    specs, sch = m.specs_from_workload(w)
    n = w.n
    # Verlet skin and inner-list skin (< 0: the walks use the full list), the measured best of each
    # potential; 0 takes the library's per-box-size LJTS default
    skin, inner_skin = (0.5, 0.12) if w.potential == 1 else (0.0, -1.0)
    ctx = m.mdeos_create(autotune=0 if args.no_autotune else 1, precision=prec, potential=w.potential, skin=skin,
                         prune_skin=inner_skin)
    print(f"# workload {w.name}: {n} cells, {int(w.N.sum())} atoms, {w.sched.n_steps} steps, "
          f"precision {args.precision}", file=sys.stderr, flush=True)
    for i in range(args.warmup):
        m.mdeos_eval_batch(ctx, specs, sch)
        print(f"# warmup {i + 1}/{args.warmup} done", file=sys.stderr, flush=True)
    kernel_ms, launches = [], []
    sync()
    t0 = time.perf_counter()
    for i in range(args.steps):
        res = m.mdeos_eval_batch(ctx, specs, sch)
        ms, nl = m.mdeos_last_advance_time(ctx)
        kernel_ms.append(ms)
        launches.append(nl)
        print(f"# step {i + 1}/{args.steps}: advance {ms:.1f} ms in {nl} launch(es)", file=sys.stderr, flush=True)
    sync()
    wall = time.perf_counter() - t0
    ms_per_step = wall / args.steps * 1e3
    evals = n * args.steps / wall
    atom_steps = float(w.atom_steps()) * args.steps / wall
    failed = int(((res["status"] & (1 | 8)) != 0).sum())

    # roofline of the advance kernel: algorithmic FLOPs / event-timed duration
    ne = energy_steps(w.sched)
    fp, fpe = (FLOP_PAIR_EAM, FLOP_PAIR_EAM_ENERGY) if w.potential == 1 else (FLOP_PAIR, FLOP_PAIR_ENERGY)
    flops = float(np.sum(res["pairs"] * (fp * w.sched.n_steps + fpe * ne)))
    k_s = float(np.mean(kernel_ms)) / 1e3
    achieved = flops / k_s / 1e12
    traffic = traffic_from_profile(args.workload, args.precision)
    roof = {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP32, "unit": "TFLOP/s",
            "frac": round(achieved / PEAK_FP32, 4), "traffic": traffic,
            "kernel_ms": round(float(np.mean(kernel_ms)), 3), "flops_per_launch": flops,
            "advance_launches_per_step": int(max(launches)),
            "flop_per_pair": fp, "flop_per_pair_energy_step": fp + fpe,
            "pairs_per_atom_step": float(np.sum(res["pairs"]) / np.sum(w.N)),
            "state_bytes_per_launch": float(2 * 72 * np.sum(w.N))}
    if traffic is not None:
        roof["traffic_GBps"] = round(traffic / k_s / 1e9, 1)

    out = {
        "metric": METRIC, "value": round(evals, 3), "unit": "EOS evals/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": w.name, "cells": n, "atoms_per_cell": sorted(set(int(x) for x in w.N)),
                   "md_steps": w.sched.n_steps, "avg_window": w.sched.n_avg,
                   "rc": sorted(set(float(x) for x in w.rc)), "dt": float(w.dt[0]),
                   "rho": [round(float(w.rho.min()), 3), round(float(w.rho.max()), 3)],
                   "T": [round(float(w.T.min()), 3), round(float(w.T.max()), 3)],
                   "precision_mode": args.precision, "autotune": not args.no_autotune,
                   "potential": "eam (Sutton-Chen 9-6 stand-in)" if w.potential == 1 else "ljts",
                   "skin": skin if skin > 0 else "per box size: 0.3 up to 150 atoms, 0.4 up to 600 or rc > 3.5, 0.6 above", "inner_skin": inner_skin if inner_skin > 0 and args.precision == "fp64" else None,
                   "precision": "fp32 pair forces; fp64 state, energy/virial sums, reductions and re-pin"
                   if args.precision == "fp64" else
                   "fp32 pair forces; Kahan fp32 per-atom energy/virial sums; fp64 state, reductions, re-pin"},
        "atom_steps_per_s": atom_steps,
        "failed_cells": failed,
        "roofline": roof,
    }
    if default and not args.no_plain:
        # plain path on a stratified sample (same kernels, one cell per launch)
        idx = np.linspace(0, n - 1, args.plain_sample).astype(int)
        sub = (m.CellSpec * len(idx))(*[specs[int(i)] for i in idx])
        t1 = time.perf_counter()
        plain = m.mdeos_eval_plain(ctx, sub, sch)
        t_plain = time.perf_counter() - t1
        plain_evals = len(idx) / t_plain
        bitwise = bool(plain.tobytes() == res[idx].tobytes())
        dP = np.abs(plain["P"] - res[idx]["P"]) / np.maximum(np.hypot(plain["P_se"], res[idx]["P_se"]), 1e-300)
        out["plain"] = {"sample": int(len(idx)), "evals_per_s": round(plain_evals, 3),
                        "batched_over_plain": round(evals / plain_evals, 2), "bitwise_equal_to_batched": bitwise,
                        "max_dP_over_combined_se": float(dP.max())}
        # single-cell latency: the 256-atom case, one cell per call
        w1 = wl.cfg1()
        s1, q1 = m.specs_from_workload(w1)
        m.mdeos_eval_plain(ctx, s1, q1)
        lat = []
        for _ in range(5):
            t1 = time.perf_counter()
            r1 = m.mdeos_eval_plain(ctx, s1, q1)
            lat.append(time.perf_counter() - t1)
        out["cfg1"] = {"workload": w1.name, "wall_ms_per_eval": round(float(np.median(lat)) * 1e3, 3),
                       "P": float(r1["P"][0]), "P_se": float(r1["P_se"][0]), "T": float(r1["T"][0]),
                       "T_se": float(r1["T_se"][0])}
    m.mdeos_destroy(ctx)
    if default and not args.no_serve:
        # the serving stream at its full mesh, three rates, each over a prefix
        # of continuum steps (step 0 is every cell's cold lift)
        legs = []
        for rate, t_steps in SERVE_LEGS:
            print(f"# serving leg: 128 x 128 mesh, {rate:.0f} queries/s, {t_steps} continuum steps", file=sys.stderr,
                  flush=True)
            legs.append(serve_leg_child(rate, t_steps))
            print(f"#   {json.dumps(legs[-1])}", file=sys.stderr, flush=True)
        out["serving"] = {"workload": "cfg4-serving-128x128", "legs": legs, "plain_latency": plain_latency(m, wl)}
    if default and not args.no_cpu:
        affinity = len(os.sched_getaffinity(0))
        workers = args.cpu_workers or min(16, affinity)
        cidx = np.linspace(0, n - 1, args.cpu_sample).astype(int)
        print(f"# cpu baseline: oracle on {len(cidx)} cells with {workers} processes", file=sys.stderr, flush=True)
        cwall, wp, wt = cpu_baseline(w, cidx, res, workers)
        c1 = cfg1_oracle_rates(wl, workers)
        out["cpu_baseline"] = {"value": round(len(cidx) / cwall, 4), "unit": "EOS evals/s", "cores": workers,
                               "kind": "oracle",
                               "sample": f"{len(cidx)} stratified cells of {w.name}, full 2000-step schedule, "
                                         f"{cwall:.1f} s wall, one cell per process",
                               "host_cpu_count": os.cpu_count(), "affinity_cpus": affinity, "cfg1": c1}
        out["parity"] = {"cells": int(len(cidx)), "P_within_3_combined_se": int(wp), "T_within_3_combined_se": int(wt)}
    if args.copy_mib > 0:
        # a plain device copy of known size, last on the device (counter calibration)
        nbytes = args.copy_mib << 20
        a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
        bb = torch.empty_like(a)
        sync()
        torch.neg(a, out=bb)
        sync()
        out["copy_calibration"] = {"bytes": nbytes, "kernel": "torch.neg(float32)"}
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
