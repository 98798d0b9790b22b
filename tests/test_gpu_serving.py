"""Serving loop on the GPU: continuous batching with warm starts.

Each cell's queries are served in order, the first lifted cold and later ones
warm-started from the resident state. A served result must equal, bitwise,
the same query sequence run alone through lift / warm_start / advance /
restrict: the cell's arithmetic does not depend on which other cells shared
its chunks, on chunk boundaries or on launch shapes.
"""
import time

import numpy as np
import pytest

from paper_2508_06012_amd import mdeos as m
from paper_2508_06012_amd import workloads as wl

pytestmark = pytest.mark.gpu

COLD = dict(n_steps=200, n_avg=100, rescale_steps=(50, 100))
WARM = dict(n_steps=100, n_avg=50, rescale_steps=(0, 25))
RC, DT, SEED = 2.5, 0.004, 77


def sched(d):
    return m.make_schedule(d["n_steps"], d["n_avg"], d["rescale_steps"], 10, 10, 0.5)


def queries(n_cells=6, per_cell=3, seed=1):
    rng = np.random.default_rng(seed)
    out = []
    for q in range(per_cell):
        for c in range(n_cells):
            n_c = (3, 4, 5)[c % 3]
            rho = rng.uniform(0.4, 1.0)
            T = rng.uniform(1.0, 2.5)
            out.append((c, float(rho), float(wl.e_from_T(T, 4 * n_c ** 3)), n_c))
    return out


def serve_all(ctx, qs, chunk, timeout=90.0, rc=RC, dt=DT, max_slots=0):
    m.mdeos_serve_start(ctx, sched(COLD), sched(WARM), rc, dt, SEED, chunk_steps=chunk, max_slots=max_slots)
    tickets = []
    for c, rho, e, n_c in qs:
        tickets.append(m.mdeos_serve_submit(ctx, c, rho, e, n_c, m.mdeos_serve_now(ctx)))
    got = {}
    t0 = time.time()
    while len(got) < len(qs) and time.time() - t0 < timeout:
        tk, res, td = m.mdeos_serve_poll(ctx, 1024)
        for k, r in zip(tk, res):
            got[int(k)] = r
        time.sleep(0.01)
    stats = m.mdeos_serve_stats_get(ctx)
    m.mdeos_serve_stop(ctx, drain=True)
    return tickets, got, stats


def alone(ctx, c, seq, rc=RC, dt=DT):
    """The same query sequence of one cell through the batch API."""
    out = []
    _, rho, e, n_c = seq[0]
    h = m.mdeos_lift(ctx, m.make_specs(rho, e, n_c, rc, dt, SEED, c), sched(COLD))
    m.mdeos_advance(ctx, h, 0 or 10 ** 6)
    out.append(m.mdeos_restrict(ctx, h)[0])
    for _, rho, e, n_c in seq[1:]:
        m.mdeos_warm_start(ctx, h, rho, e, sched(WARM))
        m.mdeos_advance(ctx, h, 10 ** 6)
        out.append(m.mdeos_restrict(ctx, h)[0])
    m.mdeos_release(ctx, h)
    return out


@pytest.mark.parametrize("chunk", [37, 100])
def test_served_equals_alone_bitwise(chunk):
    ctx = m.mdeos_create()
    try:
        qs = queries()
        print(f"serving {len(qs)} queries, chunk {chunk}", flush=True)
        tickets, got, stats = serve_all(ctx, qs, chunk)
        assert len(got) == len(qs), (len(got), stats)
        assert stats["cold"] == 6 and stats["warm"] == 12, stats
        for c in range(6):
            seq = [q for q in qs if q[0] == c]
            tk = [t for t, q in zip(tickets, qs) if q[0] == c]
            ref = alone(ctx, c, seq)
            for k in range(len(seq)):
                r = got[tk[k]]
                assert r["status"] & (m.CELL_NONFINITE | m.CELL_OVERFLOW) == 0
                assert r.tobytes() == ref[k].tobytes(), (c, k, r, ref[k])
    finally:
        m.mdeos_destroy(ctx)


def test_served_equals_alone_bitwise_embedded_atom():
    """The serving loop on an embedded-atom context (densities per a^3)."""
    ctx = m.mdeos_create(potential=m.POT_EAM)
    try:
        rng = np.random.default_rng(3)
        qs = []
        for q in range(3):
            for c in range(4):
                n_c = (3, 4)[c % 2]
                T = rng.uniform(7.0, 20.0)
                qs.append((c, float(rng.uniform(4.0, 5.0)), float(wl.e_from_T(T, 4 * n_c ** 3)), n_c))
        print(f"serving {len(qs)} embedded-atom queries", flush=True)
        tickets, got, stats = serve_all(ctx, qs, 50, rc=1.5, dt=0.001)
        assert len(got) == len(qs), (len(got), stats)
        for c in range(4):
            seq = [q for q in qs if q[0] == c]
            tk = [t for t, q in zip(tickets, qs) if q[0] == c]
            ref = alone(ctx, c, seq, rc=1.5, dt=0.001)
            for k in range(len(seq)):
                r = got[tk[k]]
                assert r["status"] & (m.CELL_NONFINITE | m.CELL_OVERFLOW) == 0
                assert r.tobytes() == ref[k].tobytes(), (c, k)
    finally:
        m.mdeos_destroy(ctx)


def test_hbm_budget_evicts_and_completes():
    # room for about three resident cells: the others wait or evict idle ones
    budget = 3 * m.mdeos_cell_bytes(5) + 4096
    ctx = m.mdeos_create(hbm_budget=budget)
    try:
        qs = queries(n_cells=6, per_cell=2, seed=3)
        tickets, got, stats = serve_all(ctx, qs, 50)
        assert len(got) == len(qs), stats
        assert stats["evictions"] > 0
        assert stats["resident_bytes"] <= budget
        for r in got.values():
            assert r["status"] & (m.CELL_NONFINITE | m.CELL_OVERFLOW) == 0
            assert np.isfinite(r["P"]) and np.isfinite(r["T"])
    finally:
        m.mdeos_destroy(ctx)


def test_warm_start_below_cold_relifts():
    """A warm target with no kinetic energy left above the new cold lattice
    falls back to a cold lift (and says so)."""
    ctx = m.mdeos_create()
    try:
        h = m.mdeos_lift(ctx, m.make_specs(0.9, 3.0, 4, RC, DT, SEED, 5), sched(COLD))
        m.mdeos_advance(ctx, h, 10 ** 6)
        # hot disordered state, then ask for almost no energy above the cold lattice
        m.mdeos_warm_start(ctx, h, 0.9, 1e-6, sched(WARM))
        m.mdeos_advance(ctx, h, 10 ** 6)
        r = m.mdeos_restrict(ctx, h)[0]
        assert r["status"] & m.CELL_COLD_RELIFT
        assert np.isfinite(r["P"])
        m.mdeos_release(ctx, h)
    finally:
        m.mdeos_destroy(ctx)


def test_staggered_arrivals_equal_alone_bitwise():
    """Continuous batching proper: queries arrive one by one while chunks of
    earlier queries run on the device. Each submission records whether cells
    were in flight at that moment; most must have been. Every result is
    bitwise equal to the cell's query sequence run alone."""
    ctx = m.mdeos_create()
    try:
        qs = queries(n_cells=8, per_cell=3, seed=7)
        rng = np.random.default_rng(2)
        print(f"staggered serving of {len(qs)} queries", flush=True)
        m.mdeos_serve_start(ctx, sched(COLD), sched(WARM), RC, DT, SEED, chunk_steps=25)
        tickets, busy, got = [], 0, {}
        for c, rho, e, n_c in qs:
            busy += 1 if m.mdeos_serve_stats_get(ctx)["active"] > 0 else 0
            tickets.append(m.mdeos_serve_submit(ctx, c, rho, e, n_c, m.mdeos_serve_now(ctx)))
            time.sleep(float(rng.uniform(0.0, 0.004)))
            tk, res, _ = m.mdeos_serve_poll(ctx, 1024)
            got.update({int(k): r for k, r in zip(tk, res)})
        t0 = time.time()
        while len(got) < len(qs) and time.time() - t0 < 90.0:
            tk, res, _ = m.mdeos_serve_poll(ctx, 1024)
            got.update({int(k): r for k, r in zip(tk, res)})
            time.sleep(0.01)
        stats = m.mdeos_serve_stats_get(ctx)
        m.mdeos_serve_stop(ctx, drain=True)
        print(f"  submitted while cells were in flight: {busy} of {len(qs)}; chunks {stats['chunks']}", flush=True)
        assert len(got) == len(qs), (len(got), stats)
        assert busy >= len(qs) // 2, busy
        for c in range(8):
            seq = [q for q in qs if q[0] == c]
            tk = [t for t, q in zip(tickets, qs) if q[0] == c]
            ref = alone(ctx, c, seq)
            for k in range(len(seq)):
                r = got[tk[k]]
                assert r["status"] & (m.CELL_NONFINITE | m.CELL_OVERFLOW) == 0
                assert r.tobytes() == ref[k].tobytes(), (c, k)
    finally:
        m.mdeos_destroy(ctx)


def test_restart_releases_the_last_sessions_resident_cells():
    """A stopped session leaves its cells resident; the next start releases
    them. With room for about three resident cells, a second session of the
    same three-cell query set completes (it would wait for capacity forever if
    the first session's cells still held the budget) and gives the same bits."""
    budget = 3 * m.mdeos_cell_bytes(5) + 4096
    ctx = m.mdeos_create(hbm_budget=budget)
    try:
        qs = queries(n_cells=3, per_cell=2, seed=5)
        t1, got1, st1 = serve_all(ctx, qs, 50, timeout=60.0)
        assert len(got1) == len(qs), st1
        t2, got2, st2 = serve_all(ctx, qs, 50, timeout=60.0)
        assert len(got2) == len(qs), st2
        for a, b in zip(t1, t2):
            assert got1[a].tobytes() == got2[b].tobytes()
    finally:
        m.mdeos_destroy(ctx)


def test_stop_without_drain_while_chunks_run():
    """Stopping without draining while chunks run on the device: the
    queries not yet admitted are dropped, the admitted ones finish, and every
    delivered result is bitwise that of its cell's query prefix run alone."""
    ctx = m.mdeos_create()
    try:
        qs = queries(n_cells=8, per_cell=3, seed=9)
        m.mdeos_serve_start(ctx, sched(COLD), sched(WARM), RC, DT, SEED, chunk_steps=25)
        tickets = [m.mdeos_serve_submit(ctx, c, rho, e, n_c, m.mdeos_serve_now(ctx)) for c, rho, e, n_c in qs]
        t0 = time.time()
        while m.mdeos_serve_stats_get(ctx)["chunks"] < 3 and time.time() - t0 < 30.0:
            time.sleep(0.002)
        m.mdeos_serve_stop(ctx, drain=False)
        stats = m.mdeos_serve_stats_get(ctx)
        tk, res, _ = m.mdeos_serve_poll(ctx, 1024)
        got = {int(k): r for k, r in zip(tk, res)}
        print(f"  delivered {len(got)} of {len(qs)} after {stats['chunks']} chunks", flush=True)
        assert stats["active"] == 0
        assert 0 < len(got) <= len(qs)
        assert set(got) <= set(tickets)
        for c in range(8):
            seq = [q for q in qs if q[0] == c]
            tk_c = [t for t, q in zip(tickets, qs) if q[0] == c]
            done = [t in got for t in tk_c]
            k = sum(done)
            assert done == [True] * k + [False] * (len(seq) - k), (c, done)  # a cell's queries run in order
            if k == 0:
                continue
            ref = alone(ctx, c, seq[:k])
            for j in range(k):
                r = got[tk_c[j]]
                assert r["status"] & (m.CELL_NONFINITE | m.CELL_OVERFLOW) == 0
                assert r.tobytes() == ref[j].tobytes(), (c, j)
    finally:
        m.mdeos_destroy(ctx)


def test_slot_cap_limits_cells_per_chunk():
    """With at most two cells advancing at once, six cells of one cold
    (200-step) and one warm (100-step) query each need 36 cell-chunks of 50
    steps, so at least 18 chunks; every result is bitwise that of the cell
    alone."""
    ctx = m.mdeos_create()
    try:
        qs = queries(n_cells=6, per_cell=2, seed=11)
        tickets, got, stats = serve_all(ctx, qs, 50, max_slots=2)
        print(f"  slot cap 2: {stats['chunks']} chunks", flush=True)
        assert len(got) == len(qs), stats
        assert stats["chunks"] >= 18, stats
        for c in range(6):
            seq = [q for q in qs if q[0] == c]
            tk = [t for t, q in zip(tickets, qs) if q[0] == c]
            ref = alone(ctx, c, seq)
            for k in range(len(seq)):
                assert got[tk[k]].tobytes() == ref[k].tobytes(), (c, k)
    finally:
        m.mdeos_destroy(ctx)


def test_cfg4_stream_served_equal_alone_on_sampled_cells():
    """The serving stream at its full mesh (128 x 128 cells of 256, 500 or
    864 atoms; cold lifts of 2000 steps, then warm starts of 500) for two
    continuum steps, submitted at 50,000 queries/s, above what the device
    sustains, so tens of thousands of queries mix in the chunks. Eight
    sampled cells, run alone through lift / advance / warm start / restrict,
    give the same bits as served."""
    queries, meta = wl.cfg4_queries(50_000.0, mesh=128, t_max=2)
    cold, warm = meta["cold"], meta["warm"]
    sc = m.make_schedule(cold.n_steps, cold.n_avg, cold.rescale_steps)
    sw = m.make_schedule(warm.n_steps, warm.n_avg, warm.rescale_steps)
    rc, dt, seed = meta["rc"], meta["dt"], wl.DEFAULT_SEED
    ctx = m.mdeos_create()
    try:
        print(f"cfg4 stream: {len(queries)} queries", flush=True)
        m.mdeos_serve_start(ctx, sc, sw, rc, dt, seed, chunk_steps=100)
        t0 = m.mdeos_serve_now(ctx)
        ticket_of = {}
        for q in queries:
            while m.mdeos_serve_now(ctx) - t0 < q.t_arrival:
                time.sleep(0.0002)
            ticket_of[(q.cell, q.step)] = m.mdeos_serve_submit(ctx, q.cell, q.rho, q.e, q.n_c, m.mdeos_serve_now(ctx))
        m.mdeos_serve_stop(ctx, drain=True)
        tk, res, _ = m.mdeos_serve_poll(ctx, 1 << 16)
        stats = m.mdeos_serve_stats_get(ctx)
        got = {int(k): r for k, r in zip(tk, res)}
        print(f"  served {len(got)} in {stats['chunks']} chunks", flush=True)
        assert len(got) == len(queries)
        assert not any(r["status"] & (m.CELL_NONFINITE | m.CELL_OVERFLOW) for r in got.values())
        sizes = meta["sizes"]
        pick = [int(np.nonzero(sizes == n)[0][j]) for n in (256, 500, 864) for j in (0, 7, 31)][:8]
        by_cell = {}
        for q in queries:
            by_cell.setdefault(q.cell, []).append(q)
        for c in pick:
            seq = sorted(by_cell[c], key=lambda q: q.step)
            h = m.mdeos_lift(ctx, m.make_specs(seq[0].rho, seq[0].e, seq[0].n_c, rc, dt, seed, c), sc)
            m.mdeos_advance(ctx, h, 10 ** 6)
            ref = [m.mdeos_restrict(ctx, h)[0]]
            for q in seq[1:]:
                m.mdeos_warm_start(ctx, h, q.rho, q.e, sw)
                m.mdeos_advance(ctx, h, 10 ** 6)
                ref.append(m.mdeos_restrict(ctx, h)[0])
            m.mdeos_release(ctx, h)
            for q, r in zip(seq, ref):
                assert got[ticket_of[(c, q.step)]].tobytes() == r.tobytes(), (c, q.step)
    finally:
        m.mdeos_destroy(ctx)
