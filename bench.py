#!/usr/bin/env python3
"""Benchmark of the superstep engine on one MI355X.

Workload: Bellman-Ford SSSP to convergence from vertex 0 on a seeded R-MAT
graph, scale 22 (4,194,304 vertices, 67,108,864 raw edges, a=0.57 b=0.19
c=0.19 d=0.05, seed 2, self-loops and duplicates removed), uint32 weights
uniform in [1, 255].  One step = one full solve: state init, all supersteps
(frontier compaction, tiled relaxation, apply) until no vertex changes, and
the final sync-set extraction.  The graph is resident in HBM before timing.

Prints one JSON line.  `value` is GTEPS = messages generated (out-edges of
the active frontier, summed over supersteps) / wall time.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s
VALU_INT32_PEAK_OPS = 256 * 64 * 2.4e9  # 256 CUs x 64 lanes x 2.4 GHz


def log(msg):
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def push_bytes_per_superstep(g, fronts):
    """Algorithmic bytes of the relaxation kernel per superstep: 8 B per
    active out-edge (destination + weight), 16 B per active-list entry, 4 B
    per distinct destination read, 4 B per vertex that improves (lower
    bracket); the upper bracket reads 4 B of destination value per edge
    instead of per distinct destination."""
    import numpy as np
    deg = np.diff(g.row_ptr).astype(np.int64)
    out = []
    for k in range(len(fronts) - 1):
        f = np.nonzero(fronts[k])[0]
        f = f[deg[f] > 0]
        ef = int(deg[f].sum())
        if len(f):
            starts = g.row_ptr[f].astype(np.int64)
            idx = np.repeat(starts - np.cumsum(np.r_[0, deg[f][:-1]]), deg[f]) + np.arange(ef)
            mark = np.zeros(g.V, bool)
            mark[g.col[idx]] = True
            nf = int(mark.sum())
        else:
            nf = 0
        ch = int(fronts[k + 1].sum())
        out.append(dict(edges=ef, list=len(f), dests=nf, changed=ch,
                        bytes=8 * ef + 16 * len(f) + 4 * nf + 4 * ch,
                        bytes_upper=12 * ef + 16 * len(f) + 4 * ch))
    return out


def copy_ceiling_gbps(torch, nbytes=1 << 30, reps=5):
    """Device-to-device copy rate (bytes read + bytes written per second):
    the practical HBM ceiling next to the 8 TB/s peak."""
    a = torch.empty(nbytes, dtype=torch.uint8, device="cuda:0")
    b = torch.empty_like(a)
    a.fill_(1)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    return 2 * nbytes / (ms / 1e3) / 1e9


def cpu_baseline(np, g, edges_per_solve, g4=None, src4=None, part=None, budget_s=20.0):
    """The oracle timed on this host: the headline SSSP solve on one thread
    (the reference mode) and on all threads (the OpenMP timing mode), with
    Dijkstra on one thread for scale; the batched workload's 256 sources as
    independent reference runs parallel over sources, and as 256 Dijkstra
    runs; the partition's PageRank (two supersteps, scaled to 30) and CC on
    all threads.  Results are checked against each other."""
    import oracle
    nthr = oracle.max_threads()

    def timed(f, min_runs=1, max_runs=5, budget=budget_s):
        times, r = [], None
        t_all = time.perf_counter()
        while len(times) < max_runs:
            t0 = time.perf_counter()
            r = f()
            times.append(time.perf_counter() - t0)
            if len(times) >= min_runs and time.perf_counter() - t_all > budget:
                break
        times.sort()
        return times[len(times) // 2], len(times), r

    t1, n1, r1 = timed(lambda: oracle.sssp(g, 0), budget=budget_s / 2)
    assert int(r1.msgs.sum()) == edges_per_solve
    tn, nn, rn = timed(lambda: oracle.sssp(g, 0, threads=0), budget=budget_s / 2)
    assert np.array_equal(rn.state, r1.state) and rn.K == r1.K
    t0 = time.perf_counter()
    dist = oracle.dijkstra(g, 0)  # the work-efficient sequential solve, for scale
    t_dij = time.perf_counter() - t0
    assert (dist == r1.state).all()
    out = {"value": edges_per_solve / tn / 1e9, "unit": "GTEPS", "cores": nthr, "kind": "oracle",
           "sample": f"full single-source solve from vertex 0 ({r1.K} supersteps, {edges_per_solve} messages): "
                     f"OpenMP timing mode on {nthr} threads, median of {nn} runs ({tn:.3f} s each)",
           "single_core": {"value": edges_per_solve / t1 / 1e9, "unit": "GTEPS", "cores": 1,
                           "sample": f"reference mode, median of {n1} runs ({t1:.2f} s each)"},
           "dijkstra_single_core_s": t_dij,
           "host_cpu": host_cpu_model(), "host_nproc": os.cpu_count()}
    if g4 is not None:
        t0 = time.perf_counter()
        D, K = oracle.sssp_many(g4, src4)
        t_bf = time.perf_counter() - t0
        t0 = time.perf_counter()
        J = oracle.dijkstra_many(g4, src4)
        t_dj = time.perf_counter() - t0
        assert np.array_equal(D, J)
        out["batched"] = {"workload": f"the batched workload's {len(src4)} sources on R-MAT scale 20",
                          "cores": nthr,
                          "bellman_ford_parallel_over_sources_s": t_bf, "queries_per_s": len(src4) / t_bf,
                          "dijkstra_parallel_over_sources_s": t_dj, "dijkstra_queries_per_s": len(src4) / t_dj}
    if part is not None:
        t0 = time.perf_counter()
        oracle.pagerank(part, 2, 0.85, threads=0)
        t_pr2 = time.perf_counter() - t0
        t0 = time.perf_counter()
        rc = oracle.cc(part, threads=0)
        t_cc = time.perf_counter() - t0
        out["partition"] = {"workload": "the scale-25 partition (part 0 of 8)", "cores": nthr,
                            "pagerank_30_s_estimated": t_pr2 * 15, "pagerank_sample": "2 supersteps, times 15",
                            "pagerank_gteps": 2 * part.E / t_pr2 / 1e9,
                            "cc_s": t_cc, "cc_supersteps": int(rc.K),
                            "cc_gteps": float(rc.msgs.sum()) / t_cc / 1e9}
    return out


def batched_bytes_per_superstep(np, g, fronts, B):
    """Algorithmic bytes of the batched SSSP kernel per superstep, from the
    union F_k over lanes of the active vertices: lower bracket 8 E_F (edges
    once) + 4 B |F| (snapshot lanes) + 8 B |N(F)| (destination lanes read
    and written) + B/8 (|F| + |N(F)|) (lane masks); upper bracket 8 B per
    lane message (a value gather and a min update per lane and edge)."""
    deg = np.diff(g.row_ptr).astype(np.int64)
    lo = up = 0
    for f in fronts:
        f = np.nonzero(f)[0]
        f = f[deg[f] > 0]
        ef = int(deg[f].sum())
        if len(f):
            starts = g.row_ptr[f].astype(np.int64)
            idx = np.repeat(starts - np.cumsum(np.r_[0, deg[f][:-1]]), deg[f]) + np.arange(ef)
            nf = int(np.unique(g.col[idx]).size)
        else:
            nf = 0
        lo += 8 * ef + 4 * B * len(f) + 8 * B * nf + (B // 8) * (len(f) + nf)
    return lo


def bench_batched(gx, torch, np, gen, steps=3):
    """256 seeded sources on R-MAT scale 20 (seed 4): one persistent batched
    launch (autotuned) against 256 sequential plain solves on the same GPU;
    every lane is compared with its plain solve."""
    import paper_2203_13005_amd as m
    g = gen.rmat(20, seed=4)
    src = gen.pick_sources(g, 256, seed=40)
    dg = gx.DeviceGraph(g, gx.GX_NEED_OUT | gx.GX_NEED_IN)
    log(f"batched: V={g.V} E={g.E}, autotuning over block/tile/width")
    best, best_ms = gx.batch_autotune(dg, gx.GX_SSSP, src)
    log(f"batched: best {best} at {best_ms:.2f} ms")
    out = torch.empty((g.V, 256), dtype=torch.int32, device="cuda:0")
    gx.batch_run(dg, gx.GX_SSSP, src, tune=best, out=out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        _, rs = gx.batch_run(dg, gx.GX_SSSP, src, tune=best, out=out)
    torch.cuda.synchronize()
    t_batch = (time.perf_counter() - t0) / steps
    # plain: 256 sequential solves, one state re-initialised per source
    st = m.State(dg, gx.GX_SSSP, source=int(src[0]))
    st.run(100_000)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plain_edges = 0
    for s_ in src:
        st.params.source = int(s_)
        st.reset()
        rsp, _ = st.run(100_000)
        plain_edges += rsp.edges
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    # untimed: every lane against its plain solve, superstep by superstep,
    # collecting the union over lanes of each superstep's active set
    union = [torch.zeros(g.V, dtype=torch.bool, device="cuda:0") for _ in range(rs.supersteps)]
    for b, s_ in enumerate(src):
        st.params.source = int(s_)
        st.reset()
        union[0][int(s_)] = True
        k = 0
        while True:
            fr, ef, ch = st.superstep(stats=True)
            if ch == 0:
                break
            k += 1
            union[k] |= st.frontier_device() != 0
        assert torch.equal(st.values(), out[:, b]), f"lane {b} differs from its plain solve"
    fronts = [u.cpu().numpy() for u in union]
    bytes_lo = batched_bytes_per_superstep(np, g, fronts, 256)
    bytes_up = 8 * plain_edges
    log(f"batched: {t_batch * 1e3:.2f} ms for 256 lanes ({rs.supersteps} supersteps); "
        f"256 plain solves {t_plain * 1e3:.1f} ms; all 256 lanes equal their plain solves")
    return {"workload": "256 seeded sources (seed 40, out-degree > 0), Bellman-Ford SSSP, R-MAT scale 20 "
                        f"({g.V} vertices, {g.E} edges after dedup, seed 4), uint32 weights in [1,255]",
            "queries_per_s": 256 / t_batch, "ms_per_batch": t_batch * 1e3, "supersteps": int(rs.supersteps),
            "plain_queries_per_s": 256 / t_plain, "plain_ms_total": t_plain * 1e3,
            "speedup_vs_plain": t_plain / t_batch, "lane_messages_per_batch": int(plain_edges),
            "lane_gteps": plain_edges / t_batch / 1e9, "lanes_checked_against_plain": 256,
            # lower bracket: compulsory bytes of the union frontiers; upper bracket: a 4 B value
            # gather and a 4 B min update per lane message; VALU: an add and a min per lane
            # message against 256 CUs x 64 lanes x 2.4 GHz int32 ops
            "roofline": {"bound": "hbm",
                         "algorithmic_bytes_lower": bytes_lo, "algorithmic_bytes_upper": bytes_up,
                         "hbm_lower_GBps": bytes_lo / t_batch / 1e9,
                         "hbm_lower_frac": bytes_lo / t_batch / 1e9 / HBM_PEAK_GBS,
                         "hbm_upper_GBps": bytes_up / t_batch / 1e9,
                         "hbm_upper_frac": bytes_up / t_batch / 1e9 / HBM_PEAK_GBS,
                         "valu_Tops": 2 * plain_edges / t_batch / 1e12,
                         "valu_frac": 2 * plain_edges / t_batch / VALU_INT32_PEAK_OPS,
                         "binds": "memory (random lane-row gathers); VALU far from its peak"},
            "tune": {"block": best.block, "tile": best.tile, "width": best.width},
            "ppr": bench_batched_ppr(gx, torch, g, dg, src)}, g, src


def bench_batched_ppr(gx, torch, g, dg, src, iters=50, reps=3):
    """Personalised PageRank lanes (50 iterations) on the same graph: 64 and
    256 seeds in one persistent launch each."""
    out = {}
    for B in (64, 256):
        seeds = src[:B]
        gx.batch_run(dg, gx.GX_PPR, seeds, iters=iters)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            gx.batch_run(dg, gx.GX_PPR, seeds, iters=iters)
        torch.cuda.synchronize()
        t = (time.perf_counter() - t0) / reps
        log(f"batched PPR: {B} lanes x {iters} iterations in {t * 1e3:.2f} ms "
            f"({t * 1e6 / iters:.1f} us per superstep)")
        out[f"lanes_{B}"] = {"ms_per_batch": t * 1e3, "us_per_superstep": t * 1e6 / iters,
                             "queries_per_s": B / t, "lane_edge_gathers_per_s": B * g.E * iters / t}
    return out


def bench_serving(gx, torch, np, gen, n_queries=10000, qps_frac=0.7, lanes=64, max_pools=4, budget_frac=0.5,
                  sample=16, outstanding=512, records=None, epoch=4):
    """16 resident R-MAT graphs (scales 16..22, seeds 100..115), 50% SSSP /
    50% PPR (50 iterations), Poisson arrivals (seed 5) at a fixed rate of
    qps_frac x the capacity measured closed-loop with `outstanding` queries
    in flight.  The HBM budget holds
    budget_frac of the lane pools of every (graph, algorithm) pair, so
    admission binds: pools are created, evicted when idle and empty, and
    queries wait for room.  After the timed run a seeded sample of the
    completed queries is checked: SSSP against the plain engine's solve from
    the same source, PPR against the same seed run alone in the batched
    engine (bitwise)."""
    import ctypes
    graphs, dgs = [], []
    t0 = time.perf_counter()
    for i in range(16):
        sc = 16 + (7 * i) // 16
        g = gen.rmat(sc, seed=100 + i)
        graphs.append(g)
        dgs.append(gx.DeviceGraph(g, gx.GX_NEED_OUT | gx.GX_NEED_IN))
    log(f"serving: 16 graphs ({sum(g.E for g in graphs)} edges) generated and loaded in "
        f"{time.perf_counter() - t0:.1f}s")
    pools = 0
    for dg in dgs:
        for algo in (gx.GX_SSSP, gx.GX_PPR):
            b = ctypes.c_size_t()
            assert gx.binding.lib.gx_server_bytes_per_lane(dg.handle, algo, ctypes.byref(b)) == 0
            pools += lanes * b.value
    budget = int(budget_frac * pools)
    rng = np.random.default_rng(5)
    cands = [np.nonzero(np.diff(g.row_ptr) > 0)[0] for g in graphs]

    def make(n):
        qs = []
        for i in range(n):
            gi = int(rng.integers(0, 16))
            qs.append((gi, gx.GX_SSSP if rng.random() < 0.5 else gx.GX_PPR, int(rng.choice(cands[gi]))))
        return qs

    def run(qs, arrivals, keep=()):
        srv = gx.Server(budget, lanes_per_pool=lanes, max_pools=max_pools, epoch_supersteps=epoch, ppr_iters=50)
        ids = [srv.add_graph(d) for d in dgs]
        done, qid_of, kept = [], {}, {}
        t_start = time.perf_counter()
        i = 0
        while len(done) < len(qs):
            now = time.perf_counter() - t_start
            while i < len(qs) and arrivals[i] <= now:
                gi, algo, s_ = qs[i]
                qid_of[srv.submit(ids[gi], algo, s_)] = i
                i += 1
            for c in srv.poll(wait_ms=0 if i < len(qs) else 20):
                assert c.status == 0
                done.append(c)
                if qid_of[c.id] in keep:
                    kept[qid_of[c.id]] = c.result
            if i < len(qs):
                time.sleep(max(0.0, min(0.002, arrivals[i] - (time.perf_counter() - t_start))))
        wall = time.perf_counter() - t_start
        srv.close()
        return done, wall, kept

    def run_closed(qs, outstanding):
        # a fixed number of queries in flight: each completion submits the next
        srv = gx.Server(budget, lanes_per_pool=lanes, max_pools=max_pools, epoch_supersteps=epoch, ppr_iters=50)
        ids = [srv.add_graph(d) for d in dgs]
        t_start = time.perf_counter()
        i = n_done = 0
        while n_done < len(qs):
            while i < len(qs) and i - n_done < outstanding:
                gi, algo, s_ = qs[i]
                srv.submit(ids[gi], algo, s_)
                i += 1
            for c in srv.poll(wait_ms=20):
                assert c.status == 0
                n_done += 1
        wall = time.perf_counter() - t_start
        srv.close()
        return wall

    cap_q = make(2048)
    capacity = len(cap_q) / run_closed(cap_q, outstanding)
    log(f"serving: closed-loop capacity {capacity:.1f} queries/s with {outstanding} in flight (budget "
        f"{budget / 2**30:.1f} GiB of {pools / 2**30:.1f} GiB for every pool)")
    qps = qps_frac * capacity
    qs = make(n_queries)
    arrivals = np.cumsum(np.random.default_rng(5).exponential(1.0 / qps, n_queries))
    check_rng = np.random.default_rng(6)
    keep = set(int(x) for x in check_rng.choice(n_queries, sample, replace=False))
    done, wall, kept = run(qs, arrivals, keep)
    if records is not None:  # per-query (graph, algorithm, submit, start, done, supersteps)
        records.extend((c.graph, c.algo, c.submit_s, c.start_s, c.done_s, c.supersteps) for c in done)
    lat = np.array([c.done_s - c.submit_s for c in done])
    wait = np.array([c.start_s - c.submit_s for c in done])
    by_algo = {}
    for name, code in (("sssp", gx.GX_SSSP), ("ppr", gx.GX_PPR)):
        la = np.array([c.done_s - c.submit_s for c in done if c.algo == code])
        if len(la):
            by_algo[name] = {"queries": int(len(la)), "p50_ms": float(np.percentile(la, 50) * 1e3),
                             "p99_ms": float(np.percentile(la, 99) * 1e3)}
    log(f"serving: {len(done)} queries at {qps:.1f} q/s offered -> {len(done) / wall:.1f} q/s, "
        f"p50 {np.percentile(lat, 50) * 1e3:.1f} ms p99 {np.percentile(lat, 99) * 1e3:.1f} ms "
        f"(admission wait p50 {np.percentile(wait, 50) * 1e3:.1f} ms); {by_algo}")
    # the seeded sample, checked outside the timed run
    for i in sorted(kept):
        gi, algo, s_ = qs[i]
        if algo == gx.GX_SSSP:
            st = gx.State(dgs[gi], gx.GX_SSSP, source=s_)
            st.run(100_000)
            assert np.array_equal(st.values_numpy(), kept[i]), f"served SSSP query {i} differs from the plain solve"
            st.close()
        else:
            alone, _ = gx.batch_run(dgs[gi], gx.GX_PPR, np.array([s_], np.int32), iters=50)
            assert np.array_equal(alone.cpu().numpy()[:, 0].view(np.uint32), kept[i].view(np.uint32)), \
                f"served PPR query {i} differs from the same seed alone"
    log(f"serving: {len(kept)} sampled queries equal their plain / alone results")
    return {"workload": "16 resident R-MAT graphs, scales 16..22 (scale 16 + floor(7i/16), seeds 100..115, "
                        "edge factor 16), queries 50% SSSP / 50% personalised PageRank (50 iterations), "
                        "Poisson arrivals (seed 5)",
            "queries": len(done), "offered_qps": qps, "closed_loop_capacity_qps": capacity,
            "closed_loop_outstanding": outstanding,
            "queries_per_s": len(done) / wall, "p50_ms": float(np.percentile(lat, 50) * 1e3),
            "p99_ms": float(np.percentile(lat, 99) * 1e3),
            "admission_wait_p50_ms": float(np.percentile(wait, 50) * 1e3), "by_algorithm": by_algo,
            "hbm_budget_gib": budget / 2**30, "all_pools_gib": pools / 2**30, "lanes_per_pool": lanes,
            "max_pools": max_pools, "sample_checked": len(kept)}


def bench_pagerank_small(gx, torch, np, gen, reps=20):
    """PageRank, 20 supersteps, d = 0.85, R-MAT scale 14 (seed 1)."""
    g = gen.rmat(14, seed=1)
    dg = gx.DeviceGraph(g, gx.GX_NEED_IN)
    st = gx.State(dg, gx.GX_PAGERANK, damping=0.85, timing=True)
    st.run(20)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    kern = 0.0
    for _ in range(reps):
        st.reset()
        rs, _ = st.run(20)
        kern += rs.edge_kernel_ms
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    # without timing events a run is one replay of a captured HIP graph
    sg = gx.State(dg, gx.GX_PAGERANK, damping=0.85)
    sg.run(20)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        sg.reset()
        sg.run(20)
    torch.cuda.synchronize()
    dg_t = (time.perf_counter() - t0) / reps
    assert np.array_equal(sg.values_numpy().view(np.uint32), st.values_numpy().view(np.uint32))
    log(f"PageRank scale 14: {dt * 1e6 / 20:.1f} us per superstep with timing events, "
        f"{dg_t * 1e6 / 20:.1f} us replayed as a graph (kernels {kern * 1e3 / reps / 20:.1f} us)")
    return {"workload": f"PageRank 20 supersteps, d=0.85, R-MAT scale 14 ({g.V} vertices, {g.E} edges, seed 1)",
            "ms_per_run": dg_t * 1e3, "us_per_superstep": dg_t * 1e6 / 20, "gteps": 20 * g.E / dg_t / 1e9,
            "what": "wall time per run (state reset included), the 20 supersteps replayed as one captured HIP "
                    "graph; the same run with a timing event pair per superstep, enqueued one by one, beside it",
            "us_per_superstep_with_timing_events": dt * 1e6 / 20,
            "pull_kernel_us_per_superstep": kern * 1e3 / reps / 20}


def bench_exchange(gx, torch, np, gen, scale=22, nparts=8, reps=3):
    """All parts of an 8-way hash vertex-cut of R-MAT scale 22 (seed 2)
    resident on the GPU: SSSP from vertex 0 superstep by superstep, every part
    emitting its sync set and merging the other parts' pairs; checked against
    the plain solve of the whole graph."""
    t0 = time.perf_counter()
    parts = [gen.rmat_part(scale, seed=2, part=p) for p in range(nparts)]
    log(f"exchange: {nparts} parts of R-MAT scale {scale} generated in {time.perf_counter() - t0:.1f}s")
    dgs = [gx.DeviceGraph(p, gx.GX_NEED_OUT) for p in parts]

    def solve():
        states = []
        for p, dg in zip(parts, dgs):
            loc = int(np.searchsorted(p.l2g, 0))
            src = loc if loc < p.V and p.l2g[loc] == 0 else -1
            states.append(gx.State(dg, gx.GX_SSSP, source=src, delta_mode=gx.GX_DELTA_ALL))
        torch.cuda.synchronize()
        t = time.perf_counter()
        K, pairs = 0, 0
        while True:
            K += 1
            for st in states:
                st.superstep(stats=False)
            sent = [st.sync_delta(on_device=True) for st in states]
            pairs += sum(int(x[0].numel()) for x in sent)
            active = 0
            for q, st in enumerate(states):
                others = [x for i, x in enumerate(sent) if i != q and x[0].numel()]
                gid = torch.cat([o[0] for o in others]) if others else sent[q][0][:0]
                val = torch.cat([o[1] for o in others]) if others else sent[q][1][:0]
                active += st.apply_delta(gid, val)
            if active == 0:
                break
        torch.cuda.synchronize()
        return time.perf_counter() - t, K, pairs, states

    solve()
    times = []
    for _ in range(reps):
        dt, K, pairs, states = solve()
        times.append(dt)
    g = gen.rmat(scale, seed=2)
    ref = gx.State(gx.DeviceGraph(g, gx.GX_NEED_OUT), gx.GX_SSSP, source=0)
    rs, _ = ref.run(100_000)
    dist = ref.values_numpy()
    for p, st in zip(parts, states):
        assert np.array_equal(st.values_numpy(), dist[p.l2g]), "exchange differs from the whole-graph solve"
    assert K == rs.supersteps
    dt = sorted(times)[len(times) // 2]
    log(f"exchange: {nparts} parts, K={K}, {pairs} pairs exchanged, {dt * 1e3:.1f} ms per solve")
    out = {"workload": f"all {nparts} parts of a hash vertex-cut of R-MAT scale {scale} (seed 2) resident, "
                       "SSSP from vertex 0 with the sync sets exchanged every superstep (gx_sync_delta / "
                       "gx_apply_delta), equal to the whole-graph solve",
           "parts": nparts, "replicas": int(sum(p.V for p in parts)), "edges": int(sum(p.E for p in parts)),
           "supersteps": K, "pairs_exchanged_per_solve": pairs, "ms_per_solve": dt * 1e3,
           "whole_graph_messages_per_solve": int(rs.edges), "gteps": rs.edges / dt / 1e9}
    del states, dgs, ref
    out["pagerank"] = bench_exchange_pagerank(gx, torch, np, gen, g, parts)
    return out


def bench_exchange_pagerank(gx, torch, np, gen, g, parts, T=30):
    """PageRank, 30 supersteps, across all parts of the vertex-cut: merged
    sums of replicas to their masters in part order, masters apply with the
    whole graph's dangling mass, replicas take the masters' ranks; within
    1e-6 of the whole-graph PageRank."""
    parts = gen.cover_isolated(parts, g.V)
    deg = np.diff(g.row_ptr).astype(np.int32)
    states = []
    for p in parts:
        dg = gx.DeviceGraph(p, gx.GX_NEED_IN, V_global=g.V, outdeg_global=deg[p.l2g])
        states.append(gx.State(dg, gx.GX_PAGERANK, damping=0.85, phases=gx.GX_PHASES_MASTERS,
                               delta_mode=gx.GX_DELTA_MASTERS))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sums = bcast = 0
    for _ in range(T):
        for st in states:
            st.msg_gen()
            st.msg_merge()
        D = 0.0
        for st in states:
            D += st.dangling_get()
        for st in states:
            st.dangling_set(D)
        sent = [st.partial_emit() for st in states]
        sums += sum(int(x[0].numel()) for x in sent)
        for q, st in enumerate(states):
            for p in range(len(states)):
                if p != q and sent[p][0].numel():
                    st.partial_add(*sent[p])
        for st in states:
            st.msg_apply(stats=False)
        bc = [st.sync_delta(on_device=True) for st in states]
        bcast += sum(int(x[0].numel()) for x in bc)
        for q, st in enumerate(states):
            others = [b for p, b in enumerate(bc) if p != q and b[0].numel()]
            if others:
                st.apply_delta(torch.cat([o[0] for o in others]), torch.cat([o[1] for o in others]))
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    whole = gx.State(gx.DeviceGraph(g, gx.GX_NEED_IN), gx.GX_PAGERANK, damping=0.85)
    whole.run(T)
    xw = whole.values_numpy()
    err = max(float(np.max(np.abs(st.values_numpy() - xw[p.l2g]))) for p, st in zip(parts, states))
    assert err <= 1e-6, f"PageRank exchange differs from the whole-graph PageRank by {err}"
    log(f"exchange PageRank: {T} supersteps in {dt * 1e3:.1f} ms ({dt * 1e3 / T:.2f} ms per superstep), "
        f"{sums} merged sums and {bcast} ranks exchanged, max |diff| vs whole graph {err:.2e}")
    return {"workload": f"PageRank {T} supersteps across the {len(parts)} parts (isolated vertices mastered by "
                        "part 0), merged sums to masters in part order, masters' ranks back to replicas",
            "ms": dt * 1e3, "ms_per_superstep": dt * 1e3 / T, "merged_sums_exchanged": sums,
            "ranks_exchanged": bcast, "max_abs_diff_vs_whole_graph": err,
            "gteps": T * g.E / dt / 1e9}


def bench_lp(gx, torch, np, gen, g=None, scale=22, cap=15, reps=3):
    """Label propagation (most frequent neighbour label, smallest on a tie)
    on the symmetrised R-MAT scale-22 graph (seed 2), at most 15 iterations;
    the first iteration is checked against the oracle's iteration."""
    import oracle
    if g is None:
        g = gen.rmat(scale, seed=2)
    dg = gx.DeviceGraph(g, gx.GX_NEED_SYM)
    st = gx.State(dg, gx.GX_LP, timing=True)
    st.superstep()
    adj = oracle.SymAdjacency(g)
    t0 = time.perf_counter()
    want = adj.lp_step(np.arange(g.V, dtype=np.uint32))
    cpu_iter_s = time.perf_counter() - t0
    assert np.array_equal(st.values_numpy(), want), "LP iteration 1 differs from the oracle"
    times, kern = [], []
    for _ in range(reps + 1):
        st.reset()
        torch.cuda.synchronize()
        t = time.perf_counter()
        rs, steps = st.run(cap, per_step=True, allow_cap=True)
        times.append(time.perf_counter() - t)
        kern.append(rs.edge_kernel_ms)
    times, kern = times[1:], kern[1:]
    i = int(np.argsort(times)[len(times) // 2])
    dt, it = times[i], int(rs.supersteps)
    E_sym = int(steps[0][1])
    log(f"LP: {it} iterations ({'converged' if rs.converged else 'cap'}), {dt * 1e3:.2f} ms per run, "
        f"{dt * 1e3 / it:.3f} ms per iteration; one oracle iteration on one core {cpu_iter_s:.2f} s")
    alg = 4 * E_sym + 16 * g.V  # neighbour ids + labels read once per vertex + new labels written (lower bracket)
    return {"workload": f"label propagation on R-MAT scale {scale} (seed 2, symmetrised: {g.V} vertices, "
                        f"{E_sym} neighbour entries), at most {cap} iterations",
            "iterations": it, "converged": bool(rs.converged), "changed_per_iteration": [s[2] for s in steps],
            "ms_per_run": dt * 1e3, "ms_per_iteration": dt * 1e3 / it,
            "kernel_ms_per_iteration": kern[i] / it, "gteps": E_sym * it / dt / 1e9,
            "algorithmic_bytes_per_iteration": alg,
            "frac_of_hbm_peak": alg / (kern[i] / it / 1e3) / 1e9 / HBM_PEAK_GBS,
            "oracle_one_iteration_one_core_s": cpu_iter_s}


def bench_phases(gx, torch, np, gen, g=None, reps=5):
    """SSSP from vertex 0 on R-MAT scale 22 (seed 2) driven by the template's
    three calls made separately, in BSP order (Gen, Merge, Apply) and in GAS
    order (Merge, Apply, Gen), against the fused superstep; the same number
    of supersteps, the same distances."""
    if g is None:
        g = gen.rmat(22, seed=2)
    dg = gx.DeviceGraph(g, gx.GX_NEED_OUT)
    fused = gx.State(dg, gx.GX_SSSP, source=0)
    rs, _ = fused.run(100_000)
    K = int(rs.supersteps)
    want = fused.values_numpy().copy()

    def timed(fn):
        ts = []
        for _ in range(reps + 1):
            torch.cuda.synchronize()
            t = time.perf_counter()
            st = fn()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t)
        assert np.array_equal(st.values_numpy(), want)
        ts = sorted(ts[1:])
        return ts[len(ts) // 2] * 1e3

    def run_fused():
        fused.reset()
        fused.run(100_000)
        return fused

    split = gx.State(dg, gx.GX_SSSP, source=0, phases=True)

    def run_bsp():
        split.reset()
        for _ in range(K):
            split.msg_gen()
            split.msg_merge()
            split.msg_apply(stats=False)
        return split

    def run_gas():
        split.reset()
        split.msg_merge()
        split.msg_apply(stats=False)
        split.msg_gen()
        for _ in range(K):
            split.msg_merge()
            split.msg_apply(stats=False)
            split.msg_gen()
        return split

    out = {"workload": f"SSSP from vertex 0 on R-MAT scale 22 (seed 2), {K} supersteps",
           "fused_ms_per_solve": timed(run_fused), "bsp_separate_calls_ms_per_solve": timed(run_bsp),
           "gas_separate_calls_ms_per_solve": timed(run_gas)}
    log(f"template calls: fused {out['fused_ms_per_solve']:.2f} ms, BSP order "
        f"{out['bsp_separate_calls_ms_per_solve']:.2f} ms, GAS order {out['gas_separate_calls_ms_per_solve']:.2f} ms")
    return out


def host_cpu_model():
    """The host CPU's model name (/proc/cpuinfo), else the machine type."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or platform.machine()


def host_link_gbps(torch, nbytes=1 << 30, reps=3):
    """Pinned host -> device copy rate (the host link the load and the
    streamed supersteps cross)."""
    h = torch.empty(nbytes, dtype=torch.uint8, pin_memory=True)
    h.fill_(1)
    d = torch.empty(nbytes, dtype=torch.uint8, device="cuda:0")
    d.copy_(h, non_blocking=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        d.copy_(h, non_blocking=True)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    del h, d
    return nbytes / dt / 1e9


def bench_stream(gx, torch, np, gen, g=None):
    """Streamed supersteps (Section "Pipeline Shuffling") of SSSP from vertex 0
    on R-MAT scale 22 (seed 2), triplets in pinned host memory.  The stage
    costs are measured in the serial form at the superstep with the most
    messages (the paper calibrates at the SSSP iteration with the largest
    workload): k1 and k3 per triplet from the downloads and uploads of a
    large-block run, k2 from the computation at two block sizes, and a, the
    constant cost of one block, from the serial wall time at two block
    counts.  The Lemma's block size (Pipeline*) is then timed against a fixed
    block of 2^20 triplets and against no pipeline (one block, the stages in
    turn), with the paper's three rotating buffers and with eight, and a
    sweep of block sizes gives the measured best."""
    if g is None:
        g = gen.rmat(22, seed=2)
    res = gx.State(gx.DeviceGraph(g, gx.GX_NEED_OUT), gx.GX_SSSP, source=0)
    _, steps = res.run(100_000, per_step=True)
    want = res.values_numpy().copy()
    del res
    kmax = int(np.argmax([x[1] for x in steps]))  # superstep with the most messages
    E = g.E
    handles = {3: gx.Stream(g, gx.GX_SSSP, source=0, block_edges_max=E, ring=3),
               8: gx.Stream(g, gx.GX_SSSP, source=0, block_edges_max=1 << 22, ring=8)}

    def at(k, block, serial, ring=3):
        st = handles[ring]
        st.reset()
        for _ in range(k):
            st.superstep(1 << 22)
        return st.superstep(block, serial=serial)

    def timed(block, serial, ring=3):
        ts = sorted(at(kmax, block, serial, ring)["wall_ms"] for _ in range(3))
        return ts[1]

    b1, b2 = 1 << 16, 1 << 22
    r1, r2 = at(kmax, b1, True), at(kmax, b2, True)
    k1 = r2["download_ms"] * 1e-3 / E
    k3 = r2["upload_ms"] * 1e-3 / E
    tc1, tc2 = r1["compute_ms"] * 1e-3 / r1["blocks"], r2["compute_ms"] * 1e-3 / r2["blocks"]
    k2 = max((tc2 - tc1) / (b2 - b1), 0.0)
    w1, w2 = timed(b1, True), timed(b2, True)
    a = max((w1 - w2) * 1e-3 / (r1["blocks"] - r2["blocks"]), 0.0)
    blocks, bsize, t_model = gx.pipeline_plan(k1, k2, k3, a, E)
    bopt = int(np.ceil(E / blocks))
    forms = {"no_pipeline": {"block_triplets": E, "ring": 1, "wall_ms": timed(E, True)},
             "fixed_block_2^20": {"block_triplets": 1 << 20, "ring": 3, "wall_ms": timed(1 << 20, False)},
             "pipeline_star": {"block_triplets": bopt, "ring": 3, "wall_ms": timed(bopt, False)}}
    if bopt <= 1 << 22:
        forms["pipeline_star_ring8"] = {"block_triplets": bopt, "ring": 8, "wall_ms": timed(bopt, False, 8)}
    sweep = {f"2^{e}_ring{r}": timed(1 << e, False, r) for e in (16, 18, 20, 22) for r in (3, 8)}
    best = min(sweep, key=sweep.get)
    forms["pipeline_star"]["model_ms"] = t_model * 1e3
    # the whole solve, streamed at the Lemma's block size
    st = handles[3]
    st.reset()
    t0 = time.perf_counter()
    K = msgs = 0
    while True:
        r = st.superstep(bopt)
        K += 1
        msgs += r["messages"]
        if r["changed"] == 0:
            break
    solve_s = time.perf_counter() - t0
    assert np.array_equal(st.values_numpy(), want), "streamed solve differs from the resident one"
    link = host_link_gbps(torch)
    log(f"stream: k1={k1 * 1e9:.3f} k2={k2 * 1e9:.3f} k3={k3 * 1e9:.3f} ns/triplet, a={a * 1e6:.1f} us per block; "
        f"Lemma: {blocks} blocks of {bsize:.0f} (model {t_model * 1e3:.2f} ms); superstep {kmax}: "
        + ", ".join(f"{n} {f['wall_ms']:.2f} ms" for n, f in forms.items())
        + f"; best of sweep {best} {sweep[best]:.2f} ms; solve {solve_s * 1e3:.1f} ms; host link {link:.1f} GB/s")
    return {"workload": f"SSSP from vertex 0 on R-MAT scale 22 (seed 2), {E} triplets (12 B down, 4 B up each) "
                        f"streamed from pinned host memory every superstep",
            "calibration_superstep": kmax, "messages_at_calibration": int(steps[kmax][1]),
            "coef": {"k1_ns": k1 * 1e9, "k2_ns": k2 * 1e9, "k3_ns": k3 * 1e9, "a_us": a * 1e6},
            "lemma_blocks": blocks, "lemma_block_triplets": bsize, "model_ms": t_model * 1e3,
            "forms": forms, "sweep_pipelined_ms": sweep, "sweep_best": best,
            "pipeline_star_speedup_vs_none": forms["no_pipeline"]["wall_ms"] / forms["pipeline_star"]["wall_ms"],
            "pipeline_star_speedup_vs_fixed": forms["fixed_block_2^20"]["wall_ms"] / forms["pipeline_star"]["wall_ms"],
            "solve": {"supersteps": K, "ms": solve_s * 1e3, "messages": int(msgs),
                      "host_bytes_per_superstep": 16 * E, "GBps_over_host_link": 16 * E * K / solve_s / 1e9},
            "host_link_h2d_GBps": link}


def bench_split(gx, torch, np, gen, g=None):
    """The graph split between the GPU and the CPU daemon (Section "Workload
    Balancing", Lemma "minmaxcidi"): SSSP from vertex 0 on R-MAT scale 22
    (seed 2).  c_j = a whole solve's time per edge on each worker alone; the
    Lemma's share d_cpu = D (1/c_cpu) / (1/c_cpu + 1/c_gpu) is timed against
    an even split and the GPU alone, each superstep running both parts at
    once and exchanging their sync sets."""
    if g is None:
        g = gen.rmat(22, seed=2)
    E = g.E
    whole = gx.State(gx.DeviceGraph(g, gx.GX_NEED_OUT), gx.GX_SSSP, source=0)
    whole.run(100_000)
    ts = []
    for _ in range(5):
        whole.reset()
        torch.cuda.synchronize()
        t = time.perf_counter()
        rs, _ = whole.run(100_000)
        ts.append(time.perf_counter() - t)
    t_gpu = sorted(ts)[2]
    want = whole.values_numpy().copy()
    del whole
    cw = gx.CpuPart(g, gx.GX_SSSP, source=0)
    t = time.perf_counter()
    while cw.superstep()[2]:
        pass
    t_cpu = time.perf_counter() - t
    assert np.array_equal(cw.values_numpy(), want)
    del cw
    c = np.array([t_gpu / E, t_cpu / E])
    d = gx.balance_split(c, E)
    share = float(d[1] / E)

    def run(share):
        parts = gen.split_by_share(g, share)

        def local(p):
            loc = int(np.searchsorted(p.l2g, 0))
            return loc if loc < p.V and p.l2g[loc] == 0 else -1

        gpu = gx.State(gx.DeviceGraph(parts[0], gx.GX_NEED_OUT), gx.GX_SSSP, source=local(parts[0]))
        cpu = gx.CpuPart(parts[1], gx.GX_SSSP, source=local(parts[1]))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        K = tc = 0
        while True:
            K += 1
            gpu.superstep(stats=False)
            t1 = time.perf_counter()
            cpu.superstep()
            tc += time.perf_counter() - t1
            gg, gv, _ = gpu.sync_delta()
            cg, cv = cpu.sync_delta()
            act = cpu.apply_delta(gg, gv)
            act += gpu.apply_delta(torch.tensor(cg, device="cuda:0"), torch.tensor(cv.view(np.int32), device="cuda:0"))
            if act == 0:
                break
        dt = time.perf_counter() - t0
        best = np.full(g.V, 0xFFFFFFFF, np.uint32)
        np.minimum.at(best, parts[0].l2g, gpu.values_numpy())
        np.minimum.at(best, parts[1].l2g, cpu.values_numpy())
        held = np.zeros(g.V, bool)
        held[parts[0].l2g] = True
        held[parts[1].l2g] = True
        assert np.array_equal(best[held], want[held]), f"split at share {share} differs from the whole-graph solve"
        return {"cpu_share": share, "cpu_edges": int(parts[1].E), "gpu_edges": int(parts[0].E), "supersteps": K,
                "ms_per_solve": dt * 1e3, "cpu_superstep_ms_total": tc * 1e3}

    out = {"workload": f"SSSP from vertex 0 on R-MAT scale 22 (seed 2) split by edge hash between the GPU and the "
                       f"CPU daemon ({os.cpu_count()} host threads), sync sets exchanged every superstep",
           "c_gpu_ns_per_edge": c[0] * 1e9, "c_cpu_ns_per_edge": c[1] * 1e9, "gpu_alone_ms": t_gpu * 1e3,
           "cpu_alone_ms": t_cpu * 1e3, "lemma_cpu_share": share,
           "lemma_predicted_ms": E / np.sum(1.0 / c) * 1e3,
           "lemma_split": run(share), "even_split": run(0.5)}
    log(f"split: c_gpu {c[0] * 1e9:.4f} c_cpu {c[1] * 1e9:.3f} ns/edge; Lemma share {share:.5f} -> "
        f"{out['lemma_split']['ms_per_solve']:.2f} ms (model {out['lemma_predicted_ms']:.2f} ms), even split "
        f"{out['even_split']['ms_per_solve']:.1f} ms, GPU alone {t_gpu * 1e3:.2f} ms, CPU alone {t_cpu * 1e3:.0f} ms")
    return out


def bench_partition(gx, torch, np, gen, reps=3):
    """One part (1 of 8) of a hash vertex-cut of R-MAT scale 25 (seed 3):
    30 PageRank supersteps and min-label CC to convergence."""
    t0 = time.perf_counter()
    p = gen.rmat_part(25, seed=3, part=0)
    log(f"partition: V_p={p.V} E_p={p.E} generated in {time.perf_counter() - t0:.1f}s")
    dg = gx.DeviceGraph(p, gx.GX_NEED_IN | gx.GX_NEED_SYM)
    st = gx.State(dg, gx.GX_PAGERANK, damping=0.85, timing=True)
    st.run(30)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    kern = 0.0
    for _ in range(reps):
        st.reset()
        rs, _ = st.run(30)
        kern += rs.edge_kernel_ms
    torch.cuda.synchronize()
    t_pr = (time.perf_counter() - t0) / reps
    pr_bytes = 30 * (4 * p.E + 20 * p.V)
    cc = gx.State(dg, gx.GX_CC, timing=True)
    cc.run(100_000)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    cc_edges = 0
    t_solve = t_sync = 0.0
    for _ in range(reps):
        t1 = time.perf_counter()
        cc.reset()
        rs_cc, steps = cc.run(100_000, per_step=True, detail=True)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        cc_edges += rs_cc.edges
        gids, vals, skip = cc.sync_delta(on_device=True)  # the sync set stays in HBM
        torch.cuda.synchronize()
        t_solve += t2 - t1
        t_sync += time.perf_counter() - t2
    t_cc = (time.perf_counter() - t0) / reps
    log(f"partition CC: solve {t_solve / reps * 1e3:.2f} ms (kernels {sum(d['kernel_ms'] for d in steps):.2f} ms), "
        f"sync set {t_sync / reps * 1e3:.2f} ms; PageRank {t_pr * 1e3:.2f} ms")
    # The sync set taken after every superstep (lazy upload of the changed
    # vertices other parts need, and the skip decision), untimed.
    gbuf = torch.empty(p.V, dtype=torch.int32, device="cuda:0")
    vbuf = torch.empty_like(gbuf)

    def per_step_deltas(state, max_steps, until_idle):
        out = []
        state.reset()
        for _ in range(max_steps):
            _, _, changed = state.superstep(stats=True)
            g_, _, skip = state.sync_delta(on_device=True, out=(gbuf, vbuf))
            out.append((int(g_.numel()), bool(skip)))
            if until_idle and changed == 0:
                break
        return out

    cc_d = per_step_deltas(cc, 100_000, True)
    pr_d = per_step_deltas(st, 30, False)
    log(f"partition sync sets per superstep: CC {[n for n, _ in cc_d]} ({sum(k for _, k in cc_d)} skipped); "
        f"PageRank {pr_d[0][0]}..{pr_d[-1][0]} ({sum(k for _, k in pr_d)} skipped)")
    return {"workload": f"part 0 of an 8-way hash vertex-cut of R-MAT scale 25 (seed 3): V_p={p.V}, E_p={p.E}; "
                        "PageRank 30 supersteps + min-label CC to convergence + final sync set",
            "pagerank_ms": t_pr * 1e3, "pagerank_gteps": 30 * p.E / t_pr / 1e9,
            "pagerank_pull_roofline_frac": pr_bytes / (kern / reps / 1e3) / 1e9 / HBM_PEAK_GBS,
            "cc_ms": t_cc * 1e3, "cc_solve_ms": t_solve / reps * 1e3, "cc_sync_set_ms": t_sync / reps * 1e3,
            "cc_supersteps": int(rs_cc.supersteps), "cc_gteps": cc_edges / reps / t_cc / 1e9,
            "cc_kernel_ms": sum(d["kernel_ms"] for d in steps),
            "sync_set_final": int(gids.numel()),
            "sync_set_per_superstep": {"cc": [n for n, _ in cc_d], "cc_skipped": sum(k for _, k in cc_d),
                                       "pagerank": [n for n, _ in pr_d],
                                       "pagerank_skipped": sum(k for _, k in pr_d),
                                       "what": "changed vertices another part needs, emitted after every "
                                               "superstep (lazy upload); skipped = empty sets"},
            "cc_per_superstep": [dict(edges=d["edges"], pulled=d["pulled"], us=round(d["kernel_ms"] * 1e3, 1))
                                 for d in steps]}, p


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "sssp_rmat22_relaxation_traffic.json")
KERNEL_SOURCES = os.path.join(ROOT, "paper_2203_13005_amd", "csrc")


# The sources the relaxation kernels, their launches and the graph layout
# they read come from (the batched, serving, label-propagation, streaming
# and CPU-daemon files hold none of them).
RELAXATION_SOURCES = ("gx_device.h", "gx_graph.hip", "gx_internal.h", "gx_plain.hip")


def kernel_source_hash():
    """Hash of the sources behind the relaxation kernels (kernels, layouts,
    launch code): a traffic record taken on other sources is not reported."""
    import hashlib
    h = hashlib.sha256()
    for name in RELAXATION_SOURCES:
        h.update(name.encode())
        h.update(open(os.path.join(KERNEL_SOURCES, name), "rb").read())
    return h.hexdigest()[:16]


def summarize_pmc(fetch_dir, write_dir, solves):
    """Turns two rocprofv3 --pmc passes (FETCH_SIZE, WRITE_SIZE) over
    `bench.py --copy-calibration` into the traffic record bench.py reports.
    Each counter is scaled so the 1 GiB device copy reads (writes) 1 GiB."""
    import csv
    import glob

    def load(d, counter):
        rows = []
        for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            rows += [r for r in csv.DictReader(open(f)) if r.get("Counter_Name") == counter]
        return rows

    out = {"source_sha256_16": kernel_source_hash(), "solves_profiled": None}
    for counter, d in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir)):
        rows = load(d, counter)
        copy = [float(r["Counter_Value"]) for r in rows if "copy" in r["Kernel_Name"].lower() and
                float(r["Counter_Value"]) > 500_000]
        relax = [float(r["Counter_Value"]) for r in rows if "k_relax" in r["Kernel_Name"] or "k_fixup" in r["Kernel_Name"]]
        if not copy or not relax:
            raise SystemExit(f"{counter}: no calibration copy or no relaxation dispatches in {d}")
        factor = (1 << 30) / 1024.0 / max(copy)  # KiB of a 1 GiB copy / measured
        out[counter] = {"calibration_copy_kib": max(copy), "factor": factor,
                        "relaxation_dispatches": len(relax), "relaxation_kib_total": sum(relax),
                        "relaxation_bytes_total_calibrated": sum(relax) * 1024.0 * factor}
    out["solves_profiled"] = solves
    out["note"] = ("push and pull dispatches of every solve in the profiled run (validation, warm-up, detail "
                   "and timed solves, all identical) summed and divided by the number of solves")
    out["bytes_per_solve"] = (out["FETCH_SIZE"]["relaxation_bytes_total_calibrated"] +
                              out["WRITE_SIZE"]["relaxation_bytes_total_calibrated"]) / solves
    os.makedirs(os.path.dirname(TRAFFIC_FILE), exist_ok=True)
    json.dump(out, open(TRAFFIC_FILE, "w"), indent=1)
    print(json.dumps(out, indent=1))


def load_traffic():
    """Measured HBM bytes per relaxation launch, or None when absent or
    taken on a different kernel source."""
    try:
        t = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    if t.get("source_sha256_16") != kernel_source_hash():
        return None
    return t


LEGS = ("sssp", "pagerank", "partition", "lp", "phases", "stream", "split", "exchange", "batched", "serving")


def bench_sssp(args, gx, torch, np, gen):
    """The headline: one SSSP solve per step on R-MAT scale 22 (seed 2),
    source 0.  Returns (fields of the JSON line, host graph, messages per
    solve)."""
    dev = torch.device("cuda:0")
    log(f"generating R-MAT scale {args.scale}")
    t0 = time.perf_counter()
    g = gen.rmat(args.scale, seed=2)
    log(f"V={g.V} E={g.E} generated in {time.perf_counter() - t0:.1f}s")
    t0 = time.perf_counter()
    dg = gx.DeviceGraph(g, gx.GX_NEED_OUT, device=dev)  # out-CSR (push) + in-CSR (pull)
    torch.cuda.synchronize()
    load_s = time.perf_counter() - t0
    load_bytes = dg.arena_bytes
    log(f"loaded in {load_s:.2f}s ({load_bytes / load_s / 1e9:.2f} GB/s of device images, host packaging included)")

    # Untimed validation pass: per-superstep frontiers for the byte model.
    st = gx.State(dg, gx.GX_SSSP, source=0, pull_fraction=args.pull_fraction)
    fronts = [np.zeros(g.V, bool)]
    fronts[0][0] = True
    while True:
        fr, ef, ch = st.superstep(stats=True)
        fronts.append(st.frontier_numpy())
        if ch == 0:
            break
    per_step = push_bytes_per_superstep(g, fronts)
    K = len(per_step)
    edges_per_solve = sum(p["edges"] for p in per_step)
    bytes_per_solve = sum(p["bytes"] for p in per_step)
    dist_ref = st.values_numpy().copy()
    st.close()
    log(f"K={K} supersteps, {edges_per_solve} messages/solve, {bytes_per_solve / 1e9:.3f} GB algorithmic "
        f"relaxation bytes/solve")

    state = gx.State(dg, gx.GX_SSSP, source=0, timing=True, pull_fraction=args.pull_fraction)
    cap = 1 << 20
    # the sync set stays in HBM (device buffers allocated once), ready for an exchange
    sync_out = (torch.empty(cap, dtype=torch.int32, device="cuda:0"), torch.empty(cap, dtype=torch.int32, device="cuda:0"))
    for _ in range(args.warmup):
        state.reset()
        state.run(100_000)
        state.sync_delta(cap=cap, on_device=True, out=sync_out)
    torch.cuda.synchronize()

    state.reset()
    _, detail = state.run(100_000, per_step=True, detail=True)
    assert np.array_equal(state.values_numpy(), dist_ref)
    for i, d in enumerate(detail):
        log(f"  superstep {i:2d}: |F|={d['frontier']:>8d} edges={d['edges']:>9d} changed={d['changed']:>8d} "
            f"{'pull' if d['pulled'] else 'push'} {d['kernel_ms'] * 1e3:8.1f} us")
    kern_ms = 0.0
    launches = 0
    edges = 0
    log(f"timing {args.steps} solves")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    marks = [t0]  # host clock after each solve (its run returns after the solve's last superstep)
    for _ in range(args.steps):
        state.reset()
        rs, _ = state.run(100_000)
        state.sync_delta(cap=cap, on_device=True, out=sync_out)
        kern_ms += rs.edge_kernel_ms
        launches += rs.edge_kernel_launches
        edges += rs.edges
        marks.append(time.perf_counter())
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    solve_ms = np.diff(marks) * 1e3
    assert edges == edges_per_solve * args.steps
    assert np.array_equal(state.values_numpy(), dist_ref)
    log(f"{dt * 1e3 / args.steps:.3f} ms/solve, relaxation kernel {kern_ms / args.steps:.3f} ms/solve "
        f"over {launches / args.steps:.1f} launches")
    # The timed solves repeat one source; one solve from each of 16 other
    # sources (seeded, out-degree > 0, no sync set) shows the spread.
    src_ms, src_msgs, src_steps = [], 0, []
    for s_ in (gen.pick_sources(g, args.other_sources, seed=21) if args.other_sources > 0 else []):
        stx = gx.State(dg, gx.GX_SSSP, source=int(s_), pull_fraction=args.pull_fraction)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        rsx, _ = stx.run(100_000)
        torch.cuda.synchronize()
        src_ms.append((time.perf_counter() - t1) * 1e3)
        src_msgs += rsx.edges
        src_steps.append(int(rsx.supersteps))
        stx.close()
    if src_ms:
        log(f"{len(src_ms)} other sources: {np.mean(src_ms):.3f} ms/solve on average ({min(src_ms):.3f}-"
            f"{max(src_ms):.3f}), {src_msgs / (sum(src_ms) / 1e3) / 1e9:.1f} GTEPS, "
            f"{min(src_steps)}-{max(src_steps)} supersteps")

    achieved = bytes_per_solve * args.steps / (kern_ms / 1e3) / 1e9
    bytes_upper = sum(p["bytes_upper"] for p in per_step)
    achieved_upper = bytes_upper * args.steps / (kern_ms / 1e3) / 1e9
    copy_gbps = copy_ceiling_gbps(torch)
    log(f"device copy ceiling {copy_gbps:.0f} GB/s")
    link_gbps = host_link_gbps(torch)
    log(f"host link (pinned host to device) {link_gbps:.1f} GB/s; the load moved {load_bytes / 1e9:.2f} GB at "
        f"{load_bytes / load_s / 1e9:.2f} GB/s")
    traffic = load_traffic()
    out = {
        "value": edges / dt / 1e9,
        "ms_per_step": dt * 1e3 / args.steps,
        "solve_ms": {"median": float(np.median(solve_ms)), "min": float(solve_ms.min()),
                     "max": float(solve_ms.max()),
                     "what": "host clock between consecutive solves of the timed loop (the sync set of each "
                             "solve is still in flight at its mark)"},
        "config": {
            "workload": f"Bellman-Ford SSSP to convergence from vertex 0, R-MAT scale {args.scale} "
                        f"({g.V} vertices, {16 * g.V} raw edges, a=0.57 b=0.19 c=0.19 d=0.05, seed 2, "
                        f"self-loops and duplicates removed), uint32 weights in [1,255]",
            "V": g.V, "E": g.E, "supersteps": K, "messages_per_solve": edges_per_solve,
            "parallelism": "single GPU",
        },
        "other_sources": None if not src_ms else {
            "what": f"one solve from each of {len(src_ms)} seeded sources with out-degree > 0 (seed 21), "
                    "no sync set; the timed solves above repeat source 0",
            "ms_per_solve_mean": float(np.mean(src_ms)), "ms_per_solve_min": min(src_ms),
            "ms_per_solve_max": max(src_ms), "gteps": src_msgs / (sum(src_ms) / 1e3) / 1e9,
            "supersteps": src_steps},
        "load": {"what": "gx_graph_load: host validation and packaging (out-CSR, in-edge records), "
                         "16 MiB blocks through three rotating pinned buffers on a copy stream",
                 "seconds": load_s, "device_bytes": load_bytes, "GBps": load_bytes / load_s / 1e9,
                 "host_link_GBps": link_gbps,
                 "bound": "host packaging on the CPU threads (the copies would take "
                          f"{load_bytes / link_gbps / 1e9 * 1e3:.0f} ms of the {load_s * 1e3:.0f} ms at the link's rate)"},
        "roofline": {
            "bound": "hbm",
            "kernel": "relaxation: k_relax<true> (push or pull as the frontier decides) + k_fixup, per superstep",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": None if traffic is None else traffic["bytes_per_solve"],
            "traffic_unit": "HBM bytes of the relaxation kernels per solve (FETCH_SIZE + WRITE_SIZE, "
                            "copy-calibrated); achieved = algorithmic bytes per solve / their time per solve",
            "algorithmic_bytes_per_solve": bytes_per_solve,
            "algorithmic_bytes_upper_per_solve": bytes_upper,
            "achieved_upper": achieved_upper,
            "frac_upper": achieved_upper / HBM_PEAK_GBS,
            "copy_ceiling_GBps": copy_gbps,
            "frac_of_copy_ceiling": achieved / copy_gbps,
            "kernel_ms_per_solve": kern_ms / args.steps,
            "launches_per_solve": launches / args.steps,
            "per_superstep": [dict(edges=p["edges"], bytes=p["bytes"], pulled=int(d["pulled"]),
                                   us=round(d["kernel_ms"] * 1e3, 1)) for p, d in zip(per_step, detail)],
        },
    }
    return out, g, edges_per_solve


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--scale", type=int, default=22)
    ap.add_argument("--legs", default=",".join(LEGS),
                    help="comma-separated legs to run (default: all of " + ",".join(LEGS) + ")")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--pull-fraction", type=float, default=0.0,
                    help="SSSP switch point to the pull form (0 = library default, >= 1 = push only)")
    ap.add_argument("--serving-queries", type=int, default=10000)
    ap.add_argument("--other-sources", type=int, default=16,
                    help="after the timed solves, one solve from each of this many other sources (0 = none)")
    ap.add_argument("--summarize-pmc", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="write the traffic record from two rocprofv3 --pmc output folders and exit")
    ap.add_argument("--pmc-solves", type=int, default=0,
                    help="solves in the profiled run (1 validation + warmup + 1 detail + steps)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy (for HBM counter calibration)")
    args = ap.parse_args()
    if args.summarize_pmc:
        summarize_pmc(args.summarize_pmc[0], args.summarize_pmc[1], args.pmc_solves)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU exchange is not built.",
              file=sys.stderr)
        sys.exit(2)
    legs = [x for x in args.legs.split(",") if x]
    bad = [x for x in legs if x not in LEGS]
    if bad:
        ap.error(f"unknown legs {bad}; choose from {LEGS}")

    import numpy as np
    import torch

    import gen
    import paper_2203_13005_amd as gx

    out = {
        "metric": "GTEPS per superstep and % HBM roofline; batched-vs-plain SSSP queries/s, p50/p99",
        "value": None,
        "unit": "GTEPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": None,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "gpu": torch.cuda.get_device_name(0) if torch.cuda.is_available() else None,
        "config": {"workload": "none (headline leg not run)"},
    }
    g = edges_per_solve = None
    if "sssp" in legs:
        head, g, edges_per_solve = bench_sssp(args, gx, torch, np, gen)
        out.update(head)
    if "pagerank" in legs:
        out["pagerank_scale14"] = bench_pagerank_small(gx, torch, np, gen)
    part = None
    if "partition" in legs:
        out["partition_scale25"], part = bench_partition(gx, torch, np, gen)
    if "stream" in legs:
        out["stream_sssp_scale22"] = bench_stream(gx, torch, np, gen, g)
    if "split" in legs:
        out["split_sssp_scale22"] = bench_split(gx, torch, np, gen, g)
    if "phases" in legs:
        out["template_calls_sssp_scale22"] = bench_phases(gx, torch, np, gen, g)
    if "lp" in legs:
        out["lp_scale22"] = bench_lp(gx, torch, np, gen, g)
    if "exchange" in legs:
        out["exchange_8parts_scale22"] = bench_exchange(gx, torch, np, gen)
    g4 = src4 = None
    if "batched" in legs:
        out["batched"], g4, src4 = bench_batched(gx, torch, np, gen)
    if "serving" in legs:
        out["serving"] = bench_serving(gx, torch, np, gen, n_queries=args.serving_queries)
    if args.copy_calibration:
        a = torch.empty(1 << 30, dtype=torch.uint8, device="cuda:0")
        b = torch.empty_like(a)
        a.fill_(1)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
        log("copy calibration: 1 GiB device-to-device copy done")
    if g is not None and not args.no_cpu_baseline:
        log("timing the CPU oracle")
        out["cpu_baseline"] = cpu_baseline(np, g, edges_per_solve, g4, src4, part)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
