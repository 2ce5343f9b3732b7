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


def log(msg):
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def push_bytes_per_superstep(g, fronts):
    """Algorithmic bytes of the relaxation kernel per superstep: 8 B per
    active out-edge (destination + weight), 16 B per active-list entry, 4 B
    per distinct destination read, 4 B per vertex that improves."""
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
        out.append(dict(edges=ef, list=len(f), dests=nf, changed=int(fronts[k + 1].sum()),
                        bytes=8 * ef + 16 * len(f) + 4 * nf + 4 * int(fronts[k + 1].sum())))
    return out


def cpu_baseline(g, edges_per_solve, budget_s=20.0):
    import oracle
    times = []
    t_all = time.perf_counter()
    while True:
        t0 = time.perf_counter()
        r = oracle.sssp(g, 0)
        times.append(time.perf_counter() - t0)
        if time.perf_counter() - t_all > budget_s or len(times) >= 5:
            break
    times.sort()
    med = times[len(times) // 2]
    assert int(r.msgs.sum()) == edges_per_solve
    return {"value": edges_per_solve / med / 1e9, "unit": "GTEPS", "cores": 1, "kind": "oracle",
            "sample": f"full single-source solve from vertex 0 ({r.K} supersteps, {edges_per_solve} messages), "
                      f"single-threaded C oracle, median of {len(times)} runs ({med:.2f} s each)",
            "host_cpu": platform.processor() or platform.machine(), "host_nproc": os.cpu_count()}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--scale", type=int, default=22)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--pull-fraction", type=float, default=0.0,
                    help="SSSP switch point to the pull form (0 = library default, >= 1 = push only)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy (for HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU exchange is not built.",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import gen
    import paper_2203_13005_amd as gx

    dev = torch.device("cuda:0")
    log(f"generating R-MAT scale {args.scale}")
    t0 = time.perf_counter()
    g = gen.rmat(args.scale, seed=2)
    log(f"V={g.V} E={g.E} generated in {time.perf_counter() - t0:.1f}s")
    t0 = time.perf_counter()
    dg = gx.DeviceGraph(g, gx.GX_NEED_OUT, device=dev)  # out-CSR (push) + in-CSR (pull)
    torch.cuda.synchronize()
    load_s = time.perf_counter() - t0
    log(f"loaded in {load_s:.2f}s ({(g.E * 8 + g.V * 4) / load_s / 1e9:.2f} GB/s host->device incl. packaging)")

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
    for _ in range(args.warmup):
        state.reset()
        state.run(100_000)
        state.sync_delta(cap=cap)
    torch.cuda.synchronize()
    assert np.array_equal(state.values_numpy(), dist_ref)

    state.reset()
    _, detail = state.run(100_000, per_step=True, detail=True)
    for i, d in enumerate(detail):
        log(f"  superstep {i:2d}: |F|={d['frontier']:>8d} edges={d['edges']:>9d} changed={d['changed']:>8d} "
            f"{'pull' if d['pulled'] else 'push'} {d['kernel_ms'] * 1e3:8.1f} us")
    kern_ms = 0.0
    launches = 0
    edges = 0
    log(f"timing {args.steps} solves")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        state.reset()
        rs, _ = state.run(100_000)
        state.sync_delta(cap=cap)
        kern_ms += rs.edge_kernel_ms
        launches += rs.edge_kernel_launches
        edges += rs.edges
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    assert edges == edges_per_solve * args.steps
    assert np.array_equal(state.values_numpy(), dist_ref)
    log(f"{dt * 1e3 / args.steps:.3f} ms/solve, relaxation kernel {kern_ms / args.steps:.3f} ms/solve "
        f"over {launches / args.steps:.1f} launches")

    if args.copy_calibration:
        a = torch.empty(1 << 30, dtype=torch.uint8, device=dev)
        b = torch.empty_like(a)
        a.fill_(1)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        log("copy calibration: 1 GiB device-to-device copy done")

    achieved = bytes_per_solve * args.steps / (kern_ms / 1e3) / 1e9
    out = {
        "metric": "GTEPS per superstep and % HBM roofline; batched-vs-plain SSSP queries/s, p50/p99",
        "value": edges / dt / 1e9,
        "unit": "GTEPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {
            "workload": f"Bellman-Ford SSSP to convergence from vertex 0, R-MAT scale {args.scale} "
                        f"({g.V} vertices, {16 * g.V} raw edges, a=0.57 b=0.19 c=0.19 d=0.05, seed 2, "
                        f"self-loops and duplicates removed), uint32 weights in [1,255]",
            "V": g.V, "E": g.E, "supersteps": K, "messages_per_solve": edges_per_solve,
            "parallelism": "single GPU",
        },
        "roofline": {
            "bound": "hbm",
            "kernel": "relaxation: k_push<true> / k_pull<true> (one of the two works per superstep)",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": None,
            "algorithmic_bytes_per_solve": bytes_per_solve,
            "kernel_ms_per_solve": kern_ms / args.steps,
            "launches_per_solve": launches / args.steps,
            "per_superstep": [dict(edges=p["edges"], bytes=p["bytes"], pulled=int(d["pulled"]),
                                   us=round(d["kernel_ms"] * 1e3, 1)) for p, d in zip(per_step, detail)],
        },
    }
    if not args.no_cpu_baseline:
        log("timing the CPU oracle")
        out["cpu_baseline"] = cpu_baseline(g, edges_per_solve)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
