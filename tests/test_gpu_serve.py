"""Serving loop on MI355X: queries over several resident graphs, admitted as
lanes free up, must each match the oracle and match their own result when
run alone."""
import time

import numpy as np
import pytest

import gen
import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2203_13005_amd as m
    return m


@pytest.fixture(scope="module")
def graphs():
    return [gen.rmat(10, seed=100), gen.rmat(11, seed=101), gen.rmat(12, seed=102)]


def serve(gx, graphs, queries, budget=1 << 30, lanes=32, epoch=3, stagger_s=0.0, max_pools=4, dgs=None,
          gaps=None):
    if dgs is None:
        dgs = [gx.DeviceGraph(g, gx.GX_NEED_OUT | gx.GX_NEED_IN) for g in graphs]
    srv = gx.Server(budget, lanes_per_pool=lanes, max_pools=max_pools, epoch_supersteps=epoch, ppr_iters=50)
    ids = [srv.add_graph(d) for d in dgs]
    qids = {}
    for i, (gi, algo, s) in enumerate(queries):
        qids[srv.submit(ids[gi], algo, s)] = i
        if gaps is not None:
            time.sleep(gaps[i])
        elif stagger_s:
            time.sleep(stagger_s)
    done = {}
    t0 = time.time()
    while len(done) < len(queries):
        for c in srv.poll(wait_ms=50):
            assert c.status == 0
            done[qids[c.id]] = c
        assert time.time() - t0 < 120, "serving did not finish"
    srv.close()
    return done


def mixed_queries(graphs, n, seed):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        gi = int(rng.integers(0, len(graphs)))
        g = graphs[gi]
        cand = np.nonzero(np.diff(g.row_ptr) > 0)[0]
        algo = 1 if i % 2 == 0 else 3  # GX_SSSP / GX_PPR
        out.append((gi, algo, int(rng.choice(cand))))
    return out


def check(gx, graphs, q, c, threads=1):
    gi, algo, s = q
    g = graphs[gi]
    if algo == gx.GX_SSSP:
        ref = oracle.sssp(g, s, threads=threads)
        assert np.array_equal(c.result, ref.state)
        assert c.supersteps == ref.K
    else:
        ref = oracle.ppr(g, s, 50, threads=threads)
        assert np.max(np.abs(c.result.astype(np.float64) - ref)) <= 1e-6


def test_serving_mixed_matches_oracle_and_alone(gx, graphs):
    queries = mixed_queries(graphs, 48, seed=5)
    done = serve(gx, graphs, queries, stagger_s=0.002)
    for i, q in enumerate(queries):
        check(gx, graphs, q, done[i])
    # the same query alone gives the same bits
    for i in (0, 1, 6, 13):
        alone = serve(gx, graphs, [queries[i]])
        assert np.array_equal(alone[0].result.view(np.uint32), done[i].result.view(np.uint32)), i


def test_serving_admits_while_running(gx, graphs):
    # queries arriving while others run join at superstep boundaries; the
    # arrival gap is an eighth of one query's own time on the device, so
    # several arrive during each query's life whatever the speed
    queries = [(2, gx.GX_PPR, int(s)) for s in gen.pick_sources(graphs[2], 20, seed=9)]
    one = serve(gx, graphs, queries[:1], epoch=2)[0]
    gap = max((one.done_s - one.start_s) / 8, 1e-4)
    done = serve(gx, graphs, queries, lanes=32, epoch=2, stagger_s=gap)
    spans = [(c.start_s, c.done_s) for c in done.values()]
    # some query was admitted after another had started but before it finished
    assert any(a0 < b0 < a1 for a0, a1 in spans for b0, _ in spans), (gap, sorted(spans)[:4])
    for i, q in enumerate(queries):
        check(gx, graphs, q, done[i])


def test_serving_small_budget_queues(gx, graphs):
    g = graphs[0]
    queries = mixed_queries([g], 12, seed=11)
    dg = gx.DeviceGraph(g, gx.GX_NEED_OUT | gx.GX_NEED_IN)
    import ctypes
    b_sssp, b_ppr = ctypes.c_size_t(), ctypes.c_size_t()
    gx.binding.lib.gx_server_bytes_per_lane(dg.handle, gx.GX_SSSP, ctypes.byref(b_sssp))
    gx.binding.lib.gx_server_bytes_per_lane(dg.handle, gx.GX_PPR, ctypes.byref(b_ppr))
    # the bytes of one 64-lane pool of the larger kind: a 32-lane pool always
    # fits, the two kinds may have to take turns (idle empty pools are evicted)
    budget = int(max(b_sssp.value, b_ppr.value) * 64)
    done = serve(gx, [g], queries, budget=budget, lanes=32)
    for i, q in enumerate(queries):
        check(gx, [g], q, done[i])


def test_serving_tight_budget_serves_every_pair(gx, graphs):
    """Six (graph, algorithm) pairs under a budget of about two 32-lane pools
    of the largest kind, with steady traffic to one pair: every other pair
    still gets a pool in turn (resident pools are drained to make room), and
    every result matches the oracle."""
    import ctypes
    dgs = [gx.DeviceGraph(g, gx.GX_NEED_OUT | gx.GX_NEED_IN) for g in graphs]
    per_lane = 0
    for d in dgs:
        for algo in (gx.GX_SSSP, gx.GX_PPR):
            b = ctypes.c_size_t()
            gx.binding.lib.gx_server_bytes_per_lane(d.handle, algo, ctypes.byref(b))
            per_lane = max(per_lane, b.value)
    rng = np.random.default_rng(21)
    queries = []
    for i in range(72):
        gi, algo = (2, gx.GX_PPR) if i % 2 == 0 else (int(rng.integers(0, 3)), (gx.GX_SSSP, gx.GX_PPR)[i % 4 // 2])
        cand = np.nonzero(np.diff(graphs[gi].row_ptr) > 0)[0]
        queries.append((gi, algo, int(rng.choice(cand))))
    done = serve(gx, graphs, queries, budget=int(per_lane * 64 * 1.1), lanes=64, epoch=2, stagger_s=0.001,
                 dgs=dgs)
    for i, q in enumerate(queries):
        check(gx, graphs, q, done[i])


def test_serving_rejects_budget_below_one_pool(gx, graphs):
    dg = gx.DeviceGraph(graphs[2], gx.GX_NEED_OUT | gx.GX_NEED_IN)
    srv = gx.Server(1 << 16, lanes_per_pool=32)
    gid = srv.add_graph(dg)
    with pytest.raises(gx.GxError) as ei:
        srv.submit(gid, gx.GX_SSSP, 0)
    assert ei.value.status == 2  # GX_ENOMEM
    srv.close()


@pytest.mark.slow
def test_serving_bench_shape_scale16_to_22(gx):
    """The served workload's shape: graphs of scales 16, 17, 18 and 22
    (seeds as in the 16-graph mix), 64-lane pools, up to four pools running
    at once, queries arriving on Poisson gaps while others run, a budget
    that cannot hold every pool at once.  A seeded sample of 16 queries
    (8 SSSP, 8 PPR, at least two of each on the scale-22 graph) is checked
    against the oracle, and four of them against the same query alone."""
    graphs = [gen.rmat(16, seed=100), gen.rmat(17, seed=103), gen.rmat(18, seed=105), gen.rmat(22, seed=114)]
    dgs = [gx.DeviceGraph(g, gx.GX_NEED_OUT | gx.GX_NEED_IN) for g in graphs]
    rng = np.random.default_rng(55)
    queries = []
    for i in range(64):
        gi = 3 if i % 4 == 0 else int(rng.integers(0, 3))
        cand = np.nonzero(np.diff(graphs[gi].row_ptr) > 0)[0]
        # SSSP and PPR alternate in pairs, so the scale-22 queries (every fourth) hold both kinds
        queries.append((gi, 1 if i % 8 < 4 else 3, int(rng.choice(cand))))
    gaps = rng.exponential(0.004, len(queries))
    import ctypes
    pool = {}
    for gi, dg in enumerate(dgs):
        for algo in (gx.GX_SSSP, gx.GX_PPR):
            b = ctypes.c_size_t()
            assert gx.binding.lib.gx_server_bytes_per_lane(dg.handle, algo, ctypes.byref(b)) == 0
            pool[gi, algo] = 64 * b.value
    # room for both scale-22 pools and two of the small ones: not for all eight
    budget = pool[3, gx.GX_SSSP] + pool[3, gx.GX_PPR] + 2 * max(v for k, v in pool.items() if k[0] < 3)
    assert sum(pool.values()) > budget
    done = serve(gx, graphs, queries, budget=budget, lanes=64, epoch=4, max_pools=4, dgs=dgs, gaps=gaps)
    spans = [(c.start_s, c.done_s) for c in done.values()]
    assert any(a0 < b0 < a1 for a0, a1 in spans for b0, _ in spans)
    big = [i for i, q in enumerate(queries) if q[0] == 3]
    sample = [i for i in big if queries[i][1] == 1][:2] + [i for i in big if queries[i][1] == 3][:2]
    rest = [i for i in rng.permutation(len(queries)) if i not in sample]
    sample += [i for i in rest if queries[i][1] == 1][:6] + [i for i in rest if queries[i][1] == 3][:6]
    assert len(sample) == 16
    for i in sample:
        check(gx, graphs, queries[i], done[i], threads=0)
    for i in sample[:2] + sample[4:6]:
        alone = serve(gx, graphs, [queries[i]], budget=budget, lanes=64, epoch=4, dgs=dgs)
        assert np.array_equal(alone[0].result.view(np.uint32), done[i].result.view(np.uint32)), i
