"""Pins of the CPU oracle against results fixed independently of it.

Each check reaches the expected value by a different route than the oracle
(Dijkstra, union-find, BFS, dense LU, closed forms, a hand-worked example,
whole-array relaxation), so a dropped term, a wrong sign, index or operand
order in the oracle fails at least one of them.
"""
import json
import os

import numpy as np
import pytest

import gen
import oracle

INF = oracle.INF
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def random_graph(V, E, seed, wmax=255):
    rng = np.random.default_rng(seed)
    src = rng.integers(0, V, E)
    dst = rng.integers(0, V, E)
    w = rng.integers(1, wmax + 1, E)
    return gen.from_edges(V, src, dst, w)


def load_hand():
    with open(os.path.join(GOLDEN, "hand_sssp_cc_7v.json")) as f:
        h = json.load(f)
    e = np.array(h["edges"])
    g = gen.from_edges(h["V"], e[:, 0], e[:, 1], e[:, 2])
    return h, g


# ---------------------------------------------------------------- hand example

def test_hand_example_sssp():
    h, g = load_hand()
    run = oracle.sssp(g, h["sssp_source"])
    assert run.K == h["sssp_K"]
    assert run.state.tolist() == h["sssp_dist"]
    assert run.msgs.tolist() == h["sssp_messages"]
    dists, fronts = oracle.sssp_frontiers(g, h["sssp_source"])
    assert [np.nonzero(f)[0].tolist() for f in fronts] == h["sssp_frontiers"]
    assert [d.tolist() for d in dists[1:]] == h["sssp_dist_after_step"]


def test_hand_example_cc():
    h, g = load_hand()
    run = oracle.cc(g)
    assert run.state.tolist() == h["cc_labels"]
    assert run.K == h["cc_K"]
    assert run.changed.tolist() == h["cc_changed"]


# ---------------------------------------------------------------- SSSP

SSSP_CASES = [("rand", 40, 120, s) for s in range(6)] + [("rand", 64, 64, 7), ("rand", 50, 400, 8)]


@pytest.mark.parametrize("kind,V,E,seed", SSSP_CASES)
def test_sssp_equals_dijkstra_and_hop_bound(kind, V, E, seed):
    g = random_graph(V, E, seed)
    for s in (0, V // 3):
        run = oracle.sssp(g, s)
        dj, hops = oracle.dijkstra(g, s, with_hops=True)
        assert np.array_equal(run.state, dj)
        reach = hops >= 0
        assert run.K == 1 + int(hops[reach].max())
        # every intermediate state equals the best path of <= k edges
        dists, _ = oracle.sssp_frontiers(g, s)
        for k, dk in enumerate(dists):
            assert np.array_equal(dk, oracle.hop_bounded_distances(g, s, k)), k


@pytest.mark.parametrize("scale,seed", [(10, 1), (12, 2), (14, 5)])
def test_sssp_rmat_dijkstra_and_certificate(scale, seed):
    g = gen.rmat(scale, seed=seed)
    run = oracle.sssp(g, 0)
    dj, hops = oracle.dijkstra(g, 0, with_hops=True)
    assert np.array_equal(run.state, dj)
    assert run.K == 1 + int(hops[hops >= 0].max())
    d = run.state.astype(np.int64)
    src = g.src
    fin = d[src] < INF
    # triangle inequality on every edge out of a reached vertex
    assert np.all(d[g.col[fin]] <= d[src[fin]] + g.w[fin])
    # every reached non-source vertex has a tight in-edge
    tight = np.zeros(g.V, bool)
    t = fin & (d[g.col] == d[src] + g.w)
    tight[g.col[t]] = True
    reached = d < INF
    reached[0] = False
    assert np.all(tight[reached])
    # frontier bookkeeping: |F_{k+1}| of step k is |F| of step k+1
    assert np.array_equal(run.changed[:-1], run.front[1:])
    assert run.changed[-1] == 0
    deg = np.diff(g.row_ptr)
    assert run.msgs[0] == deg[0]


def test_sssp_special_cases():
    # single vertex, no edges
    g = gen.from_edges(1, [], [])
    r = oracle.sssp(g, 0)
    assert r.K == 1 and r.state.tolist() == [0]
    # chain of V vertices: K = V
    V = 9
    g = gen.from_edges(V, np.arange(V - 1), np.arange(1, V), np.arange(1, V))
    r = oracle.sssp(g, 0)
    assert r.K == V
    assert r.state.tolist() == np.cumsum(np.r_[0, np.arange(1, V)]).tolist()
    # saturation: a path whose length exceeds 2^32-1 stays at INF
    g = gen.from_edges(3, [0, 1], [1, 2], [0xFFFFFFF0, 0xFFFFFFF0])
    r = oracle.sssp(g, 0)
    assert r.state.tolist() == [0, 0xFFFFFFF0, INF]
    # unreachable vertices stay INF; the source with no out-edge needs 1 step
    g = gen.from_edges(4, [1, 2], [2, 3], [5, 5])
    r = oracle.sssp(g, 0)
    assert r.K == 1 and r.state.tolist() == [0, INF, INF, INF]


# ---------------------------------------------------------------- CC

@pytest.mark.parametrize("V,E,seed", [(50, 40, 1), (60, 90, 2), (64, 30, 3), (200, 150, 4)])
def test_cc_equals_union_find(V, E, seed):
    g = random_graph(V, E, seed)
    r = oracle.cc(g)
    assert np.array_equal(r.state, oracle.union_find_labels(g))
    assert r.K == 1 + oracle.cc_max_hops(g)


@pytest.mark.parametrize("scale,seed", [(11, 1), (13, 6)])
def test_cc_rmat(scale, seed):
    g = gen.rmat(scale, seed=seed)
    r = oracle.cc(g)
    assert np.array_equal(r.state, oracle.union_find_labels(g))
    assert r.K == 1 + oracle.cc_max_hops(g)


def test_cc_partition_uses_global_ids():
    p = gen.rmat_part(12, seed=3, part=0)
    r = oracle.cc(p)
    uf = oracle.union_find_labels(p)
    assert np.array_equal(r.state, uf)
    # labels are global ids of the component's smallest member
    assert set(np.unique(r.state)).issubset(set(p.l2g.tolist()))
    assert r.K == 1 + oracle.cc_max_hops(p)


# ---------------------------------------------------------------- PageRank

def test_pagerank_mass_and_floor():
    g = gen.rmat(10, seed=3)
    d = 0.85
    _, hist = oracle.pagerank(g, 20, d, history=True)
    for x in hist:
        assert abs(x.sum() - 1.0) < 1e-12
    for x in hist[1:]:
        assert x.min() >= (1 - d) / g.V - 1e-18


def test_pagerank_closed_forms():
    d = 0.85
    # directed cycle: uniform at every step
    V = 7
    g = gen.from_edges(V, np.arange(V), (np.arange(V) + 1) % V)
    x, hist = oracle.pagerank(g, 10, d, history=True)
    for xt in hist:
        assert np.allclose(xt, 1.0 / V, atol=1e-15, rtol=0)
    # no edges: every vertex dangling, uniform at every step
    g = gen.from_edges(5, [], [])
    assert np.allclose(oracle.pagerank(g, 3, d), 0.2, atol=1e-15, rtol=0)
    # two vertices 0 -> 1 (1 dangling): x0_t = x* + (1/2 - x*) (-d/2)^t,
    # x* = 1/(2+d) (solved by hand from the fixed point)
    g = gen.from_edges(2, [0], [1])
    _, hist = oracle.pagerank(g, 12, d, history=True)
    xs = 1.0 / (2.0 + d)
    for t, xt in enumerate(hist):
        x0 = xs + (0.5 - xs) * (-d / 2) ** t
        assert abs(xt[0] - x0) < 1e-14 and abs(xt[1] - (1 - x0)) < 1e-14


@pytest.mark.parametrize("V,E,seed", [(30, 60, 1), (80, 150, 2), (200, 900, 3), (300, 250, 4)])
def test_pagerank_fixed_point_dense_lu(V, E, seed):
    g = random_graph(V, E, seed)
    x = oracle.pagerank(g, 300, 0.85)
    ref = oracle.pagerank_fixed_point_dense(g, 0.85)
    assert np.max(np.abs(x - ref)) < 1e-12


def test_pagerank_fixed_point_rmat():
    g = gen.rmat(9, seed=11)
    x = oracle.pagerank(g, 300, 0.85)
    ref = oracle.pagerank_fixed_point_dense(g, 0.85)
    assert np.max(np.abs(x - ref)) < 1e-12


@pytest.mark.parametrize("V,E,seed", [(40, 80, 5), (120, 200, 6)])
def test_ppr_fixed_point_dense_lu(V, E, seed):
    g = random_graph(V, E, seed)
    s = 3
    x, hist = oracle.ppr(g, s, 400, 0.85, history=True)
    for xt in hist:
        assert abs(xt.sum() - 1.0) < 1e-12
    ref = oracle.ppr_fixed_point_dense(g, s, 0.85)
    assert np.max(np.abs(x - ref)) < 1e-12


def test_ppr_star_closed_form():
    # star 0 -> 1..n, leaves dangling; seed 0.  Fixed point by hand:
    # x0 = (1-d) + d * L, each leaf = d * x0 / n, L = n * leaf = d x0
    # => x0 = (1-d) / (1 - d^2) = 1/(1+d), leaf = d / (n (1+d)).
    n, d = 6, 0.85
    g = gen.from_edges(n + 1, np.zeros(n, int), np.arange(1, n + 1))
    x = oracle.ppr(g, 0, 400, d)
    assert abs(x[0] - 1 / (1 + d)) < 1e-13
    assert np.allclose(x[1:], d / (n * (1 + d)), atol=1e-13, rtol=0)


# ---------------------------------------------------------------- sync set

def test_delta_sets_follow_state_changes():
    p = gen.rmat_part(12, seed=3, part=0)
    rem = oracle.remote_mask(p, "cc")
    assert rem.sum() > 0
    # CC superstep by superstep; delta of each step = changed & remote
    lab = p.l2g.astype(np.uint32).copy()
    synced = lab.copy()
    front = np.zeros(p.V, bool)
    front[np.unique(np.r_[p.src, p.col])] = True
    skipped = 0
    for _ in range(100):
        new, nf = oracle.min_superstep(p, lab, front, weighted=False, both_dirs=True)
        gids, vals, skip = oracle.delta(p, rem, new, synced)
        want = np.nonzero(nf & (rem != 0))[0]
        assert gids.tolist() == p.l2g[want].tolist()
        assert vals.tolist() == new[want].tolist()
        assert np.all(np.diff(gids) > 0)
        skipped += skip
        lab, front = new, nf
        if not nf.any():
            break
    # after the last upload the remote copies equal the final state
    assert np.array_equal(synced[rem != 0], lab[rem != 0])
    # a pass with no change has an empty set (skippable)
    gids, _, skip = oracle.delta(p, rem, lab, synced)
    assert skip and len(gids) == 0


def test_delta_lazy_keeps_only_final_value():
    p = gen.rmat_part(11, seed=3, part=0)
    rem = oracle.remote_mask(p, "pr")
    x0 = np.full(p.V, 1.0 / p.V, np.float32)
    synced = x0.view(np.uint32).copy()
    x5 = oracle.pagerank(p, 5).astype(np.float32)
    gids, vals, _ = oracle.delta(p, rem, x5, synced)
    changed = (x5.view(np.uint32) != x0.view(np.uint32)) & (rem != 0)
    assert gids.tolist() == p.l2g[changed].tolist()
    assert vals.tolist() == x5.view(np.uint32)[changed].tolist()


# ---------------------------------------------------------------- OpenMP timing mode

@pytest.mark.parametrize("threads", [2, 0])
@pytest.mark.parametrize("scale,seed", [(10, 1), (14, 3)])
def test_openmp_mode_equals_reference_bitwise(scale, seed, threads):
    """The timing mode on several threads gives the single-threaded
    reference's results bit for bit: SSSP and CC values and every
    superstep's counters, PageRank and PPR float64 values."""
    g = gen.rmat(scale, seed=seed)
    a, b = oracle.sssp(g, 0), oracle.sssp(g, 0, threads=threads)
    assert a.K == b.K and np.array_equal(a.state, b.state)
    for f in ("front", "msgs", "changed"):
        assert np.array_equal(getattr(a, f), getattr(b, f)), f
    p = gen.rmat_part(scale, seed=seed, part=1)
    a, b = oracle.cc(p), oracle.cc(p, threads=threads)
    assert a.K == b.K and np.array_equal(a.state, b.state) and np.array_equal(a.changed, b.changed)
    x1, x2 = oracle.pagerank(g, 12), oracle.pagerank(g, 12, threads=threads)
    assert np.array_equal(x1.view(np.uint64), x2.view(np.uint64))
    s = int(np.argmax(np.diff(g.row_ptr)))
    y1, y2 = oracle.ppr(g, s, 15), oracle.ppr(g, s, 15, threads=threads)
    assert np.array_equal(y1.view(np.uint64), y2.view(np.uint64))


def test_openmp_many_sources_equal_single_runs():
    g = gen.rmat(11, seed=4)
    srcs = gen.pick_sources(g, 24, seed=40)
    D, K = oracle.sssp_many(g, srcs)
    J = oracle.dijkstra_many(g, srcs, threads=3)
    for b, s in enumerate(srcs):
        r = oracle.sssp(g, int(s))
        assert np.array_equal(D[b], r.state) and K[b] == r.K
        assert np.array_equal(J[b], r.state)
    X = oracle.ppr_many(g, srcs[:6], 20)
    for b in range(6):
        assert np.array_equal(X[b].view(np.uint64), oracle.ppr(g, int(srcs[b]), 20).view(np.uint64))


# ---------------------------------------------------------------- label propagation

def _undirected(V, pairs):
    e = np.array(pairs, dtype=np.int64).reshape(-1, 2)
    return gen.from_edges(V, e[:, 0], e[:, 1], np.ones(len(e), np.int64))


def test_hand_example_lp():
    with open(os.path.join(GOLDEN, "hand_lp_8v.json")) as f:
        h = json.load(f)
    g = _undirected(h["V"], h["edges"])
    steps = oracle.lp_steps(g)
    assert [s.tolist() for s in steps[1:]] == h["labels_after_iteration"]
    run = oracle.lp(g, 15)
    assert run.K == h["K"] and run.changed.tolist() == h["changed"]
    assert run.state.tolist() == h["labels_after_iteration"][-1]


@pytest.mark.parametrize("n", [3, 4, 7])
def test_lp_complete_graph(n):
    # iteration 1: vertex 0 sees ids 1..n-1 once each -> 1; every other
    # vertex sees 0 among its distinct ids -> 0.  Iteration 2: 0 is the
    # majority (or the smaller of a 1-1 tie at n = 3) everywhere.
    g = _undirected(n, [(i, j) for i in range(n) for j in range(i + 1, n)])
    steps = oracle.lp_steps(g)
    assert steps[1].tolist() == [1] + [0] * (n - 1)
    assert steps[2].tolist() == [0] * n
    run = oracle.lp(g)
    assert run.K == 3 and run.changed.tolist() == [n, 1, 0]


@pytest.mark.parametrize("m", [2, 5])
def test_lp_star_oscillates_to_the_cap(m):
    # the hub takes the smallest leaf id, the leaves the hub's label, and the
    # two sides swap every iteration: after an odd count, hub 1 and leaves 0
    g = _undirected(m + 1, [(0, j) for j in range(1, m + 1)])
    run = oracle.lp(g, 15)
    assert run.K == -1
    assert run.state.tolist() == [1] + [0] * m
    assert run.changed.tolist() == [m + 1] * 15
    assert oracle.lp(g, 4).state.tolist() == [0] + [1] * m


def test_lp_path_first_iteration():
    n = 9
    g = _undirected(n, [(i, i + 1) for i in range(n - 1)])
    assert oracle.lp_steps(g, 1)[1].tolist() == [1] + list(range(0, n - 2)) + [n - 2]


def test_lp_degenerate_cases():
    # no edges: every label stays, one iteration that changes nothing
    g = gen.from_edges(5, np.array([], np.int64), np.array([], np.int64), np.array([], np.int64))
    run = oracle.lp(g)
    assert run.K == 1 and run.state.tolist() == list(range(5))
    # self-loops carry nothing, duplicates count once: the same as the clean graph
    clean = _undirected(4, [(0, 1), (1, 2), (2, 3)])
    dirty = _undirected(4, [(0, 1), (1, 0), (0, 1), (1, 2), (2, 3), (3, 3), (2, 2), (3, 2)])
    for a, b in zip(oracle.lp_steps(clean), oracle.lp_steps(dirty)):
        assert np.array_equal(a, b)
    # two disjoint cliques settle on their smallest ids
    pairs = [(i, j) for i in range(4) for j in range(i + 1, 4)] + \
            [(i, j) for i in range(4, 9) for j in range(i + 1, 9)]
    assert oracle.lp(_undirected(9, pairs)).state.tolist() == [0] * 4 + [4] * 5


def test_lp_partition_starts_from_global_ids():
    p = gen.rmat_part(10, seed=3, part=2)
    steps = oracle.lp_steps(p, 1)
    assert np.array_equal(steps[0], p.l2g.astype(np.uint32))
    # every new label is a global id of a neighbour (or the vertex's own, when isolated)
    assert np.isin(steps[1], p.l2g).all()


@pytest.mark.parametrize("seed", [0, 1])
def test_lp_certificate_random(seed):
    """Every label after an iteration occurs among the neighbours' labels of
    the iteration before at least as often as any other, and no smaller
    label occurs as often (counted with Python dictionaries over a
    numpy-built neighbour set)."""
    rng = np.random.default_rng(seed)
    V = 60
    src, dst = rng.integers(0, V, 200), rng.integers(0, V, 200)
    g = gen.from_edges(V, src, dst, np.ones(200, np.int64))
    nbrs = [set() for _ in range(V)]
    for u, v in zip(src, dst):
        if u != v:
            nbrs[u].add(int(v))
            nbrs[v].add(int(u))
    steps = oracle.lp_steps(g, 15)
    for old, new in zip(steps[:-1], steps[1:]):
        for v in range(V):
            if not nbrs[v]:
                assert new[v] == old[v]
                continue
            cnt = {}
            for u in nbrs[v]:
                cnt[int(old[u])] = cnt.get(int(old[u]), 0) + 1
            top = max(cnt.values())
            assert cnt.get(int(new[v]), 0) == top
            assert all(lab >= new[v] for lab, c in cnt.items() if c == top)


# ---------------------------------------------------------------- pipeline block size

def test_pipeline_hand_example():
    # d = 12, k1 = k3 = 1, k2 = 2, a = 4, worked by hand from the equation:
    # s=2 (b=6): 6+16+0+16+6 = 44; s=3 (b=4): 4+12+12+12+4 = 44;
    # s=4 (b=3): 3+10+20+10+3 = 46; s=5 (b=2.4): 48.8; s=6 (b=2): 52
    t = oracle.pipeline_time(1, 2, 1, 4, 12, [2, 3, 4, 5, 6])
    assert np.allclose(t, [44, 44, 46, 48.8, 52])
    assert oracle.pipeline_brute_force(1, 2, 1, 4, 12) == (2, 44.0)


def test_pipeline_lemma_closed_forms():
    # computation dominant (k2 largest): b = Q = sqrt(a d / (k1 + k3)),
    # T = k2 d + 2 sqrt((k1 + k3) a d): k = (1, 3, 1), a = 2, d = 100 -> Q = 10
    assert oracle.pipeline_brute_force(1, 3, 1, 2, 100) == (10, 340.0)
    # download dominant with a / (k1 - k2) < Q: b = a / (k1 - k2) = 5,
    # T = k1 d + (k1 + k3) a / (k1 - k2) = 400 + 25
    s, t = oracle.pipeline_brute_force(4, 2, 1, 10, 100)
    assert (s, round(t, 9)) == (20, 425.0)
    # upload dominant: the same with k1 and k3 swapped, T = k3 d + (k1 + k3) a / (k3 - k2)
    # (the Lemma's case (iii) prints k1 d; the equation gives k3 d = 400 here)
    s, t = oracle.pipeline_brute_force(1, 2, 4, 10, 100)
    assert (s, round(t, 9)) == (20, 425.0)


def test_pipeline_degenerate_forms():
    # no per-call cost: more blocks always hide more, T = k1 d + (k2 + k3) d / s
    s, t = oracle.pipeline_brute_force(3, 2, 1, 0.0, 50)
    assert s == 50 and abs(t - (3 * 50 + 3 * 50 / 50)) < 1e-9
    # no transfers: T = s a + k2 d, fewest blocks
    s, t = oracle.pipeline_brute_force(0.0, 2, 0.0, 5, 40)
    assert s == 2 and abs(t - (2 * 5 + 2 * 40)) < 1e-9


# ---------------------------------------------------------------- workload balancing

def test_balance_brute_force_pins():
    # equal costs: the even split, value c D / m
    split, v = oracle.balance_brute_force([2.0, 2.0], 10)
    assert sorted(split) == [5, 5] and v == 10.0
    # costs 1 and 3 over D = 8: d = (6, 2), both nodes at 6 (the Lemma's D / (1 + 1/3) = 6)
    split, v = oracle.balance_brute_force([1.0, 3.0], 8)
    assert split == [6, 2] and v == 6.0
    # three nodes 1, 2, 4 over D = 7: (4, 2, 1), every node at 4 = D / (1 + 1/2 + 1/4)
    split, v = oracle.balance_brute_force([1.0, 2.0, 4.0], 7)
    assert split == [4, 2, 1] and v == 4.0
    # no split does better than the Lemma's value, and integers cost at most one entity's time
    rng = np.random.default_rng(3)
    for _ in range(20):
        c = rng.uniform(0.5, 5.0, int(rng.integers(2, 4)))
        D = int(rng.integers(1, 25))
        _, v = oracle.balance_brute_force(c, D)
        lemma = D / np.sum(1.0 / c)
        assert lemma - 1e-12 <= v <= lemma + c.max() + 1e-12
