"""Parity of the HIP superstep engine with the CPU oracle (runs on MI355X).

SSSP distances, CC labels, frontiers, superstep counts and sync sets must
match the oracle bit for bit; PageRank must stay within max-abs 1e-6 of the
float64 oracle (float32 on the device).
"""
import json
import os

import numpy as np
import pytest

import gen
import oracle

pytestmark = pytest.mark.gpu

PR_TOL = 1e-6
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def gx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2203_13005_amd as m
    return m


def load(gx, g, needs=None):
    if needs is None:
        needs = gx.GX_NEED_OUT | gx.GX_NEED_IN | gx.GX_NEED_SYM
    return gx.DeviceGraph(g, needs)


def random_graph(V, E, seed):
    rng = np.random.default_rng(seed)
    return gen.from_edges(V, rng.integers(0, V, E), rng.integers(0, V, E), rng.integers(1, 256, E))


def star_into(V, hub=0):
    src = np.arange(V)
    src = src[src != hub]
    return gen.from_edges(V, src, np.full(len(src), hub), (src % 255) + 1)


# ------------------------------------------------------------------ SSSP

# pull_fraction: 1.0 = always push, 1e-9 = pull whenever a message exists,
# 0 = the default switch point
MODES = [1.0, 1e-9, 0.0]


def test_pull_reports_mixed_xcd_rotations(gx, monkeypatch):
    """A pull workgroup takes the slice of the XCD it runs on, assuming the
    hardware deals a launch's workgroups to the 8 XCDs in turn from some
    starting XCD; each records the rotation it sees and the host fails the
    superstep if one launch saw two (every other pulling test passes that
    check).  Offsetting the odd workgroups' XCD from the host makes every pull
    superstep see two rotations: the run fails with GX_EDEVICE and the state
    stays failed, while a push-only state and an unshifted state give the
    oracle's distances."""
    g = gen.rmat(12, seed=3)
    dg = load(gx, g, gx.GX_NEED_OUT)
    ref = oracle.sssp(g, 0)
    monkeypatch.setenv("GX_XCD_CHECK_SHIFT", "1")
    st = gx.State(dg, gx.GX_SSSP, source=0, pull_fraction=1e-9)
    with pytest.raises(gx.GxError) as ei:
        st.run(10_000)
    assert ei.value.status == gx.binding.GX_EDEVICE and "rotation" in str(ei.value)
    with pytest.raises(gx.GxError):
        st.superstep()
    st.close()
    push = gx.State(dg, gx.GX_SSSP, source=0, pull_fraction=1.0)
    push.run(10_000)
    assert np.array_equal(push.values_numpy(), ref.state)
    push.close()
    monkeypatch.delenv("GX_XCD_CHECK_SHIFT")
    ok = gx.State(dg, gx.GX_SSSP, source=0, pull_fraction=1e-9)
    ok.run(10_000)
    assert np.array_equal(ok.values_numpy(), ref.state)
    ok.close()


def check_sssp_stepwise(gx, g, s, pull_fraction=0.0):
    dg = load(gx, g, gx.GX_NEED_OUT)
    st = gx.State(dg, gx.GX_SSSP, source=s, pull_fraction=pull_fraction)
    dists, fronts = oracle.sssp_frontiers(g, s)
    deg = np.diff(g.row_ptr)
    for k in range(1, len(dists)):
        f_prev = fronts[k - 1]
        fr, edges, changed = st.superstep(stats=True)
        assert fr == f_prev.sum(), k
        assert edges == deg[f_prev].sum(), k
        assert changed == fronts[k].sum(), k
        assert np.array_equal(st.values_numpy(), dists[k]), k
        assert np.array_equal(st.frontier_numpy(), fronts[k]), k
    return st


def test_sssp_hand_example(gx):
    h = json.load(open(os.path.join(GOLDEN, "hand_sssp_cc_7v.json")))
    e = np.array(h["edges"])
    g = gen.from_edges(h["V"], e[:, 0], e[:, 1], e[:, 2])
    st = check_sssp_stepwise(gx, g, 0)
    assert st.values_numpy().tolist() == h["sssp_dist"]
    st2 = gx.State(load(gx, g, gx.GX_NEED_OUT), gx.GX_SSSP, source=0)
    rs, steps = st2.run(100, per_step=True)
    assert rs.supersteps == h["sssp_K"] and rs.converged == 1
    assert [s[1] for s in steps] == h["sssp_messages"]


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("V,E,seed", [(64, 200, 1), (300, 3000, 2), (1000, 500, 3), (5000, 40000, 4)])
def test_sssp_random_stepwise(gx, V, E, seed, mode):
    g = random_graph(V, E, seed)
    check_sssp_stepwise(gx, g, 0, mode)


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("scale,seed", [(12, 1), (16, 2), (18, 3)])
def test_sssp_rmat_against_oracle(gx, scale, seed, mode):
    g = gen.rmat(scale, seed=seed)
    ref = oracle.sssp(g, 0)
    st = gx.State(load(gx, g, gx.GX_NEED_OUT), gx.GX_SSSP, source=0, pull_fraction=mode)
    rs, steps = st.run(10_000, per_step=True)
    assert rs.supersteps == ref.K
    assert np.array_equal(st.values_numpy(), ref.state)
    steps = np.array(steps)
    assert np.array_equal(steps[:, 0], ref.front)
    assert np.array_equal(steps[:, 1], ref.msgs)
    assert np.array_equal(steps[:, 2], ref.changed)


@pytest.mark.parametrize("mode", MODES)
def test_sssp_hub_spanning_many_tiles(gx, mode):
    # vertex 0 has 20000 out-edges (10 push tiles); a chain hangs off it
    V = 20001
    src = np.r_[np.zeros(V - 1, int), np.arange(1, 200)]
    dst = np.r_[np.arange(1, V), np.arange(2, 201)]
    w = np.r_[np.full(V - 1, 255), np.ones(199, int)]
    g = gen.from_edges(V, src, dst, w)
    check_sssp_stepwise(gx, g, 0, mode)


@pytest.mark.parametrize("mode", MODES)
def test_sssp_in_hub_spanning_many_pull_tiles(gx, mode):
    # vertex 5 has in-degree 9000 (crosses five 2048-edge pull tiles) and the
    # sources reach it at different supersteps
    V = 9002
    src = np.r_[np.arange(6, V), np.zeros(V - 6, int), [0, 1, 2, 3], [1, 2, 3, 4]]
    dst = np.r_[np.full(V - 6, 5), np.arange(6, V), [1, 2, 3, 4], [5, 5, 5, 5]]
    w = np.r_[np.full(V - 6, 7), (np.arange(V - 6) % 255) + 1, [1, 1, 1, 1], [200, 100, 50, 1]]
    g = gen.from_edges(V, src, dst, w)
    check_sssp_stepwise(gx, g, 0, mode)


@pytest.mark.parametrize("mode", [1e-9, 0.0])
def test_sssp_pull_rmat20(gx, mode):
    # scale 20: 16384 destination blocks dealt over the XCD slices
    g = gen.rmat(20, seed=5)
    ref = oracle.sssp(g, 0)
    st = gx.State(load(gx, g, gx.GX_NEED_OUT), gx.GX_SSSP, source=0, pull_fraction=mode)
    rs, steps = st.run(10_000, per_step=True)
    assert rs.supersteps == ref.K
    assert np.array_equal(st.values_numpy(), ref.state)
    steps = np.array(steps)
    assert np.array_equal(steps[:, 1], ref.msgs)
    assert np.array_equal(steps[:, 2], ref.changed)


@pytest.mark.parametrize("mode", [1e-9, 0.0])
def test_sssp_pull_large_distances(gx, mode):
    # a weight-255 chain of 2000 vertices with leaves hanging off it:
    # distances reach ~5e5 and some vertices stay unreached
    L, leaves = 2000, 30000
    rng = np.random.default_rng(11)
    V = L + leaves
    chain_s, chain_d = np.arange(L - 1), np.arange(1, L)
    ls = rng.integers(0, L, 4 * leaves)
    ld = rng.integers(L, V, 4 * leaves)
    xs, xd = rng.integers(L, V, leaves), rng.integers(L, V, leaves)
    src = np.r_[chain_s, ls, xs]
    dst = np.r_[chain_d, ld, xd]
    w = np.r_[np.full(L - 1, 255), rng.integers(1, 256, 4 * leaves), rng.integers(1, 256, leaves)]
    g = gen.from_edges(V, src, dst, w)
    ref = oracle.sssp(g, 0)
    assert ref.state[L - 1] == 255 * (L - 1)
    st = gx.State(load(gx, g, gx.GX_NEED_OUT), gx.GX_SSSP, source=0, pull_fraction=mode)
    rs, steps = st.run(100_000, per_step=True)
    assert rs.supersteps == ref.K
    assert np.array_equal(st.values_numpy(), ref.state)
    steps = np.array(steps)
    assert np.array_equal(steps[:, 2], ref.changed)


@pytest.mark.parametrize("mode", [1e-9, 0.0])
def test_sssp_pull_racing_stores_on_hubs(gx, mode):
    # Three hubs each receive an in-edge from every vertex: their records
    # spread over ~49 source bands, so many pull work units store candidates
    # for one hub at once; the fix-up pass must leave the minimum.  Weights
    # are chosen so the best candidate is rare and arrives in the same
    # superstep as many worse ones.
    V = 200_000
    rng = np.random.default_rng(23)
    hubs = np.array([7, 100_003, 199_998])
    src, dst, w = [], [], []
    for h in hubs:
        s_ = np.arange(V)
        s_ = s_[s_ != h]
        src.append(s_)
        dst.append(np.full(len(s_), h))
        w.append(rng.integers(1, 256, len(s_)))
    # a random sparse layer so the sources get distinct distances
    rs = rng.integers(0, V, 4 * V)
    rd = rng.integers(0, V, 4 * V)
    src.append(rs); dst.append(rd); w.append(rng.integers(1, 256, 4 * V))
    g = gen.from_edges(V, np.concatenate(src), np.concatenate(dst), np.concatenate(w))
    check_sssp_stepwise(gx, g, 0, mode)


def test_cc_pull_racing_stores_on_hubs(gx):
    V = 150_000
    rng = np.random.default_rng(29)
    hub = 120_000
    s_ = np.arange(V)
    s_ = s_[s_ != hub]
    src = np.r_[s_, rng.integers(0, V, V)]
    dst = np.r_[np.full(len(s_), hub), rng.integers(0, V, V)]
    g = gen.from_edges(V, src, dst)
    ref = oracle.cc(g)
    st = gx.State(load(gx, g, gx.GX_NEED_SYM), gx.GX_CC, pull_fraction=1e-9)
    rs, _ = st.run(10_000)
    assert rs.supersteps == ref.K
    assert np.array_equal(st.values_numpy(), ref.state)


def test_sssp_edge_cases(gx):
    g = gen.from_edges(1, [], [])
    st = gx.State(load(gx, g, gx.GX_NEED_OUT), gx.GX_SSSP, source=0)
    rs, _ = st.run(10)
    assert rs.supersteps == 1 and st.values_numpy().tolist() == [0]
    # source without out-edges; others unreachable
    g = gen.from_edges(40, [1, 2], [2, 3], [5, 5])
    st = gx.State(load(gx, g, gx.GX_NEED_OUT), gx.GX_SSSP, source=0)
    rs, _ = st.run(10)
    assert rs.supersteps == 1
    assert st.values_numpy().tolist() == [0] + [gx.INF] * 39
    # superstep cap: a chain needs V supersteps
    V = 50
    g = gen.from_edges(V, np.arange(V - 1), np.arange(1, V), np.ones(V - 1, int))
    st = gx.State(load(gx, g, gx.GX_NEED_OUT), gx.GX_SSSP, source=0)
    with pytest.raises(gx.GxError) as ei:
        st.run(10)
    assert ei.value.status == 4  # GX_ENOTCONVERGED, state valid
    d = st.values_numpy()
    assert d[:11].tolist() == list(range(11)) and np.all(d[11:] == gx.INF)
    rs, _ = st.run(100)  # resume to convergence
    assert st.values_numpy().tolist() == list(range(V))


@pytest.mark.parametrize("mode", MODES)
def test_sssp_wide_weights_push_only(gx, mode):
    # weights beyond 8 bits: the banded pull records cannot hold them, so
    # every superstep pushes whatever the switch point asks for; sums that
    # overflow 32 bits saturate at INF (unreachable) on both sides
    V, E = 5000, 30000
    rng = np.random.default_rng(21)
    src = np.r_[rng.integers(0, V, E), np.arange(100)]
    dst = np.r_[rng.integers(0, V, E), np.arange(1, 101)]
    w = np.r_[rng.integers(1, 1 << 31, E), np.full(100, 0x7FFFFFF0)]
    g = gen.from_edges(V, src, dst, w)
    st = check_sssp_stepwise(gx, g, 0, pull_fraction=mode)
    ref = oracle.sssp(g, 0)
    d = st.values_numpy()
    assert np.array_equal(d, ref.state)
    assert (d == gx.INF).sum() > 0 and d[d != gx.INF].max() > 1 << 31
    st = gx.State(load(gx, g, gx.GX_NEED_OUT), gx.GX_SSSP, source=0, pull_fraction=mode)
    rs, steps = st.run(10_000, per_step=True, detail=True)
    assert rs.supersteps == ref.K and not any(x["pulled"] for x in steps)
    assert np.array_equal(st.values_numpy(), ref.state)


def test_vertex_ids_beyond_24_bits(gx):
    # V > 2^24: destination ids and source bands above 2^24 in the pull
    # records of both SSSP (sources stored relative to their band next to an
    # 8-bit weight) and CC, checked superstep by superstep for SSSP
    V = (1 << 24) + 37
    rng = np.random.default_rng(5)
    hi = rng.integers(V - 3000, V, 20000)
    src = np.r_[rng.integers(0, V, 150_000), hi, np.zeros(2000, int)]
    dst = np.r_[rng.integers(0, V, 150_000), rng.permutation(hi), rng.integers(V - 3000, V, 2000)]
    g = gen.from_edges(V, src, dst, rng.integers(1, 256, len(src)))
    dg = load(gx, g, gx.GX_NEED_OUT | gx.GX_NEED_SYM)
    ref = oracle.sssp(g, 0)
    st = gx.State(dg, gx.GX_SSSP, source=0, pull_fraction=1e-9)
    rs, steps = st.run(10_000, per_step=True, detail=True)
    assert rs.supersteps == ref.K and all(x["pulled"] for x in steps if x["edges"] > 0)
    assert np.array_equal(st.values_numpy(), ref.state)
    del st
    check_sssp_stepwise(gx, g, 0, pull_fraction=1e-9)
    ref = oracle.cc(g)
    st = gx.State(dg, gx.GX_CC, pull_fraction=1e-9)
    rs, steps = st.run(10_000, per_step=True, detail=True)
    assert rs.supersteps == ref.K and any(x["pulled"] for x in steps)
    assert np.array_equal(st.values_numpy(), ref.state)


def test_sssp_deterministic_rerun(gx):
    g = gen.rmat(16, seed=9)
    dg = load(gx, g, gx.GX_NEED_OUT)
    outs = []
    for _ in range(2):
        st = gx.State(dg, gx.GX_SSSP, source=0)
        st.run(10_000)
        outs.append(st.values_numpy())
    assert np.array_equal(outs[0], outs[1])


# ------------------------------------------------------------------ CC

@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("V,E,seed", [(64, 50, 1), (500, 400, 2), (3000, 2500, 3), (20000, 60000, 4)])
def test_cc_random(gx, V, E, seed, mode):
    g = random_graph(V, E, seed)
    ref = oracle.cc(g)
    st = gx.State(load(gx, g, gx.GX_NEED_SYM), gx.GX_CC, pull_fraction=mode)
    rs, steps = st.run(10_000, per_step=True)
    assert np.array_equal(st.values_numpy(), ref.state)
    assert rs.supersteps == ref.K
    steps = np.array(steps)
    assert np.array_equal(steps[:, 0], ref.front)
    assert np.array_equal(steps[:, 2], ref.changed)


def test_cc_hand_example(gx):
    h = json.load(open(os.path.join(GOLDEN, "hand_sssp_cc_7v.json")))
    e = np.array(h["edges"])
    g = gen.from_edges(h["V"], e[:, 0], e[:, 1], e[:, 2])
    st = gx.State(load(gx, g, gx.GX_NEED_SYM), gx.GX_CC)
    rs, steps = st.run(100, per_step=True)
    assert st.values_numpy().tolist() == h["cc_labels"]
    assert rs.supersteps == h["cc_K"]
    assert [s[2] for s in steps] == h["cc_changed"]


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("scale,seed", [(14, 3), (17, 5)])
def test_cc_rmat_partition(gx, scale, seed, mode):
    p = gen.rmat_part(scale, seed=seed, part=0)
    ref = oracle.cc(p)
    st = gx.State(load(gx, p, gx.GX_NEED_SYM), gx.GX_CC, pull_fraction=mode)
    rs, steps = st.run(10_000, per_step=True)
    assert np.array_equal(st.values_numpy(), ref.state)
    assert rs.supersteps == ref.K
    assert np.array_equal(np.array(steps)[:, 2], ref.changed)


# ------------------------------------------------------------------ PageRank

def check_pr(gx, g, T, d=0.85, tol=PR_TOL, tile=0):
    ref = oracle.pagerank(g, T, d)
    st = gx.State(gx.DeviceGraph(g, gx.GX_NEED_IN, pr_tile_edges=tile), gx.GX_PAGERANK, damping=d)
    rs, steps = st.run(T, per_step=True)
    x = st.values_numpy().astype(np.float64)
    err = np.max(np.abs(x - ref)) if g.V else 0.0
    assert err <= tol, err
    assert rs.supersteps == T and all(s[0] == g.V and s[1] == g.E for s in steps)
    return st, x, ref


def test_pagerank_rmat_scale14_20_steps(gx):
    g = gen.rmat(14, seed=1)
    st, x, ref = check_pr(gx, g, 20)
    rel = np.max(np.abs(x - ref) / ref)
    assert rel < 1e-4


def test_pagerank_graph_replay_equals_eager(gx):
    """A PageRank run without timing events is captured once as a HIP graph
    and replayed, also after a reset (the state re-created in the same
    memory).  Every replay, with other eager device work in between, equals
    the run enqueued superstep by superstep (timing events on) bit for bit,
    per-superstep counts included, and so does a run that continues from
    superstep 20 (another ring slot: another graph)."""
    g = gen.rmat(12, seed=7)
    dg = gx.DeviceGraph(g, gx.GX_NEED_IN)
    eager = gx.State(dg, gx.GX_PAGERANK, damping=0.85, timing=True)
    _, s20 = eager.run(20, per_step=True)
    e20 = eager.values_numpy().view(np.uint32).copy()
    _, s40 = eager.run(20, per_step=True)
    e40 = eager.values_numpy().view(np.uint32).copy()
    eager.close()
    st = gx.State(dg, gx.GX_PAGERANK, damping=0.85)
    for rep in range(4):
        st.reset()
        _, steps = st.run(20, per_step=True)
        assert np.array_equal(st.values_numpy().view(np.uint32), e20), rep
        assert steps == s20, rep
        other = gx.State(dg, gx.GX_PAGERANK, damping=0.85, timing=True)
        other.run(3)
        other.close()
    _, steps = st.run(20, per_step=True)
    assert np.array_equal(st.values_numpy().view(np.uint32), e40)
    assert steps == s40
    ref = oracle.pagerank(g, 40)
    assert np.max(np.abs(st.values_numpy().astype(np.float64) - ref)) <= PR_TOL
    st.close()


PR_TILES = [0, 256, 512, 1024, 2048]  # 0 = the size the library picks


@pytest.mark.parametrize("tile", PR_TILES)
@pytest.mark.parametrize("V,E,seed", [(50, 100, 1), (3000, 9000, 2), (10000, 300, 3)])
def test_pagerank_random(gx, V, E, seed, tile):
    check_pr(gx, random_graph(V, E, seed), 15, tile=tile)


@pytest.mark.parametrize("tile", PR_TILES)
def test_pagerank_hub_rows_span_tiles(gx, tile):
    # in-degree 9000 at vertex 0 and 3000 at vertex 1: rows cross several
    # tiles; plus rows ending exactly on a tile boundary
    V = 9001
    src = np.r_[np.arange(1, V), np.arange(2, 3002)]
    dst = np.r_[np.zeros(V - 1, int), np.ones(3000, int)]
    g = gen.from_edges(V, src, dst)
    check_pr(gx, g, 10, tile=tile)
    g = star_into(2049)  # E = 2048: a whole number of tiles of every size
    check_pr(gx, g, 10, tile=tile)
    g = star_into(4097, hub=4096)  # E = 4096, the hub is the last row
    check_pr(gx, g, 10, tile=tile)


@pytest.mark.parametrize("tile", PR_TILES)
def test_pagerank_edge_cases(gx, tile):
    check_pr(gx, gen.from_edges(1, [], []), 5, tile=tile)
    check_pr(gx, gen.from_edges(7, [], []), 5, tile=tile)
    g = gen.from_edges(2, [0], [1])
    check_pr(gx, g, 12, tile=tile)


def test_pagerank_fix_over_many_workgroups(gx):
    # 256-edge tiles: thousands of tiles, so the crossing rows are completed
    # by many fix-up workgroups (256 tiles each); the hub's row starts in the
    # first workgroup's range and ends in the second's, and a second hub
    # crosses the next boundary; results stay bitwise reproducible
    V = 200_000
    rng = np.random.default_rng(11)
    src = np.r_[rng.integers(0, V, 600_000), np.arange(2, 70_002), np.arange(3, 30_003)]
    dst = np.r_[rng.integers(0, V, 600_000), np.full(70_000, 40), np.full(30_000, 150_000)]
    g = gen.from_edges(V, src, dst)
    st, x, ref = check_pr(gx, g, 12, tile=256)
    st2, x2, _ = check_pr(gx, g, 12, tile=256)
    assert np.array_equal(x.view(np.uint64), x2.view(np.uint64))
    g = gen.rmat(16, seed=6)
    check_pr(gx, g, 10, tile=256)


@pytest.mark.parametrize("tile", [0, 2048])
def test_pagerank_deterministic_and_checkpoint(gx, tile):
    g = gen.rmat(15, seed=4)
    dg = gx.DeviceGraph(g, gx.GX_NEED_IN, pr_tile_edges=tile)
    a = gx.State(dg, gx.GX_PAGERANK)
    a.run(20)
    b = gx.State(dg, gx.GX_PAGERANK)
    b.run(20)
    assert np.array_equal(a.values_numpy().view(np.uint32), b.values_numpy().view(np.uint32))
    c = gx.State(dg, gx.GX_PAGERANK)
    c.run(7)
    c.run(13)
    assert np.array_equal(a.values_numpy().view(np.uint32), c.values_numpy().view(np.uint32))


# ------------------------------------------------------------------ sync set

@pytest.mark.parametrize("mode", [1.0, 1e-9])
def test_sync_delta_cc_partition(gx, mode):
    p = gen.rmat_part(14, seed=3, part=0)
    rem = oracle.remote_mask(p, "cc")
    st = gx.State(load(gx, p, gx.GX_NEED_SYM), gx.GX_CC, pull_fraction=mode)
    lab = p.l2g.astype(np.uint32).copy()
    synced = lab.copy()
    front = np.zeros(p.V, bool)
    front[np.unique(np.r_[p.src, p.col])] = True
    skips = 0
    for k in range(200):
        lab, front = oracle.min_superstep(p, lab, front, weighted=False, both_dirs=True)
        st.superstep()
        gids, vals, skip = st.sync_delta()
        rg, rv, rskip = oracle.delta(p, rem, lab, synced)
        assert np.array_equal(gids, rg) and np.array_equal(vals, rv) and skip == rskip, k
        skips += skip
        if not front.any():
            break
    assert np.array_equal(st.values_numpy(), lab)


@pytest.mark.parametrize("mode", [1.0, 1e-9])
def test_sync_delta_sssp_lazy_and_capacity(gx, mode):
    p = gen.rmat_part(14, seed=3, part=0)
    rem = oracle.remote_mask(p, "sssp")
    src = int(np.argmax(np.diff(p.row_ptr)))
    st = gx.State(load(gx, p, gx.GX_NEED_OUT), gx.GX_SSSP, source=src, pull_fraction=mode)
    dists, _ = oracle.sssp_frontiers(p, src)
    synced = dists[0].copy()
    # lazy: sync only every 3rd superstep; only final values are sent
    for k in range(1, len(dists)):
        st.superstep()
        if k % 3 == 0 or k == len(dists) - 1:
            rg, rv, rskip = oracle.delta(p, rem, dists[k], synced)
            if len(rg) > 1:
                with pytest.raises(gx.GxError):
                    st.sync_delta(cap=len(rg) - 1)  # too small: nothing committed
            gids, vals, skip = st.sync_delta()
            assert np.array_equal(gids, rg) and np.array_equal(vals, rv) and skip == rskip, k


def test_sync_delta_pagerank_all_mode(gx):
    g = gen.rmat(12, seed=8)
    st = gx.State(load(gx, g, gx.GX_NEED_IN), gx.GX_PAGERANK, delta_mode=gx.GX_DELTA_ALL)
    prev = st.values_numpy().copy()
    for _ in range(3):
        st.superstep()
        cur = st.values_numpy().copy()
        gids, vals, skip = st.sync_delta()
        want = np.nonzero(cur.view(np.uint32) != prev.view(np.uint32))[0]
        assert np.array_equal(gids, want)
        assert np.array_equal(vals, cur.view(np.uint32)[want])
        prev = cur
    # unpartitioned graph in REMOTE mode: nothing is remote, every sync skippable
    st2 = gx.State(load(gx, g, gx.GX_NEED_IN), gx.GX_PAGERANK)
    st2.superstep()
    gids, _, skip = st2.sync_delta()
    assert skip and len(gids) == 0


# ------------------------------------------------------------------ full size

@pytest.mark.slow
@pytest.mark.parametrize("mode", [0.0, 1.0])
def test_sssp_full_scale22_source0(gx, mode):
    """The benchmarked workload: R-MAT scale 22, source 0, to convergence
    (default switch point = the benchmarked launch configuration)."""
    g = gen.rmat(22, seed=2)
    ref = oracle.sssp(g, 0)
    st = gx.State(load(gx, g, gx.GX_NEED_OUT), gx.GX_SSSP, source=0, pull_fraction=mode)
    rs, steps = st.run(10_000, per_step=True)
    assert rs.supersteps == ref.K
    assert np.array_equal(st.values_numpy(), ref.state)
    steps = np.array(steps)
    assert np.array_equal(steps[:, 1], ref.msgs)
    assert np.array_equal(steps[:, 2], ref.changed)


@pytest.mark.slow
def test_partition_scale25_pagerank30_and_cc(gx):
    """One worker's part (1 of 8) of a hash vertex-cut of R-MAT scale 25:
    30 PageRank supersteps and label-propagation CC to convergence, with the
    sync set of the final CC state checked against the oracle's."""
    p = gen.rmat_part(25, seed=3, part=0)
    dg = load(gx, p, gx.GX_NEED_IN | gx.GX_NEED_SYM)
    ref = oracle.pagerank(p, 30, 0.85)
    st = gx.State(dg, gx.GX_PAGERANK, damping=0.85)
    st.run(30)
    x = st.values_numpy().astype(np.float64)
    assert np.max(np.abs(x - ref)) <= PR_TOL
    assert np.max(np.abs(x - ref) / ref) < 1e-4
    del st
    ref_cc = oracle.cc(p)
    st = gx.State(dg, gx.GX_CC)
    rs, steps = st.run(100_000, per_step=True)
    assert rs.supersteps == ref_cc.K
    assert np.array_equal(st.values_numpy(), ref_cc.state)
    assert np.array_equal(np.array(steps)[:, 2], ref_cc.changed)
    rem = oracle.remote_mask(p, "cc")
    synced = p.l2g.astype(np.uint32).copy()
    rg, rv, _ = oracle.delta(p, rem, ref_cc.state, synced)
    gids, vals, skip = st.sync_delta()
    assert np.array_equal(gids, rg) and np.array_equal(vals, rv) and not skip
