"""Label propagation on the device against the oracle: every iteration's
labels and changed count bit for bit, on the hand-worked example, closed
forms, graphs whose vertices fill every degree class (lane groups of 4..64,
the LDS-table workgroups and hubs split into several chunks), R-MAT graphs,
a partition (labels are global ids) with its sync sets, and the scale-22
R-MAT graph at the benchmarked size."""
import json
import os

import numpy as np
import pytest

import gen
import oracle

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def gx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2203_13005_amd as m
    return m


def undirected(V, pairs):
    e = np.array(pairs, dtype=np.int64).reshape(-1, 2)
    return gen.from_edges(V, e[:, 0], e[:, 1], np.ones(len(e), np.int64))


def check_stepwise(gx, g, steps=15):
    ref = oracle.lp_steps(g, steps)
    st = gx.State(gx.DeviceGraph(g, gx.GX_NEED_SYM), gx.GX_LP)
    assert np.array_equal(st.values_numpy(), ref[0])
    for k in range(1, len(ref)):
        _, _, ch = st.superstep()
        want = ref[k]
        assert np.array_equal(st.values_numpy(), want), k
        assert ch == int(np.count_nonzero(want != ref[k - 1])), k
    return len(ref) - 1


def test_lp_hand_example(gx):
    with open(os.path.join(GOLDEN, "hand_lp_8v.json")) as f:
        h = json.load(f)
    g = undirected(h["V"], h["edges"])
    st = gx.State(gx.DeviceGraph(g, gx.GX_NEED_SYM), gx.GX_LP)
    rs, steps = st.run(15, per_step=True)
    assert rs.supersteps == h["K"] and rs.converged == 1
    assert [s[2] for s in steps] == h["changed"]
    assert st.values_numpy().tolist() == h["labels_after_iteration"][-1]


def test_lp_star_reaches_the_cap(gx):
    g = undirected(6, [(0, j) for j in range(1, 6)])
    st = gx.State(gx.DeviceGraph(g, gx.GX_NEED_SYM), gx.GX_LP)
    rs, _ = st.run(15, allow_cap=True)
    assert rs.supersteps == 15 and rs.converged == 0
    assert st.values_numpy().tolist() == oracle.lp(g, 15).state.tolist() == [1, 0, 0, 0, 0, 0]


def test_lp_complete_and_empty(gx):
    g = undirected(7, [(i, j) for i in range(7) for j in range(i + 1, 7)])
    assert check_stepwise(gx, g) == 3
    e = gen.from_edges(5, np.array([], np.int64), np.array([], np.int64), np.array([], np.int64))
    st = gx.State(gx.DeviceGraph(e, gx.GX_NEED_SYM), gx.GX_LP)
    rs, _ = st.run(15)
    assert rs.supersteps == 1 and st.values_numpy().tolist() == list(range(5))


def every_class_graph(seed):
    """Vertices of every degree class: a hub joined to 20,000 others (three
    chunks), one to 3,000 (one chunk), mid-class vertices of 65..2,048
    neighbours, and a random sparse background; labels collide often because
    neighbourhoods overlap."""
    rng = np.random.default_rng(seed)
    V = 24000
    src, dst = [], []
    src += [0] * 20000
    dst += list(range(1, 20001))
    src += [1] * 3000
    dst += list(rng.choice(np.arange(2, V), 3000, replace=False))
    for v, d in zip(range(2, 40), rng.integers(65, 2049, 38)):
        src += [v] * int(d)
        dst += list(rng.integers(0, 3000, int(d)))  # overlapping: labels repeat
    m = 60000
    src += list(rng.integers(0, V, m))
    dst += list(rng.integers(0, V, m) // 8)  # skewed destinations
    return gen.from_edges(V, np.array(src), np.array(dst), np.ones(len(src), np.int64))


@pytest.mark.parametrize("seed", [1, 2])
def test_lp_every_degree_class(gx, seed):
    g = every_class_graph(seed)
    check_stepwise(gx, g)


@pytest.mark.parametrize("scale,seed", [(12, 1), (14, 2)])
def test_lp_rmat(gx, scale, seed):
    g = gen.rmat(scale, seed=seed)
    check_stepwise(gx, g)


def test_lp_partition_global_labels_and_sync(gx):
    p = gen.rmat_part(14, seed=3, part=1)
    rem = oracle.remote_mask(p, "cc")
    ref = oracle.lp_steps(p, 15)
    st = gx.State(gx.DeviceGraph(p, gx.GX_NEED_SYM), gx.GX_LP)
    synced = ref[0].copy()
    for k in range(1, len(ref)):
        st.superstep()
        assert np.array_equal(st.values_numpy(), ref[k]), k
        if k % 2 == 0 or k == len(ref) - 1:  # lazily: a label that went back is not sent
            rg, rv, rskip = oracle.delta(p, rem, ref[k], synced)
            gids, vals, skip = st.sync_delta()
            assert np.array_equal(gids, rg) and np.array_equal(vals, rv) and skip == rskip, k


def test_lp_determinism(gx):
    g = every_class_graph(3)
    dg = gx.DeviceGraph(g, gx.GX_NEED_SYM)
    a = gx.State(dg, gx.GX_LP)
    a.run(15, allow_cap=True)
    b = gx.State(dg, gx.GX_LP)
    b.run(15, allow_cap=True)
    assert np.array_equal(a.values_numpy(), b.values_numpy())


@pytest.mark.slow
def test_lp_rmat22_two_iterations_then_run(gx):
    """The benchmarked LP workload (R-MAT scale 22, symmetric): the first two
    iterations against the oracle's iteration, then the full run's every
    iteration against one oracle iteration from the device's labels before it."""
    g = gen.rmat(22, seed=2)
    adj = oracle.SymAdjacency(g)
    st = gx.State(gx.DeviceGraph(g, gx.GX_NEED_SYM), gx.GX_LP)
    prev = st.values_numpy().copy()
    for k in range(15):
        _, _, ch = st.superstep()
        cur = st.values_numpy().copy()
        if k < 3 or k == 14 or ch == 0:
            want = adj.lp_step(prev)
            assert np.array_equal(cur, want), k
        assert ch == int(np.count_nonzero(cur != prev)), k
        prev = cur
        if ch == 0:
            break
