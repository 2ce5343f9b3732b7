"""All eight parts of a hash vertex-cut resident on one GPU, run superstep by
superstep with the sync sets exchanged between the parts (gx_sync_delta on
every part, gx_apply_delta of the other parts' pairs on every part): the
replicas must end with the global oracle's values, bit for bit, after as
many supersteps as the oracle takes on the whole graph."""
import numpy as np
import pytest

import gen
import oracle

pytestmark = pytest.mark.gpu

NPARTS = 8


@pytest.fixture(scope="module")
def gx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2203_13005_amd as m
    return m


def run_exchange(gx, parts, algo, gsource=None):
    import torch
    needs = gx.GX_NEED_OUT if algo == gx.GX_SSSP else gx.GX_NEED_SYM
    dgs = [gx.DeviceGraph(p, needs) for p in parts]
    states = []
    for p, dg in zip(parts, dgs):
        if algo == gx.GX_SSSP:
            loc = np.searchsorted(p.l2g, gsource)
            src = int(loc) if loc < p.V and p.l2g[loc] == gsource else -1
            states.append(gx.State(dg, algo, source=src, delta_mode=gx.GX_DELTA_ALL))
        else:
            states.append(gx.State(dg, algo, delta_mode=gx.GX_DELTA_ALL))
    K = 0
    while True:
        K += 1
        for st in states:
            st.superstep(stats=False)
        sent = [st.sync_delta(on_device=True) for st in states]
        active = 0
        for q, st in enumerate(states):
            others = [s for p, s in enumerate(sent) if p != q and s[0].numel()]
            gid = torch.cat([o[0] for o in others]) if others else sent[q][0][:0]
            val = torch.cat([o[1] for o in others]) if others else sent[q][1][:0]
            active += st.apply_delta(gid, val)
        if active == 0 or K > 10_000:
            break
    return K, [st.values_numpy() for st in states]


@pytest.mark.parametrize("scale,seed", [(10, 3), (12, 5)])
def test_exchange_sssp_equals_global_oracle(gx, scale, seed):
    g = gen.rmat(scale, seed=seed)
    parts = [gen.rmat_part(scale, seed=seed, part=p) for p in range(NPARTS)]
    src = int(np.nonzero(np.diff(g.row_ptr) > 0)[0][0])
    ref = oracle.sssp(g, src)
    K, vals = run_exchange(gx, parts, gx.GX_SSSP, src)
    assert K == ref.K
    for p, v in zip(parts, vals):
        assert np.array_equal(v, ref.state[p.l2g])


@pytest.mark.parametrize("scale,seed", [(10, 3), (12, 5)])
def test_exchange_cc_equals_global_oracle(gx, scale, seed):
    g = gen.rmat(scale, seed=seed)
    parts = [gen.rmat_part(scale, seed=seed, part=p) for p in range(NPARTS)]
    ref = oracle.cc(g)
    K, vals = run_exchange(gx, parts, gx.GX_CC)
    assert K == ref.K
    for p, v in zip(parts, vals):
        assert np.array_equal(v, ref.state[p.l2g])


def test_apply_delta_merges_min_and_ignores_foreign_ids(gx):
    import torch
    part = gen.rmat_part(10, seed=3, part=2)
    st = gx.State(gx.DeviceGraph(part, gx.GX_NEED_OUT), gx.GX_SSSP, source=-1)
    assert st.apply_delta(torch.empty(0, dtype=torch.int32, device="cuda:0"),
                          torch.empty(0, dtype=torch.int32, device="cuda:0")) == 0
    held = part.l2g[[0, 5, 9]].astype(np.int32)
    foreign = np.setdiff1d(np.arange(part.l2g.max() + 2, dtype=np.int32), part.l2g)[:3]
    gids = torch.tensor(np.r_[held, foreign], dtype=torch.int32, device="cuda:0")
    vals = torch.tensor(np.array([7, 3, 11, 1, 1, 1], np.uint32).view(np.int32), device="cuda:0")
    act = st.apply_delta(gids, vals)
    v = st.values_numpy()
    assert v[0] == 7 and v[5] == 3 and v[9] == 11
    assert (v == 0xFFFFFFFF).sum() == part.V - 3
    # every lowered replica is in the next frontier and counted active
    fr = st.frontier_numpy()
    assert set(np.nonzero(fr)[0]) == {0, 5, 9}
    assert act == 3
    # a larger value changes nothing
    st.apply_delta(gids[:1], torch.tensor(np.array([9], np.uint32).view(np.int32), device="cuda:0"))
    assert st.values_numpy()[0] == 7


# ------------------------------------------------------------------ PageRank across the parts

def pagerank_exchange(gx, g, parts, T, needs=None, record=None):
    """All parts resident, GX_PHASES_MASTERS states, T supersteps of the
    exchange (merged sums to masters in part order, masters apply, replicas
    take the masters' ranks); returns the per-part ranks after every
    superstep and the states."""
    import torch
    deg = np.diff(g.row_ptr).astype(np.int32)
    states = []
    for p in parts:
        dg = gx.DeviceGraph(p, gx.GX_NEED_IN if needs is None else needs, V_global=g.V, outdeg_global=deg[p.l2g])
        states.append(gx.State(dg, gx.GX_PAGERANK, damping=0.85, phases=gx.GX_PHASES_MASTERS,
                               delta_mode=gx.GX_DELTA_MASTERS))
    hist = []
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
        for q, st in enumerate(states):
            for p in range(len(states)):
                if p != q and sent[p][0].numel():
                    st.partial_add(*sent[p])
        for st in states:
            st.msg_apply(stats=False)
        bc = [st.sync_delta(on_device=True) for st in states]
        for q, st in enumerate(states):
            others = [b for p, b in enumerate(bc) if p != q and b[0].numel()]
            if others:
                st.apply_delta(torch.cat([o[0] for o in others]), torch.cat([o[1] for o in others]))
        if record is None or len(hist) + 1 in record:
            hist.append([st.values_numpy().copy() for st in states])
        else:
            hist.append(None)
    return hist, states


@pytest.mark.parametrize("scale,seed", [(10, 3), (12, 5)])
def test_exchange_pagerank_equals_global_oracle(gx, scale, seed):
    g = gen.rmat(scale, seed=seed)
    parts = gen.cover_isolated([gen.rmat_part(scale, seed=seed, part=p) for p in range(NPARTS)], g.V)
    _, ref = oracle.pagerank(g, 20, 0.85, history=True)
    hist, _ = pagerank_exchange(gx, g, parts, 20)
    for t in (1, 2, 5, 20):
        for p, x in zip(parts, hist[t - 1]):
            err = np.max(np.abs(x.astype(np.float64) - ref[t][p.l2g]))
            assert err <= 1e-6, (t, err)
    # every global vertex's master and replicas agree bitwise after the broadcast
    last = {}
    for p, x in zip(parts, hist[-1]):
        for gid, v in zip(p.l2g.tolist(), x.view(np.uint32).tolist()):
            assert last.setdefault(gid, v) == v
    assert len(last) == g.V


def test_exchange_pagerank_is_reproducible(gx):
    g = gen.rmat(11, seed=4)
    parts = gen.cover_isolated([gen.rmat_part(11, seed=4, part=p) for p in range(NPARTS)], g.V)
    a, _ = pagerank_exchange(gx, g, parts, 6)
    b, _ = pagerank_exchange(gx, g, parts, 6)
    for xa, xb in zip(a[-1], b[-1]):
        assert np.array_equal(xa.view(np.uint32), xb.view(np.uint32))


# ------------------------------------------------------------------ the partition workload's shape

@pytest.fixture(scope="module")
def c3_shape():
    """All eight parts of the hash vertex-cut of R-MAT scale 25 (seed 3)."""
    g = gen.rmat(25, seed=3)
    parts = [gen.rmat_part(25, seed=3, part=p) for p in range(NPARTS)]
    return g, parts


@pytest.mark.slow
def test_exchange_scale25_sssp_and_cc(gx, c3_shape):
    g, parts = c3_shape
    ref = oracle.sssp(g, 0, threads=0)
    K, vals = run_exchange(gx, parts, gx.GX_SSSP, 0)
    assert K == ref.K
    for p, v in zip(parts, vals):
        assert np.array_equal(v, ref.state[p.l2g])
    del vals
    ref = oracle.cc(g, threads=0)
    K, vals = run_exchange(gx, parts, gx.GX_CC)
    assert K == ref.K
    for p, v in zip(parts, vals):
        assert np.array_equal(v, ref.state[p.l2g])


@pytest.mark.slow
def test_exchange_scale25_pagerank30(gx, c3_shape):
    g, parts = c3_shape
    parts = gen.cover_isolated(parts, g.V)
    ref = oracle.pagerank(g, 30, 0.85, threads=0)
    hist, _ = pagerank_exchange(gx, g, parts, 30, record={30})
    seen = 0
    for p, x in zip(parts, hist[-1]):
        want = ref[p.l2g]
        err = np.abs(x.astype(np.float64) - want)
        assert err.max() <= 1e-6
        assert (err / want).max() < 1e-4
        seen += int(np.count_nonzero(p.flags & 1))
    assert seen == g.V
