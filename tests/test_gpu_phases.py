"""The template's three calls made separately (MSGGen, MSGMerge, MSGApply)
in BSP order (Gen -> Merge -> Apply) and in GAS order (Merge -> Apply ->
Gen): every superstep against the oracle (SSSP / CC bit for bit with their
active sets, message counts and changed counts; PageRank within 1e-6), and
equal to the fused superstep."""
import numpy as np
import pytest

import gen
import oracle

pytestmark = pytest.mark.gpu
PR_TOL = 1e-6
MODES = [1.0, 1e-9, 0.0]  # push only, pull whenever a message exists, default switch


@pytest.fixture(scope="module")
def gx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2203_13005_amd as m
    return m


def bsp(st):
    st.msg_gen()
    st.msg_merge()
    return st.msg_apply()


def min_reference(g, algo, src):
    if algo == "sssp":
        run = oracle.sssp(g, src)
        dists, _ = oracle.sssp_frontiers(g, src)
        return run, dists
    run = oracle.cc(g)
    lab = (np.arange(g.V) if g.l2g is None else g.l2g).astype(np.uint32)
    front = np.zeros(g.V, bool)
    front[np.unique(np.r_[np.repeat(np.arange(g.V), np.diff(g.row_ptr)), g.col])] = True
    states = [lab]
    for _ in range(run.K):
        lab, front = oracle.min_superstep(g, lab, front, weighted=False, both_dirs=True)
        states.append(lab)
    return run, states


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("algo", ["sssp", "cc"])
def test_bsp_order_every_superstep(gx, mode, algo):
    g = gen.rmat(13, seed=6)
    src = int(np.argmax(np.diff(g.row_ptr)))
    run, states = min_reference(g, algo, src)
    needs = gx.GX_NEED_OUT if algo == "sssp" else gx.GX_NEED_SYM
    a = gx.GX_SSSP if algo == "sssp" else gx.GX_CC
    st = gx.State(gx.DeviceGraph(g, needs), a, source=src, pull_fraction=mode, phases=True)
    for k in range(run.K):
        active, msgs, changed = bsp(st)
        assert active == run.front[k] and changed == run.changed[k], k
        # (CC sends along the deduplicated symmetric adjacency; the oracle
        # counts a message per direction of every input edge)
        assert algo == "cc" or msgs == run.msgs[k], k
        assert np.array_equal(st.values_numpy(), states[k + 1]), k
    assert changed == 0


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("algo", ["sssp", "cc"])
def test_gas_order_lags_one_superstep(gx, mode, algo):
    g = gen.rmat(12, seed=7)
    src = 0
    run, states = min_reference(g, algo, src)
    needs = gx.GX_NEED_OUT if algo == "sssp" else gx.GX_NEED_SYM
    a = gx.GX_SSSP if algo == "sssp" else gx.GX_CC
    st = gx.State(gx.DeviceGraph(g, needs), a, source=src, pull_fraction=mode, phases=True)
    # the first GAS iteration finds nothing to merge or apply, then generates
    st.msg_merge()
    assert st.msg_apply() == (0, 0, 0)
    st.msg_gen()
    assert np.array_equal(st.values_numpy(), states[0])
    for k in range(run.K):
        st.msg_merge()
        active, msgs, changed = st.msg_apply()
        st.msg_gen()
        assert active == run.front[k] and changed == run.changed[k], k
        assert algo == "cc" or msgs == run.msgs[k], k
        assert np.array_equal(st.values_numpy(), states[k + 1]), k


def test_phases_equal_fused_superstep(gx):
    g = gen.rmat(16, seed=9)
    dg = gx.DeviceGraph(g, gx.GX_NEED_OUT | gx.GX_NEED_SYM)
    for algo in (gx.GX_SSSP, gx.GX_CC):
        fused = gx.State(dg, algo, source=0)
        split = gx.State(dg, algo, source=0, phases=True)
        while True:
            f = fused.superstep()
            s = bsp(split)
            assert f == s
            assert np.array_equal(fused.values_numpy(), split.values_numpy())
            if f[2] == 0:
                break


def test_pagerank_bsp_and_gas(gx):
    g = gen.rmat(12, seed=8)
    _, hist = oracle.pagerank(g, 20, 0.85, history=True)
    dg = gx.DeviceGraph(g, gx.GX_NEED_IN)
    b = gx.State(dg, gx.GX_PAGERANK, phases=True)
    for t in range(1, 21):
        active, msgs, _ = bsp(b)
        assert active == g.V and msgs == g.E
        assert np.max(np.abs(b.values_numpy() - hist[t])) <= PR_TOL, t
    gas = gx.State(dg, gx.GX_PAGERANK, phases=True)
    gas.msg_merge()
    assert gas.msg_apply() == (0, 0, 0)
    gas.msg_gen()
    for t in range(1, 21):
        gas.msg_merge()
        gas.msg_apply()
        gas.msg_gen()
        assert np.max(np.abs(gas.values_numpy() - hist[t])) <= PR_TOL, t
    # in place, the same arithmetic in both orders
    assert np.array_equal(gas.values_numpy().view(np.uint32), b.values_numpy().view(np.uint32))
    fused = gx.State(dg, gx.GX_PAGERANK)
    fused.run(20)
    assert np.max(np.abs(fused.values_numpy() - b.values_numpy())) <= 1e-7


def test_phases_sync_delta_on_a_partition(gx):
    p = gen.rmat_part(13, seed=3, part=2)
    rem = oracle.remote_mask(p, "sssp")
    src = int(np.argmax(np.diff(p.row_ptr)))
    dists, _ = oracle.sssp_frontiers(p, src)
    st = gx.State(gx.DeviceGraph(p, gx.GX_NEED_OUT), gx.GX_SSSP, source=src, phases=True)
    synced = dists[0].copy()
    for k in range(1, len(dists)):
        bsp(st)
        rg, rv, rskip = oracle.delta(p, rem, dists[k], synced)
        gids, vals, skip = st.sync_delta()
        assert np.array_equal(gids, rg) and np.array_equal(vals, rv) and skip == rskip, k


def test_phase_misuse_is_refused(gx):
    g = gen.rmat(8, seed=1)
    dg = gx.DeviceGraph(g, gx.GX_NEED_OUT)
    st = gx.State(dg, gx.GX_SSSP, source=0, phases=True)
    st.msg_gen()
    with pytest.raises(gx.GxError):
        st.msg_gen()  # the first messages were not merged
    with pytest.raises(gx.GxError):
        st.superstep()
    fused = gx.State(dg, gx.GX_SSSP, source=0)
    with pytest.raises(gx.GxError):
        fused.msg_gen()


@pytest.mark.slow
@pytest.mark.parametrize("order", ["bsp", "gas"])
def test_sssp_scale22_through_separate_calls(gx, order):
    g = gen.rmat(22, seed=2)
    ref = oracle.sssp(g, 0)
    st = gx.State(gx.DeviceGraph(g, gx.GX_NEED_OUT), gx.GX_SSSP, source=0, phases=True)
    if order == "gas":
        st.msg_merge()
        st.msg_apply()
        st.msg_gen()
    changed = []
    for _ in range(ref.K):
        if order == "bsp":
            st.msg_gen()
        st.msg_merge()
        changed.append(st.msg_apply()[2])
        if order == "gas":
            st.msg_gen()
    assert changed == ref.changed.tolist()
    assert np.array_equal(st.values_numpy(), ref.state)
