"""Streamed supersteps (triplets in pinned host memory, blocks through three
rotating device buffers) against the oracle: every superstep's values,
frontier, messages and changed count bit for bit, and every uploaded
triplet result, for block sizes from 1 triplet to the whole graph, in the
pipelined and the serial form."""
import numpy as np
import pytest

import gen
import oracle

pytestmark = pytest.mark.gpu
INF = 0xFFFFFFFF


@pytest.fixture(scope="module")
def gx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2203_13005_amd as m
    return m


def sat_msgs(g, dist, front):
    src = np.repeat(np.arange(g.V), np.diff(g.row_ptr))
    m = np.minimum(dist[src].astype(np.uint64) + g.w.astype(np.uint64), INF).astype(np.uint32)
    return np.where(front[src], m, np.uint32(INF))


@pytest.mark.parametrize("block,serial", [(1000, False), (1000, True), (7, False), (1, False), (10 ** 9, False)])
def test_sssp_streamed_every_superstep(gx, block, serial):
    g = gen.rmat(11 if block > 1 else 8, seed=3)
    src = int(np.argmax(np.diff(g.row_ptr)))
    dists, fronts = oracle.sssp_frontiers(g, src)
    run = oracle.sssp(g, src)
    st = gx.Stream(g, gx.GX_SSSP, source=src, block_edges_max=min(block, g.E))
    b = min(block, g.E)
    for k in range(len(dists) - 1):
        s = st.superstep(b, serial=serial)
        assert s["blocks"] == -(-g.E // b) and s["triplets"] == g.E
        assert s["messages"] == run.msgs[k] and s["changed"] == run.changed[k], k
        assert np.array_equal(st.values_numpy(), dists[k + 1]), k
        assert np.array_equal(st.frontier_numpy(), fronts[k + 1]), k
        assert np.array_equal(st.results_numpy(), sat_msgs(g, dists[k], fronts[k])), k
        if serial:
            assert s["download_ms"] > 0 and s["compute_ms"] > 0 and s["upload_ms"] > 0
    assert s["changed"] == 0


@pytest.mark.parametrize("block", [4096, 333])
def test_cc_streamed_partition(gx, block):
    p = gen.rmat_part(12, seed=3, part=4)
    ref = oracle.cc(p)
    st = gx.Stream(p, gx.GX_CC, block_edges_max=block)
    for k in range(ref.K):
        s = st.superstep(block)
        assert s["changed"] == ref.changed[k], k
    assert np.array_equal(st.values_numpy(), ref.state)


def test_streamed_equals_resident_and_resets(gx):
    g = gen.rmat(15, seed=5)
    res = gx.State(gx.DeviceGraph(g, gx.GX_NEED_OUT), gx.GX_SSSP, source=0)
    res.run(10_000)
    st = gx.Stream(g, gx.GX_SSSP, source=0, block_edges_max=1 << 16)
    for _ in range(2):
        while st.superstep(50_000)["changed"]:
            pass
        assert np.array_equal(st.values_numpy(), res.values_numpy())
        st.reset()


def test_stream_edge_cases(gx):
    empty = gen.from_edges(4, np.array([], np.int64), np.array([], np.int64), np.array([], np.int64))
    st = gx.Stream(empty, gx.GX_SSSP, source=1, block_edges_max=8)
    s = st.superstep(8)
    assert s["blocks"] == 0 and s["changed"] == 0
    assert st.values_numpy().tolist() == [INF, 0, INF, INF]
    g = gen.rmat(8, seed=1)
    st = gx.Stream(g, gx.GX_SSSP, source=0, block_edges_max=64)
    with pytest.raises(gx.GxError):
        st.superstep(65)  # beyond the buffers
    with pytest.raises(gx.GxError):
        st.superstep(0)


@pytest.mark.slow
def test_sssp_scale22_streamed_with_planned_blocks(gx):
    g = gen.rmat(22, seed=2)
    ref = oracle.sssp(g, 0, threads=0)
    blocks, bsize, _ = gx.pipeline_plan(0.24e-9, 0.03e-9, 0.08e-9, 10e-6, g.E)
    b = int(np.ceil(bsize))
    st = gx.Stream(g, gx.GX_SSSP, source=0, block_edges_max=b)
    changed = []
    for k in range(ref.K):
        s = st.superstep(b)
        changed.append(s["changed"])
        assert s["messages"] == ref.msgs[k]
    assert changed == ref.changed.tolist()
    assert np.array_equal(st.values_numpy(), ref.state)
