"""A graph split between a part on the GPU and a part on the CPU daemon
(Section "Workload Balancing": workers of different computation capacity),
exchanging sync sets every superstep: equal to the whole-graph oracle bit
for bit after the oracle's number of supersteps, for any share."""
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


def hybrid(gx, g, share, algo, source=0):
    import torch
    parts = gen.split_by_share(g, share)
    needs = gx.GX_NEED_OUT if algo == gx.GX_SSSP else gx.GX_NEED_SYM

    def local(p):
        loc = int(np.searchsorted(p.l2g, source))
        return loc if loc < p.V and p.l2g[loc] == source else -1

    gpu = gx.State(gx.DeviceGraph(parts[0], needs), algo, source=local(parts[0]))
    cpu = gx.CpuPart(parts[1], algo, source=local(parts[1]))
    K = 0
    while True:
        K += 1
        gpu.superstep(stats=False)
        cpu.superstep()
        gg, gv, _ = gpu.sync_delta()
        cg, cv = cpu.sync_delta()
        act = cpu.apply_delta(gg, gv)
        act += gpu.apply_delta(torch.tensor(cg, device="cuda:0"), torch.tensor(cv.view(np.int32), device="cuda:0"))
        if act == 0:
            break
    return K, parts, gpu.values_numpy(), cpu.values_numpy()


@pytest.mark.parametrize("share", [0.01, 0.3, 0.9])
@pytest.mark.parametrize("algo", ["sssp", "cc"])
def test_gpu_cpu_split_equals_whole_graph(gx, share, algo):
    g = gen.rmat(13, seed=7)
    a = gx.GX_SSSP if algo == "sssp" else gx.GX_CC
    ref = oracle.sssp(g, 0) if algo == "sssp" else oracle.cc(g)
    K, parts, vg, vc = hybrid(gx, g, share, a)
    assert K == ref.K
    # the smallest replica of a vertex is its value in the whole graph (a part
    # sends a vertex only where another part relaxes its edges)
    best = np.full(g.V, 0xFFFFFFFF, np.uint32)
    np.minimum.at(best, parts[0].l2g, vg)
    np.minimum.at(best, parts[1].l2g, vc)
    held = np.zeros(g.V, bool)
    held[parts[0].l2g] = True
    held[parts[1].l2g] = True
    assert np.array_equal(best[held], ref.state[held])
