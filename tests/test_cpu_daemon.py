"""The CPU daemon (host threads running the same superstep) against the
oracle, alone and exchanging sync sets with another part, and the balancing
split (Lemma minmaxcidi) against the exhaustive search.  Host only."""
import numpy as np
import pytest

import gen
import oracle


@pytest.fixture(scope="module")
def gx():
    import paper_2203_13005_amd as m
    return m


@pytest.mark.parametrize("threads", [1, 4])
def test_cpu_daemon_sssp_every_superstep(gx, threads):
    g = gen.rmat(11, seed=4)
    src = int(np.argmax(np.diff(g.row_ptr)))
    dists, fronts = oracle.sssp_frontiers(g, src)
    run = oracle.sssp(g, src)
    c = gx.CpuPart(g, gx.GX_SSSP, source=src, threads=threads)
    for k in range(run.K):
        f, m, ch = c.superstep()
        assert (f, m, ch) == (run.front[k], run.msgs[k], run.changed[k]), k
        assert np.array_equal(c.values_numpy(), dists[k + 1]), k


def test_cpu_daemon_cc_and_sync(gx):
    p = gen.rmat_part(11, seed=3, part=5)
    ref = oracle.cc(p)
    rem = oracle.remote_mask(p, "cc")
    c = gx.CpuPart(p, gx.GX_CC, threads=3)
    synced = p.l2g.astype(np.uint32)
    for k in range(ref.K):
        _, _, ch = c.superstep()
        assert ch == ref.changed[k], k
        cur = c.values_numpy()
        gid, val = c.sync_delta()
        rg, rv, _ = oracle.delta(p, rem, cur, synced)  # vertices another part holds
        assert np.array_equal(gid, rg) and np.array_equal(val, rv), k
    assert np.array_equal(c.values_numpy(), ref.state)


@pytest.mark.parametrize("algo", ["sssp", "cc"])
def test_two_cpu_parts_exchange_equal_whole_graph(gx, algo):
    g = gen.rmat(11, seed=6)
    parts = gen.split_by_share(g, 0.3)
    a = gx.GX_SSSP if algo == "sssp" else gx.GX_CC
    ref = oracle.sssp(g, 0) if algo == "sssp" else oracle.cc(g)
    workers = []
    for p in parts:
        loc = int(np.searchsorted(p.l2g, 0))
        s = loc if loc < p.V and p.l2g[loc] == 0 else -1
        workers.append(gx.CpuPart(p, a, source=s, threads=2))
    K = 0
    while True:
        K += 1
        for w in workers:
            w.superstep()
        sent = [w.sync_delta() for w in workers]
        active = sum(w.apply_delta(*sent[1 - i]) for i, w in enumerate(workers))
        if active == 0:
            break
    assert K == ref.K
    # a part keeps every replica it sends from exact; the smallest replica of a
    # vertex is its value in the whole graph
    best = np.full(g.V, 0xFFFFFFFF, np.uint32)
    for p, w in zip(parts, workers):
        np.minimum.at(best, p.l2g, w.values_numpy())
    held = np.zeros(g.V, bool)
    for p in parts:
        held[p.l2g] = True
    assert np.array_equal(best[held], ref.state[held])


def test_balance_split_reaches_the_lemma_optimum(gx):
    rng = np.random.default_rng(5)
    for _ in range(30):
        c = rng.uniform(0.1, 10.0, int(rng.integers(2, 4)))
        D = int(rng.integers(1, 20))
        d = gx.balance_split(c, D)
        assert abs(d.sum() - D) < 1e-9 * max(D, 1)
        lemma = float(np.max(c * d))
        assert abs(lemma - D / np.sum(1.0 / c)) < 1e-9 * D + 1e-12
        _, best = oracle.balance_brute_force(c, D)
        assert lemma <= best + 1e-9  # no integer split beats the real-valued optimum
    with pytest.raises(gx.GxError):
        gx.balance_split([1.0, 0.0], 10)
