"""Batched lanes on MI355X: every SSSP lane must equal the oracle's
single-source solve bit for bit, every PPR lane must stay within 1e-6 of the
float64 oracle, for every launch shape the autotuner may pick."""
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


def load(gx, g):
    return gx.DeviceGraph(g, gx.GX_NEED_OUT | gx.GX_NEED_IN)


def lanes_u32(out):
    return out.cpu().numpy().view(np.uint32)


def check_sssp_lanes(g, D, sources):
    Ks = []
    for b, s in enumerate(sources):
        ref = oracle.sssp(g, int(s))
        assert np.array_equal(D[:, b], ref.state), f"lane {b} source {s}"
        Ks.append(ref.K)
    return max(Ks)


@pytest.mark.parametrize("B", [32, 64, 256])
def test_batched_sssp_lanes_equal_oracle(gx, B):
    g = gen.rmat(12, seed=4)
    src = gen.pick_sources(g, B, seed=40)
    out, rs = gx.batch_run(load(gx, g), gx.GX_SSSP, src)
    K = check_sssp_lanes(g, lanes_u32(out), src)
    assert rs.supersteps == K


@pytest.mark.parametrize("block,tile,width", [(256, 1024, 32), (256, 2048, 64), (512, 2048, 128),
                                              (512, 4096, 256), (1024, 2048, 32), (1024, 4096, 128)])
def test_batched_sssp_every_shape(gx, block, tile, width):
    g = gen.rmat(11, seed=7)
    src = gen.pick_sources(g, 256, seed=41)
    ref, _ = gx.batch_run(load(gx, g), gx.GX_SSSP, src)
    out, _ = gx.batch_run(load(gx, g), gx.GX_SSSP, src, tune=gx.Tune(block, tile, width, 0))
    assert np.array_equal(lanes_u32(out), lanes_u32(ref))
    D = lanes_u32(out)
    for b in (0, 31, 32, 200, 255):
        assert np.array_equal(D[:, b], oracle.sssp(g, int(src[b])).state)


def test_batched_sssp_autotune(gx):
    g = gen.rmat(12, seed=5)
    dg = load(gx, g)
    src = gen.pick_sources(g, 64, seed=42)
    best, ms = gx.batch_autotune(dg, gx.GX_SSSP, src)
    assert ms > 0 and best.block in (256, 512, 1024) and best.width in (32, 64)
    out, _ = gx.batch_run(dg, gx.GX_SSSP, src, tune=best)
    check_sssp_lanes(g, lanes_u32(out), src)


def test_batched_sssp_edge_cases(gx):
    # sources without out-edges, a repeated source, hubs wider than a tile
    V = 6000
    s = np.r_[np.zeros(V - 1, int), np.arange(1, 100)]
    d = np.r_[np.arange(1, V), np.arange(2, 101)]
    w = np.r_[np.full(V - 1, 200), np.ones(99, int)]
    g = gen.from_edges(V, s, d, w)
    src = np.array([0] * 3 + [5999] + list(range(1, 29)), np.int32)  # 5999 has no out-edge
    out, rs = gx.batch_run(load(gx, g), gx.GX_SSSP, src)
    check_sssp_lanes(g, lanes_u32(out), src)


def test_batched_sssp_rejects_bad_input(gx):
    g = gen.rmat(8, seed=1)
    dg = load(gx, g)
    with pytest.raises(gx.GxError):
        gx.batch_run(dg, gx.GX_SSSP, np.arange(33, dtype=np.int32))  # not a multiple of 32
    with pytest.raises(gx.GxError):
        gx.batch_run(dg, gx.GX_SSSP, np.full(32, g.V, np.int32))  # out of range


@pytest.mark.parametrize("B,iters", [(1, 30), (5, 50), (64, 50), (100, 20)])
def test_batched_ppr_lanes_equal_oracle(gx, B, iters):
    g = gen.rmat(11, seed=6)
    src = gen.pick_sources(g, B, seed=43)
    out, _ = gx.batch_run(load(gx, g), gx.GX_PPR, src, iters=iters)
    X = out.cpu().numpy()
    for b in range(0, B, max(1, B // 8)):
        ref = oracle.ppr(g, int(src[b]), iters)
        err = np.max(np.abs(X[:, b].astype(np.float64) - ref))
        assert err <= 1e-6, (b, err)


def test_batched_ppr_hub_rows_cross_tiles(gx):
    # in-degree 3000 into vertex 0 spans many 256-edge PPR tiles
    V = 3001
    src_e = np.r_[np.arange(1, V), np.zeros(40, int)]
    dst_e = np.r_[np.zeros(V - 1, int), np.arange(1, 41)]
    g = gen.from_edges(V, src_e, dst_e)
    seeds = np.array([0, 1, 2, 3000], np.int32)
    out, _ = gx.batch_run(load(gx, g), gx.GX_PPR, seeds, iters=40)
    X = out.cpu().numpy()
    for b, s in enumerate(seeds):
        assert np.max(np.abs(X[:, b] - oracle.ppr(g, int(s), 40))) <= 1e-6


def test_batched_ppr_lane_independent_of_batch(gx):
    g = gen.rmat(11, seed=8)
    dg = load(gx, g)
    src = gen.pick_sources(g, 48, seed=44)
    big, _ = gx.batch_run(dg, gx.GX_PPR, src, iters=25)
    alone, _ = gx.batch_run(dg, gx.GX_PPR, src[7:8], iters=25)
    assert np.array_equal(big.cpu().numpy()[:, 7].view(np.uint32), alone.cpu().numpy()[:, 0].view(np.uint32))
    grid2, _ = gx.batch_run(dg, gx.GX_PPR, src, iters=25, tune=gx.Tune(256, 256, 48, 64))
    assert np.array_equal(big.cpu().numpy().view(np.uint32), grid2.cpu().numpy().view(np.uint32))


def test_autotune_cache_file(gx, tmp_path, monkeypatch):
    """With GX_TUNE_CACHE naming a file, the first autotune times the
    candidates and appends its choice; a second call on the same graph,
    algorithm and lanes returns the stored shape and time without timing
    them (one line in the file still), a run with that shape equals the
    oracle, and another graph gets a line of its own."""
    path = tmp_path / "tune.txt"
    monkeypatch.setenv("GX_TUNE_CACHE", str(path))
    g = gen.rmat(11, seed=12)
    dg = load(gx, g)
    src = gen.pick_sources(g, 64, seed=47)
    best1, ms1 = gx.batch_autotune(dg, gx.GX_SSSP, src)
    assert len(path.read_text().splitlines()) == 1
    best2, ms2 = gx.batch_autotune(dg, gx.GX_SSSP, src)
    assert (best2.block, best2.tile, best2.width, best2.grid) == (best1.block, best1.tile, best1.width, best1.grid)
    assert ms2 == pytest.approx(ms1, abs=1e-5)
    assert len(path.read_text().splitlines()) == 1
    out, _ = gx.batch_run(dg, gx.GX_SSSP, src, tune=best2)
    D = lanes_u32(out)
    for b in (0, 31, 63):
        assert np.array_equal(D[:, b], oracle.sssp(g, int(src[b])).state), b
    g2 = gen.rmat(11, seed=13)
    gx.batch_autotune(load(gx, g2), gx.GX_SSSP, gen.pick_sources(g2, 64, seed=47))
    assert len(path.read_text().splitlines()) == 2


def test_batched_ppr_batch_widths_bitwise(gx):
    """Each lane adds its row's contributions in edge order whatever the
    batch width, so a batch of 3, 8, 9, 16, 17 or 32 lanes (fewer processed
    lanes than a wave holds) equals the same seeds inside a 64-lane batch bit
    for bit (R-MAT scale 14: hub rows span many 256-edge tiles)."""
    g = gen.rmat(14, seed=9)
    dg = load(gx, g)
    src = gen.pick_sources(g, 64, seed=46)
    src[0] = 0
    wide, _ = gx.batch_run(dg, gx.GX_PPR, src, iters=20)
    W = wide.cpu().numpy().view(np.uint32)
    for B in (3, 8, 9, 16, 17, 32):
        narrow, _ = gx.batch_run(dg, gx.GX_PPR, src[:B], iters=20)
        assert np.array_equal(narrow.cpu().numpy().view(np.uint32), W[:, :B]), B
    ref = oracle.ppr(g, int(src[2]), 20)
    assert np.max(np.abs(W[:, 2].view(np.float32).astype(np.float64) - ref)) <= 1e-6


@pytest.mark.slow
def test_batched_sssp_full_scale20_b256(gx):
    """The batched workload: R-MAT scale 20, 256 seeded sources, one launch
    with the default shape and one with the autotuned shape (the bench's
    launch); every lane against the oracle's single-source run from its
    source, and the superstep count."""
    g = gen.rmat(20, seed=4)
    src = gen.pick_sources(g, 256, seed=40)
    dg = load(gx, g)
    ref, K = oracle.sssp_many(g, src)
    out, rs = gx.batch_run(dg, gx.GX_SSSP, src)
    D = lanes_u32(out)
    for b in range(256):
        assert np.array_equal(D[:, b], ref[b]), b
    assert rs.supersteps == K.max()
    best, _ = gx.batch_autotune(dg, gx.GX_SSSP, src)
    out2, rs2 = gx.batch_run(dg, gx.GX_SSSP, src, tune=best)
    assert np.array_equal(lanes_u32(out2), D), best
    assert rs2.supersteps == K.max()


@pytest.mark.slow
@pytest.mark.parametrize("B", [64, 256])
def test_batched_ppr_scale16_every_lane(gx, B):
    """PPR lanes, 50 iterations, R-MAT scale 16 (vertex 0's in-row spans
    dozens of 256-edge pull tiles): every lane within 1e-6 of the float64
    oracle, and every lane bitwise the same when run alone."""
    g = gen.rmat(16, seed=6)
    assert np.bincount(g.col, minlength=g.V).max() >= 10 * 256
    src = gen.pick_sources(g, B, seed=45)
    src[0] = 0  # the hub itself as a seed
    dg = load(gx, g)
    out, rs = gx.batch_run(dg, gx.GX_PPR, src, iters=50)
    X = out.cpu().numpy().astype(np.float64)
    ref = oracle.ppr_many(g, src, 50)
    err = np.abs(X - ref.T).max(axis=0)
    assert err.max() <= 1e-6, (int(err.argmax()), float(err.max()))
    for b in (0, 1, B // 2, B - 1):
        alone, _ = gx.batch_run(dg, gx.GX_PPR, src[b:b + 1], iters=50)
        assert np.array_equal(alone.cpu().numpy()[:, 0].view(np.uint32), out.cpu().numpy()[:, b].view(np.uint32)), b


@pytest.mark.slow
@pytest.mark.parametrize("B", [64, 256])
def test_batched_ppr_scale20_bench_shape(gx, B):
    """The batched PPR workload the bench times: R-MAT scale 20 (seed 4),
    B seeds, 50 iterations.  Every lane keeps its mass (float32 sums of a
    float64-accumulated iteration) and holds at least the teleport share at
    its seed; 16 lanes spread over the tile are checked against the
    oracle."""
    g = gen.rmat(20, seed=4)
    src = gen.pick_sources(g, 256, seed=40)[:B]
    out, _ = gx.batch_run(load(gx, g), gx.GX_PPR, src, iters=50)
    X = out.cpu().numpy().astype(np.float64)
    assert np.all(X >= 0)
    assert np.abs(X.sum(axis=0) - 1.0).max() < 1e-4
    assert np.all(X[src, np.arange(B)] >= 0.15 - 1e-6)
    lanes = np.unique(np.r_[np.linspace(0, B - 1, 16).astype(int)])
    ref = oracle.ppr_many(g, src[lanes], 50)
    for i, b in enumerate(lanes):
        err = np.abs(X[:, b] - ref[i]).max()
        assert err <= 1e-6, (int(b), float(err))
