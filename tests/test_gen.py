"""Invariants of the seeded input generator (no method arithmetic here)."""
import numpy as np

import gen


def test_rmat_csr_invariants():
    g = gen.rmat(12, seed=7)
    assert g.row_ptr[0] == 0 and g.row_ptr[-1] == g.E
    assert np.all(np.diff(g.row_ptr) >= 0)
    src = g.src
    assert not np.any(src == g.col), "self-loop"
    key = src.astype(np.int64) * g.V + g.col
    assert np.all(np.diff(key) > 0), "rows sorted and no duplicates"
    assert g.w.min() >= 1 and g.w.max() <= 255
    assert 0 < g.E <= 16 * g.V


def test_rmat_is_deterministic_and_seeded():
    a = gen.rmat(10, seed=5)
    b = gen.rmat(10, seed=5)
    c = gen.rmat(10, seed=6)
    assert np.array_equal(a.col, b.col) and np.array_equal(a.w, b.w)
    assert a.E != c.E or not np.array_equal(a.col, c.col)


def test_rmat_quadrant_frequencies():
    n = 2_000_000
    q = gen.quadrant_counts(16, n, seed=9)
    p = np.array([0.57, 0.19, 0.19, 0.05])
    sd = np.sqrt(n * p * (1 - p))
    assert np.all(np.abs(q - n * p) < 6 * sd)


def test_weights_depend_only_on_endpoints():
    g1 = gen.rmat(10, seed=4)
    g2 = gen.rmat(10, seed=4, E_raw=8 * 1024)
    # a pair present in both graphs carries the same weight
    k1 = dict(zip((g1.src.astype(np.int64) * g1.V + g1.col).tolist(), g1.w.tolist()))
    k2 = zip((g2.src.astype(np.int64) * g2.V + g2.col).tolist(), g2.w.tolist())
    common = [(k, w) for k, w in k2 if k in k1]
    assert len(common) > 100
    assert all(k1[k] == w for k, w in common)


def test_partition_conserves_edges_and_flags():
    scale, seed = 12, 3
    g = gen.rmat(scale, seed=seed)
    parts = [gen.rmat_part(scale, seed=seed, part=p) for p in range(8)]
    assert sum(p.E for p in parts) == g.E
    gkeys = set((g.src.astype(np.int64) * g.V + g.col).tolist())
    seen = set()
    masters = np.zeros(g.V, np.int64)
    for pi, p in enumerate(parts):
        assert np.all(np.diff(p.l2g) > 0)
        keys = (p.l2g[p.src].astype(np.int64) * g.V + p.l2g[p.col]).tolist()
        ks = set(keys)
        assert ks <= gkeys and not (ks & seen)
        seen |= ks
        assert np.all(p.w >= 1) and np.all(p.w <= 255)
        masters[p.l2g] += (p.flags & 1)
        # remote_out implies remote_any
        assert np.all((p.flags & 2) <= (p.flags & 4) // 2 * 2)
    assert seen == gkeys
    touched = np.zeros(g.V, bool)
    touched[g.src] = True
    touched[g.col] = True
    assert np.all(masters[touched] == 1) and np.all(masters[~touched] == 0)
    # remote_any(v) in part p <=> v appears in some other part
    appear = np.zeros((8, g.V), bool)
    for pi, p in enumerate(parts):
        appear[pi, p.l2g] = True
    for pi, p in enumerate(parts):
        other = appear[np.arange(8) != pi][:, p.l2g].any(axis=0)
        assert np.array_equal((p.flags & 4) != 0, other)


def test_pick_sources_distinct_with_out_edges():
    g = gen.rmat(12, seed=4)
    s = gen.pick_sources(g, 64, seed=40)
    assert len(np.unique(s)) == 64
    assert np.all(np.diff(g.row_ptr)[s] > 0)
    assert np.array_equal(s, gen.pick_sources(g, 64, seed=40))


def test_cover_isolated_gives_every_vertex_one_master():
    g = gen.rmat(10, seed=3)
    parts = [gen.rmat_part(10, seed=3, part=p) for p in range(8)]
    cov = gen.cover_isolated(parts, g.V)
    masters = np.zeros(g.V, int)
    for p in cov:
        masters[p.l2g[(p.flags & 1) != 0]] += 1
    assert (masters == 1).all()
    for a, b in zip(parts, cov):
        ea = set(zip(a.l2g[a.src].tolist(), a.l2g[a.col].tolist()))
        eb = set(zip(b.l2g[b.src].tolist(), b.l2g[b.col].tolist()))
        assert ea == eb and np.all(np.diff(b.l2g) > 0)
    assert cov[0].V == parts[0].V + cov[0].meta["isolated_added"]
