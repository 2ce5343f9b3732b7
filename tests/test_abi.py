"""Host-side checks of the C ABI: the library loads, exports every symbol the
header declares, and rejects malformed input on the host before any device
call (these run without a GPU)."""
import ctypes
import os
import re

import numpy as np
import pytest

import gen

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "gx.h")).read()
    return sorted(set(re.findall(r"^(?:gx_status|const char \*)\s*(gx_\w+)\s*\(", text, re.M)))


def test_library_exports_every_declared_symbol():
    from paper_2203_13005_amd import binding
    lib = ctypes.CDLL(binding.library_path())
    names = declared_symbols()
    assert len(names) >= 20
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    # the binding wires every declared call
    assert set(names) <= set(binding._SIGS)


def _desc(binding, g, needs, **over):
    rp = np.ascontiguousarray(over.pop("row_ptr", g.row_ptr), np.int32)
    col = np.ascontiguousarray(over.pop("col", g.col), np.int32)
    w = over.pop("w", g.w)
    w = None if w is None else np.ascontiguousarray(w, np.uint32)
    keep = [rp, col, w]
    d = binding._GraphDesc(over.pop("V", g.V), over.pop("E", g.E), binding._np_ptr(rp), binding._np_ptr(col),
                           binding._np_ptr(w), None, None, needs)
    return d, keep


def test_graph_bytes_and_validation():
    from paper_2203_13005_amd import binding as b
    g = gen.rmat(8, seed=1)
    n = ctypes.c_size_t()
    d, keep = _desc(b, g, b.GX_NEED_OUT | b.GX_NEED_IN | b.GX_NEED_SYM)
    assert b.lib.gx_graph_bytes(ctypes.byref(d), ctypes.byref(n)) == b.GX_OK
    assert n.value >= g.E * 8 + g.E * 4
    # bad inputs are refused on the host
    cases = []
    bad_col = g.col.copy()
    bad_col[3] = g.V
    cases.append(dict(col=bad_col))
    bad_rp = g.row_ptr.copy()
    bad_rp[5], bad_rp[6] = bad_rp[6] + 1, bad_rp[5]
    cases.append(dict(row_ptr=bad_rp))
    cases.append(dict(E=g.E + 1))
    cases.append(dict(V=-1))
    cases.append(dict(w=None))
    for over in cases:
        d, keep = _desc(b, g, b.GX_NEED_OUT, **over)
        assert b.lib.gx_graph_bytes(ctypes.byref(d), ctypes.byref(n)) == b.GX_EINVAL, over.keys()
        assert b.lib.gx_last_error()
    d, keep = _desc(b, g, 0)
    assert b.lib.gx_graph_bytes(ctypes.byref(d), ctypes.byref(n)) == b.GX_EINVAL
    for tile, ok in ((0, True), (256, True), (2048, True), (128, False), (300, False), (4096, False)):
        d, keep = _desc(b, g, b.GX_NEED_IN)
        d.pr_tile_edges = tile
        st = b.lib.gx_graph_bytes(ctypes.byref(d), ctypes.byref(n))
        assert st == (b.GX_OK if ok else b.GX_EINVAL), tile


def test_load_rejects_small_arena_before_touching_device():
    from paper_2203_13005_amd import binding as b
    g = gen.rmat(8, seed=1)
    d, keep = _desc(b, g, b.GX_NEED_OUT)
    n = ctypes.c_size_t()
    assert b.lib.gx_graph_bytes(ctypes.byref(d), ctypes.byref(n)) == b.GX_OK
    h = ctypes.c_void_p()
    # a fake, aligned, never-dereferenced arena address: refused for size first
    st = b.lib.gx_graph_load(ctypes.byref(d), ctypes.c_void_p(1 << 20), n.value - 1, None, ctypes.byref(h))
    assert st == b.GX_ENOMEM and not h.value
    st = b.lib.gx_graph_load(ctypes.byref(d), ctypes.c_void_p((1 << 20) + 8), n.value, None, ctypes.byref(h))
    assert st == b.GX_EINVAL  # misaligned


def test_null_handles_are_einval():
    from paper_2203_13005_amd import binding as b
    assert b.lib.gx_graph_free(None) == b.GX_OK
    assert b.lib.gx_state_free(None) == b.GX_OK
    k = ctypes.c_int64()
    assert b.lib.gx_state_superstep(None, ctypes.byref(k)) == b.GX_EINVAL
    assert b.lib.gx_superstep(None, None, None) == b.GX_EINVAL
    n = ctypes.c_uint32()
    assert b.lib.gx_sync_delta(None, None, None, 0, ctypes.byref(n), None, None) == b.GX_EINVAL
    assert b.lib.gx_sync_delta_noalloc(None, None, None, 0, None, None) == b.GX_EINVAL
    assert b.lib.gx_msg_gen(None, None) == b.GX_EINVAL
    assert b.lib.gx_msg_merge(None, None) == b.GX_EINVAL
    assert b.lib.gx_msg_apply(None, None, None) == b.GX_EINVAL
    act = ctypes.c_int64()
    assert b.lib.gx_apply_delta(None, None, None, 0, ctypes.byref(act), None) == b.GX_EINVAL
    assert b.lib.gx_version().startswith(b"gx")


def test_server_config_validation_on_host():
    from paper_2203_13005_amd import binding as b
    h = ctypes.c_void_p()
    cfg = b._ServerConfig(None, 0, 0, 0, 0, 0.0, 0)
    assert b.lib.gx_server_create(ctypes.byref(cfg), ctypes.byref(h)) == b.GX_EINVAL  # no arena
    cfg = b._ServerConfig(ctypes.c_void_p(1 << 20), 1 << 20, 48, 0, 0, 0.0, 0)  # lanes not a multiple of 32
    assert b.lib.gx_server_create(ctypes.byref(cfg), ctypes.byref(h)) == b.GX_EINVAL
    cfg = b._ServerConfig(ctypes.c_void_p(1 << 20), 1 << 20, 64, 0, 65, 0.0, 0)  # epoch too long
    assert b.lib.gx_server_create(ctypes.byref(cfg), ctypes.byref(h)) == b.GX_EINVAL
    cfg = b._ServerConfig(ctypes.c_void_p(1 << 20), 1 << 20, 64, 0, 0, 1.5, 0)  # damping out of range
    assert b.lib.gx_server_create(ctypes.byref(cfg), ctypes.byref(h)) == b.GX_EINVAL
    n = ctypes.c_uint32()
    assert b.lib.gx_server_poll(None, None, 0, ctypes.byref(n), 0) == b.GX_EINVAL
    qid = ctypes.c_int64()
    assert b.lib.gx_server_submit(None, 0, 1, 0, None, ctypes.byref(qid)) == b.GX_EINVAL


def test_batch_and_server_null_graph():
    from paper_2203_13005_amd import binding as b
    n = ctypes.c_size_t()
    assert b.lib.gx_batch_bytes(None, b.GX_SSSP, 32, ctypes.byref(n)) == b.GX_EINVAL
    assert b.lib.gx_server_bytes_per_lane(None, b.GX_SSSP, ctypes.byref(n)) == b.GX_EINVAL


def test_symmetric_image_size_limit_is_einval():
    """CC's symmetric image holds up to 2E entries behind int32 row pointers:
    a description with 2E beyond that range is refused on the host before
    any array is read (the arrays here are far shorter than E)."""
    from paper_2203_13005_amd import binding as b
    rp = np.zeros(3, np.int32)
    col = np.zeros(1, np.int32)
    E = (1 << 30) + 1
    d = b._GraphDesc(2, E, b._np_ptr(rp), b._np_ptr(col), None, None, None, b.GX_NEED_SYM)
    n = ctypes.c_size_t()
    assert b.lib.gx_graph_bytes(ctypes.byref(d), ctypes.byref(n)) == b.GX_EINVAL
    assert b"symmetric" in b.lib.gx_last_error()


def test_pipeline_plan_matches_brute_force():
    """The Lemma's block size with the floor/ceiling rule reaches the brute
    force minimum of the time model in every case (download, computation or
    upload dominant; optimum inside or at the ends of [2, d])."""
    import numpy as np
    import oracle
    from paper_2203_13005_amd import binding as b
    rng = np.random.default_rng(7)
    cases = [(1, 2, 1, 4, 12), (4, 2, 1, 10, 100), (1, 2, 4, 10, 100), (1, 3, 1, 2, 100),
             (0.24e-9, 0.03e-9, 0.08e-9, 10e-6, 65_000_000 // 1000), (5, 1, 1, 1e-6, 1000), (1, 1, 1, 1e6, 50)]
    for _ in range(300):
        k = rng.exponential(1.0, 3) * rng.choice([0.01, 1, 100], 3)
        cases.append((k[0], k[1], k[2], float(rng.exponential(1.0) * rng.choice([0.01, 1, 100])),
                      int(rng.integers(2, 3000))))
    for k1, k2, k3, a, d in cases:
        s, bs, t = b.pipeline_plan(k1, k2, k3, a, d)
        s_bf, t_bf = oracle.pipeline_brute_force(k1, k2, k3, a, d)
        assert 2 <= s <= d and abs(bs - d / s) < 1e-9 * d
        assert t <= t_bf * (1 + 1e-9), (k1, k2, k3, a, d, s, t, s_bf, t_bf)


def test_pipeline_plan_validation():
    import pytest
    from paper_2203_13005_amd import binding as b
    with pytest.raises(b.GxError):
        b.pipeline_plan(1, 1, 1, 1, 1)  # fewer than 2 entities
    with pytest.raises(b.GxError):
        b.pipeline_plan(-1, 1, 1, 1, 100)
    assert b.lib.gx_stream_superstep(None, 1, 0, None) == b.GX_EINVAL
    assert b.lib.gx_stream_free(None) == b.GX_OK
