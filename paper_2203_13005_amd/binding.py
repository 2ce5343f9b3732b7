"""ctypes marshalling for libgx.so (see include/gx.h for the contract)."""
from __future__ import annotations

import atexit
import ctypes
import os
import weakref
from dataclasses import dataclass

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_PKG, "libgx.so")

GX_OK, GX_EINVAL, GX_ENOMEM, GX_EDEVICE, GX_ENOTCONVERGED, GX_EBUSY, GX_ENOTFOUND = range(7)
GX_PAGERANK, GX_SSSP, GX_CC, GX_PPR, GX_LP = 0, 1, 2, 3, 4
GX_NEED_OUT, GX_NEED_IN, GX_NEED_SYM = 1, 2, 4
GX_DELTA_REMOTE, GX_DELTA_ALL, GX_DELTA_MASTERS = 0, 1, 2
GX_PHASES_LOCAL, GX_PHASES_MASTERS = 1, 2
INF = 0xFFFFFFFF

_STATUS = {0: "GX_OK", 1: "GX_EINVAL", 2: "GX_ENOMEM", 3: "GX_EDEVICE", 4: "GX_ENOTCONVERGED",
           5: "GX_EBUSY", 6: "GX_ENOTFOUND"}


class GxError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class _GraphDesc(ctypes.Structure):
    _fields_ = [("V", ctypes.c_int64), ("E", ctypes.c_int64), ("row_ptr", ctypes.c_void_p),
                ("col", ctypes.c_void_p), ("w", ctypes.c_void_p), ("l2g", ctypes.c_void_p),
                ("flags", ctypes.c_void_p), ("needs", ctypes.c_uint32), ("pr_tile_edges", ctypes.c_uint32),
                ("V_global", ctypes.c_int64), ("outdeg_global", ctypes.c_void_p)]


class _Params(ctypes.Structure):
    _fields_ = [("algo", ctypes.c_int32), ("damping", ctypes.c_float), ("source", ctypes.c_int32),
                ("max_supersteps", ctypes.c_uint32), ("delta_mode", ctypes.c_uint32),
                ("timing", ctypes.c_uint32), ("pull_fraction", ctypes.c_float), ("phases", ctypes.c_uint32)]


class StepStats(ctypes.Structure):
    _fields_ = [("frontier", ctypes.c_int64), ("edges", ctypes.c_int64), ("changed", ctypes.c_int64),
                ("pulled", ctypes.c_int64), ("kernel_ms", ctypes.c_double)]

    def as_tuple(self):
        return (self.frontier, self.edges, self.changed)

    def as_dict(self):
        return dict(frontier=self.frontier, edges=self.edges, changed=self.changed, pulled=self.pulled,
                    kernel_ms=self.kernel_ms)


class RunStats(ctypes.Structure):
    _fields_ = [("supersteps", ctypes.c_int64), ("edges", ctypes.c_int64), ("converged", ctypes.c_int64),
                ("edge_kernel_ms", ctypes.c_double), ("edge_kernel_launches", ctypes.c_int64),
                ("wall_ms", ctypes.c_double)]


class Tune(ctypes.Structure):
    _fields_ = [("block", ctypes.c_uint32), ("tile", ctypes.c_uint32), ("width", ctypes.c_uint32),
                ("grid", ctypes.c_uint32)]

    def __repr__(self):
        return f"Tune(block={self.block}, tile={self.tile}, width={self.width}, grid={self.grid})"


class StreamStats(ctypes.Structure):
    _fields_ = [("blocks", ctypes.c_int64), ("triplets", ctypes.c_int64), ("messages", ctypes.c_int64),
                ("changed", ctypes.c_int64), ("wall_ms", ctypes.c_double), ("download_ms", ctypes.c_double),
                ("compute_ms", ctypes.c_double), ("upload_ms", ctypes.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class PipelineCoef(ctypes.Structure):
    _fields_ = [("k1", ctypes.c_double), ("k2", ctypes.c_double), ("k3", ctypes.c_double), ("a", ctypes.c_double)]


class _ServerConfig(ctypes.Structure):
    _fields_ = [("dev_arena", ctypes.c_void_p), ("arena_bytes", ctypes.c_size_t),
                ("lanes_per_pool", ctypes.c_uint32), ("max_pools", ctypes.c_uint32),
                ("epoch_supersteps", ctypes.c_uint32), ("damping", ctypes.c_float),
                ("ppr_iters", ctypes.c_uint32), ("sssp_epoch_supersteps", ctypes.c_uint32)]


class QueryResult(ctypes.Structure):
    _fields_ = [("id", ctypes.c_int64), ("graph", ctypes.c_int32), ("algo", ctypes.c_int32),
                ("source", ctypes.c_int32), ("status", ctypes.c_int32), ("submit_s", ctypes.c_double),
                ("start_s", ctypes.c_double), ("done_s", ctypes.c_double), ("supersteps", ctypes.c_int64)]


_P = ctypes.c_void_p
_SIGS = {
    "gx_last_error": (ctypes.c_char_p, []),
    "gx_version": (ctypes.c_char_p, []),
    "gx_graph_bytes": (ctypes.c_int32, [ctypes.POINTER(_GraphDesc), ctypes.POINTER(ctypes.c_size_t)]),
    "gx_graph_load": (ctypes.c_int32, [ctypes.POINTER(_GraphDesc), _P, ctypes.c_size_t, _P, ctypes.POINTER(_P)]),
    "gx_graph_free": (ctypes.c_int32, [_P]),
    "gx_graph_info": (ctypes.c_int32, [_P, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                                       ctypes.POINTER(ctypes.c_uint32)]),
    "gx_state_bytes": (ctypes.c_int32, [_P, ctypes.POINTER(_Params), ctypes.POINTER(ctypes.c_size_t)]),
    "gx_state_init": (ctypes.c_int32, [_P, ctypes.POINTER(_Params), _P, ctypes.c_size_t, _P, ctypes.POINTER(_P)]),
    "gx_state_free": (ctypes.c_int32, [_P]),
    "gx_state_values": (ctypes.c_int32, [_P, ctypes.POINTER(_P)]),
    "gx_state_frontier": (ctypes.c_int32, [_P, ctypes.POINTER(_P)]),
    "gx_state_superstep": (ctypes.c_int32, [_P, ctypes.POINTER(ctypes.c_int64)]),
    "gx_release_cached": (ctypes.c_int32, []),
    "gx_superstep": (ctypes.c_int32, [_P, _P, ctypes.POINTER(StepStats)]),
    "gx_run_until_converged": (ctypes.c_int32, [_P, ctypes.c_uint32, _P, ctypes.POINTER(RunStats),
                                                ctypes.POINTER(StepStats)]),
    "gx_sync_delta": (ctypes.c_int32, [_P, _P, _P, ctypes.c_uint32, ctypes.POINTER(ctypes.c_uint32),
                                       ctypes.POINTER(ctypes.c_int32), _P]),
    "gx_sync_delta_noalloc": (ctypes.c_int32, [_P, _P, _P, ctypes.c_uint32, _P, _P]),
    "gx_dangling_get": (ctypes.c_int32, [_P, ctypes.POINTER(ctypes.c_double), _P]),
    "gx_dangling_set": (ctypes.c_int32, [_P, ctypes.c_double, _P]),
    "gx_partial_emit": (ctypes.c_int32, [_P, _P, _P, ctypes.c_uint32, ctypes.POINTER(ctypes.c_uint32), _P]),
    "gx_partial_add": (ctypes.c_int32, [_P, _P, _P, ctypes.c_uint32, _P]),
    "gx_stream_bytes": (ctypes.c_int32, [_P, ctypes.c_int32, ctypes.c_uint64, ctypes.c_int32,
                                         ctypes.POINTER(ctypes.c_size_t)]),
    "gx_stream_create": (ctypes.c_int32, [_P, ctypes.c_int32, ctypes.c_int32, _P, ctypes.c_size_t, ctypes.c_uint64,
                                          ctypes.c_int32, ctypes.POINTER(_P)]),
    "gx_stream_reset": (ctypes.c_int32, [_P]),
    "gx_stream_superstep": (ctypes.c_int32, [_P, ctypes.c_uint64, ctypes.c_uint32, ctypes.POINTER(StreamStats)]),
    "gx_stream_values": (ctypes.c_int32, [_P, ctypes.POINTER(_P), ctypes.POINTER(_P)]),
    "gx_stream_results": (ctypes.c_int32, [_P, ctypes.POINTER(ctypes.POINTER(ctypes.c_uint32)),
                                           ctypes.POINTER(ctypes.c_int64)]),
    "gx_stream_free": (ctypes.c_int32, [_P]),
    "gx_pipeline_time": (ctypes.c_int32, [ctypes.POINTER(PipelineCoef), ctypes.c_double, ctypes.c_double,
                                          ctypes.POINTER(ctypes.c_double)]),
    "gx_pipeline_plan": (ctypes.c_int32, [ctypes.POINTER(PipelineCoef), ctypes.c_int64, ctypes.POINTER(ctypes.c_int64),
                                          ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]),
    "gx_cpu_create": (ctypes.c_int32, [_P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(_P)]),
    "gx_cpu_superstep": (ctypes.c_int32, [_P, ctypes.POINTER(StepStats)]),
    "gx_cpu_sync_delta": (ctypes.c_int32, [_P, _P, _P, ctypes.c_uint32, ctypes.POINTER(ctypes.c_uint32)]),
    "gx_cpu_apply_delta": (ctypes.c_int32, [_P, _P, _P, ctypes.c_uint32, ctypes.POINTER(ctypes.c_int64)]),
    "gx_cpu_values": (ctypes.c_int32, [_P, ctypes.POINTER(ctypes.POINTER(ctypes.c_uint32))]),
    "gx_cpu_free": (ctypes.c_int32, [_P]),
    "gx_balance_split": (ctypes.c_int32, [_P, ctypes.c_int32, ctypes.c_double, _P]),
    "gx_msg_gen": (ctypes.c_int32, [_P, _P]),
    "gx_msg_merge": (ctypes.c_int32, [_P, _P]),
    "gx_msg_apply": (ctypes.c_int32, [_P, _P, ctypes.POINTER(StepStats)]),
    "gx_apply_delta": (ctypes.c_int32, [_P, _P, _P, ctypes.c_uint32, ctypes.POINTER(ctypes.c_int64), _P]),
    "gx_batch_bytes": (ctypes.c_int32, [_P, ctypes.c_int32, ctypes.c_uint32, ctypes.POINTER(ctypes.c_size_t)]),
    "gx_batch_run": (ctypes.c_int32, [_P, ctypes.c_int32, _P, ctypes.c_uint32, ctypes.c_float, ctypes.c_uint32,
                                      _P, ctypes.c_size_t, _P, ctypes.POINTER(Tune), _P,
                                      ctypes.POINTER(RunStats)]),
    "gx_batch_autotune": (ctypes.c_int32, [_P, ctypes.c_int32, _P, ctypes.c_uint32, ctypes.c_float,
                                           ctypes.c_uint32, _P, ctypes.c_size_t, _P, _P, ctypes.POINTER(Tune),
                                           ctypes.POINTER(ctypes.c_double)]),
    "gx_server_bytes_per_lane": (ctypes.c_int32, [_P, ctypes.c_int32, ctypes.POINTER(ctypes.c_size_t)]),
    "gx_server_create": (ctypes.c_int32, [ctypes.POINTER(_ServerConfig), ctypes.POINTER(_P)]),
    "gx_server_add_graph": (ctypes.c_int32, [_P, _P, ctypes.POINTER(ctypes.c_int32)]),
    "gx_server_submit": (ctypes.c_int32, [_P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _P,
                                          ctypes.POINTER(ctypes.c_int64)]),
    "gx_server_poll": (ctypes.c_int32, [_P, ctypes.POINTER(QueryResult), ctypes.c_uint32,
                                        ctypes.POINTER(ctypes.c_uint32), ctypes.c_int32]),
    "gx_server_pending": (ctypes.c_int32, [_P, ctypes.POINTER(ctypes.c_int64)]),
    "gx_server_destroy": (ctypes.c_int32, [_P]),
}


def library_path() -> str:
    return _LIB_PATH


def _load():
    if not os.path.exists(_LIB_PATH):
        raise ImportError(f"{_LIB_PATH} is not built; run __graft_entry__.build() "
                          "(hipcc --offload-arch=gfx950).  There is no CPU fallback.")
    L = ctypes.CDLL(_LIB_PATH)
    for name, (res, args) in _SIGS.items():
        f = getattr(L, name, None)
        if f is None:
            continue
        f.restype = res
        f.argtypes = args
    return L


lib = _load()


# Handles still open at interpreter exit are closed before the HIP runtime
# tears down (servers, then states, then graphs), and the library's cached
# events and pinned buffers are freed after them.
_live: "weakref.WeakSet" = weakref.WeakSet()


def _close_all_at_exit():
    for kind in ("Server", "Stream", "CpuPart", "State", "DeviceGraph"):
        for obj in list(_live):
            if type(obj).__name__ == kind:
                try:
                    obj.close()
                except Exception:
                    pass
    try:
        lib.gx_release_cached()
    except Exception:
        pass


atexit.register(_close_all_at_exit)


def exported_symbols() -> list[str]:
    return [n for n in _SIGS if getattr(lib, n, None) is not None]


def _check(st: int):
    if st != GX_OK:
        raise GxError(st, lib.gx_last_error().decode(errors="replace"))


def _np_ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _stream_handle(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _arena(nbytes: int, device):
    import torch
    t = torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)
    if t.data_ptr() % 256:
        raise GxError(GX_EINVAL, "torch returned a device buffer that is not 256-byte aligned")
    return t


class DeviceGraph:
    """A worker's graph resident in HBM.  ``host`` is any object with V, E,
    row_ptr, col, w and optional l2g / flags numpy arrays (out-CSR)."""

    def __init__(self, host, needs: int, device="cuda:0", stream=None, pr_tile_edges: int = 0,
                 V_global: int = 0, outdeg_global=None):
        import torch
        self.device = torch.device(device)
        self._keep = [np.ascontiguousarray(host.row_ptr, np.int32), np.ascontiguousarray(host.col, np.int32),
                      None if host.w is None else np.ascontiguousarray(host.w, np.uint32),
                      None if getattr(host, "l2g", None) is None else np.ascontiguousarray(host.l2g, np.int32),
                      None if getattr(host, "flags", None) is None else np.ascontiguousarray(host.flags, np.uint8),
                      None if outdeg_global is None else np.ascontiguousarray(outdeg_global, np.int32)]
        rp, col, w, l2g, flags, odg = self._keep
        self.desc = _GraphDesc(int(host.V), int(host.E), _np_ptr(rp), _np_ptr(col), _np_ptr(w), _np_ptr(l2g),
                               _np_ptr(flags), int(needs), int(pr_tile_edges), int(V_global), _np_ptr(odg))
        nbytes = ctypes.c_size_t(0)
        _check(lib.gx_graph_bytes(ctypes.byref(self.desc), ctypes.byref(nbytes)))
        self.arena_bytes = nbytes.value
        with torch.cuda.device(self.device):
            self.arena = _arena(nbytes.value, self.device)
            h = ctypes.c_void_p()
            _check(lib.gx_graph_load(ctypes.byref(self.desc), ctypes.c_void_p(self.arena.data_ptr()), nbytes.value,
                                     _stream_handle(stream), ctypes.byref(h)))
        self.handle = h
        self.V, self.E, self.needs = int(host.V), int(host.E), int(needs)
        self._keep = None
        _live.add(self)

    def close(self):
        if getattr(self, "handle", None):
            lib.gx_graph_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class State:
    """Vertex state of one algorithm on a DeviceGraph (caller-owned memory)."""

    def __init__(self, graph: DeviceGraph, algo: int, source: int = 0, damping: float = 0.85,
                 max_supersteps: int = 1 << 20, delta_mode: int = GX_DELTA_REMOTE, timing: bool = False,
                 pull_fraction: float = 0.0, stream=None, phases: int = 0):
        import torch
        self.graph = graph
        self.algo = algo
        self.params = _Params(int(algo), float(damping), int(source), int(max_supersteps), int(delta_mode),
                              int(bool(timing)), float(pull_fraction), int(phases))
        nbytes = ctypes.c_size_t(0)
        _check(lib.gx_state_bytes(graph.handle, ctypes.byref(self.params), ctypes.byref(nbytes)))
        with torch.cuda.device(graph.device):
            self.mem = _arena(nbytes.value, graph.device)
            h = ctypes.c_void_p()
            _check(lib.gx_state_init(graph.handle, ctypes.byref(self.params), ctypes.c_void_p(self.mem.data_ptr()),
                                     nbytes.value, _stream_handle(stream), ctypes.byref(h)))
        self.handle = h
        _live.add(self)

    def reset(self, stream=None):
        """Re-initialises the state in the same device memory (no allocation)."""
        self.close()
        h = ctypes.c_void_p()
        _check(lib.gx_state_init(self.graph.handle, ctypes.byref(self.params), ctypes.c_void_p(self.mem.data_ptr()),
                                 self.mem.numel(), _stream_handle(stream), ctypes.byref(h)))
        self.handle = h

    def _view(self, ptr: int, nbytes: int):
        off = ptr - self.mem.data_ptr()
        assert 0 <= off and off + nbytes <= self.mem.numel()
        return self.mem[off: off + nbytes]

    def values(self):
        """Device view of the current values (float32 for PageRank, int32
        bit pattern of uint32 otherwise)."""
        import torch
        p = ctypes.c_void_p()
        _check(lib.gx_state_values(self.handle, ctypes.byref(p)))
        v = self._view(p.value, 4 * self.graph.V)
        return v.view(torch.float32) if self.algo == GX_PAGERANK else v.view(torch.int32)

    def values_numpy(self) -> np.ndarray:
        import torch
        torch.cuda.synchronize(self.graph.device)
        a = self.values().cpu().numpy()
        return a if self.algo == GX_PAGERANK else a.view(np.uint32)

    def frontier_device(self):
        """Device view (uint8 per vertex, nonzero = active in the next
        superstep) of the current frontier byte map."""
        p = ctypes.c_void_p()
        _check(lib.gx_state_frontier(self.handle, ctypes.byref(p)))
        return self._view(p.value, self.graph.V)

    def frontier_numpy(self) -> np.ndarray:
        """Boolean frontier (vertices active in the next superstep)."""
        import torch
        v = self.frontier_device()
        torch.cuda.synchronize(self.graph.device)
        return v.cpu().numpy() != 0

    @property
    def superstep_index(self) -> int:
        k = ctypes.c_int64()
        _check(lib.gx_state_superstep(self.handle, ctypes.byref(k)))
        return k.value

    def superstep(self, stats: bool = True, stream=None):
        st = StepStats()
        _check(lib.gx_superstep(self.handle, _stream_handle(stream), ctypes.byref(st) if stats else None))
        return st.as_tuple() if stats else None

    def run(self, max_supersteps: int, stream=None, per_step: bool = False, allow_cap: bool = False,
            detail: bool = False):
        rs = RunStats()
        ps = (StepStats * max(1, max_supersteps))() if per_step else None
        st = lib.gx_run_until_converged(self.handle, int(max_supersteps), _stream_handle(stream), ctypes.byref(rs),
                                        ps)
        if not (st == GX_ENOTCONVERGED and allow_cap):
            _check(st)
        steps = None
        if per_step:
            steps = [(ps[i].as_dict() if detail else ps[i].as_tuple()) for i in range(rs.supersteps)]
        return rs, steps

    def sync_delta(self, cap: int | None = None, stream=None, on_device: bool = False, out=None):
        """Returns (gids int32, value bits uint32, skippable) as numpy arrays, or
        as device tensors (int32 bit patterns) with on_device=True.  `out`
        optionally supplies the two int32 device buffers (at least `cap`
        elements each) instead of allocating them per call."""
        import torch
        cap = self.graph.V if cap is None else int(cap)
        if out is not None:
            gid, val = out
            if (gid.dtype != torch.int32 or val.dtype != torch.int32 or gid.numel() < cap or val.numel() < cap
                    or not gid.is_contiguous() or not val.is_contiguous()):
                raise ValueError("out must be two contiguous int32 device tensors of at least cap elements")
        else:
            gid = torch.empty(max(cap, 1), dtype=torch.int32, device=self.graph.device)
            val = torch.empty(max(cap, 1), dtype=torch.int32, device=self.graph.device)
        n = ctypes.c_uint32()
        sk = ctypes.c_int32()
        _check(lib.gx_sync_delta(self.handle, ctypes.c_void_p(gid.data_ptr()), ctypes.c_void_p(val.data_ptr()),
                                 cap, ctypes.byref(n), ctypes.byref(sk), _stream_handle(stream)))
        c = n.value
        if on_device:
            return gid[:c], val[:c], bool(sk.value)
        return gid[:c].cpu().numpy(), val[:c].cpu().numpy().view(np.uint32), bool(sk.value)

    def msg_gen(self, stream=None):
        """MSGGen (separate template calls; state created with phases=True)."""
        _check(lib.gx_msg_gen(self.handle, _stream_handle(stream)))

    def msg_merge(self, stream=None):
        """MSGMerge: combines the pending messages per destination."""
        _check(lib.gx_msg_merge(self.handle, _stream_handle(stream)))

    def msg_apply(self, stats: bool = True, stream=None):
        """MSGApply; with stats, returns (active, messages, changed) of the
        superstep it completed (zeros when nothing was merged)."""
        st = StepStats()
        _check(lib.gx_msg_apply(self.handle, _stream_handle(stream), ctypes.byref(st) if stats else None))
        return st.as_tuple() if stats else None

    def dangling_get(self, stream=None) -> float:
        """This part's masters' dangling mass from the last MSGGen (GX_PHASES_MASTERS)."""
        m = ctypes.c_double()
        _check(lib.gx_dangling_get(self.handle, ctypes.byref(m), _stream_handle(stream)))
        return m.value

    def dangling_set(self, mass: float, stream=None):
        _check(lib.gx_dangling_set(self.handle, float(mass), _stream_handle(stream)))

    def partial_emit(self, cap: int | None = None, stream=None):
        """(gid int32, sum float64) device tensors of the merged sums this part
        sends to the replicas' masters."""
        import torch
        cap = self.graph.V if cap is None else int(cap)
        gid = torch.empty(max(cap, 1), dtype=torch.int32, device=self.graph.device)
        val = torch.empty(max(cap, 1), dtype=torch.float64, device=self.graph.device)
        n = ctypes.c_uint32()
        _check(lib.gx_partial_emit(self.handle, ctypes.c_void_p(gid.data_ptr()), ctypes.c_void_p(val.data_ptr()),
                                   cap, ctypes.byref(n), _stream_handle(stream)))
        return gid[:n.value], val[:n.value]

    def partial_add(self, gid, val, stream=None):
        n = int(gid.numel())
        _check(lib.gx_partial_add(self.handle, ctypes.c_void_p(gid.data_ptr()) if n else None,
                                  ctypes.c_void_p(val.data_ptr()) if n else None, n, _stream_handle(stream)))

    def sync_delta_noalloc(self, gid, val, count, stream=None):
        """gx_sync_delta_noalloc: writes up to gid.numel() pairs into the given
        int32 device tensors and the pair count into the one-element int32
        device tensor `count`; asynchronous, allocates nothing."""
        import torch
        for t in (gid, val, count):
            if t.dtype != torch.int32 or not t.is_contiguous() or t.device.type != "cuda":
                raise ValueError("gid, val and count must be contiguous int32 device tensors")
        cap = min(gid.numel(), val.numel())
        _check(lib.gx_sync_delta_noalloc(self.handle, ctypes.c_void_p(gid.data_ptr()),
                                         ctypes.c_void_p(val.data_ptr()), cap, ctypes.c_void_p(count.data_ptr()),
                                         _stream_handle(stream)))

    def apply_delta(self, gids, vals, stream=None) -> int:
        """Merges (global id, value) pairs that other parts emitted (device int32
        tensors, values as bit patterns) into this part's replicas; returns the
        number of vertices active in the next superstep."""
        n = int(gids.numel())
        act = ctypes.c_int64()
        _check(lib.gx_apply_delta(self.handle, ctypes.c_void_p(gids.data_ptr()) if n else None,
                                  ctypes.c_void_p(vals.data_ptr()) if n else None, n, ctypes.byref(act),
                                  _stream_handle(stream)))
        return act.value

    def close(self):
        if getattr(self, "handle", None):
            lib.gx_state_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def batch_run(graph: DeviceGraph, algo: int, sources, damping: float = 0.85, iters: int = 50,
              tune: Tune | None = None, out=None, stream=None):
    """B lanes in one persistent launch; returns ([V, B] tensor, RunStats)."""
    import torch
    src = np.ascontiguousarray(sources, np.int32)
    B = len(src)
    nbytes = ctypes.c_size_t(0)
    _check(lib.gx_batch_bytes(graph.handle, int(algo), B, ctypes.byref(nbytes)))
    with torch.cuda.device(graph.device):
        work = _arena(nbytes.value, graph.device)
        if out is None:
            out = torch.empty((graph.V, B), dtype=torch.float32 if algo == GX_PPR else torch.int32,
                              device=graph.device)
        rs = RunStats()
        _check(lib.gx_batch_run(graph.handle, int(algo), _np_ptr(src), B, float(damping), int(iters),
                                ctypes.c_void_p(work.data_ptr()), nbytes.value, ctypes.c_void_p(out.data_ptr()),
                                ctypes.byref(tune) if tune is not None else None, _stream_handle(stream),
                                ctypes.byref(rs)))
    return out, rs


def batch_autotune(graph: DeviceGraph, algo: int, sources, damping: float = 0.85, iters: int = 50, stream=None):
    import torch
    src = np.ascontiguousarray(sources, np.int32)
    B = len(src)
    nbytes = ctypes.c_size_t(0)
    _check(lib.gx_batch_bytes(graph.handle, int(algo), B, ctypes.byref(nbytes)))
    with torch.cuda.device(graph.device):
        work = _arena(nbytes.value, graph.device)
        out = torch.empty((graph.V, B), dtype=torch.float32 if algo == GX_PPR else torch.int32, device=graph.device)
        best = Tune()
        ms = ctypes.c_double()
        _check(lib.gx_batch_autotune(graph.handle, int(algo), _np_ptr(src), B, float(damping), int(iters),
                                     ctypes.c_void_p(work.data_ptr()), nbytes.value,
                                     ctypes.c_void_p(out.data_ptr()), _stream_handle(stream), ctypes.byref(best),
                                     ctypes.byref(ms)))
    return best, ms.value


@dataclass
class Completed:
    id: int
    graph: int
    algo: int
    source: int
    status: int
    submit_s: float
    start_s: float
    done_s: float
    supersteps: int
    result: np.ndarray

    @property
    def latency_s(self) -> float:
        return self.done_s - self.submit_s


class Server:
    """Continuous-batching query server over resident graphs."""

    def __init__(self, arena_bytes: int, lanes_per_pool: int = 64, max_pools: int = 4, epoch_supersteps: int = 4,
                 damping: float = 0.85, ppr_iters: int = 50, sssp_epoch_supersteps: int = 16, device="cuda:0"):
        import torch
        self.device = torch.device(device)
        with torch.cuda.device(self.device):
            self.arena = _arena(arena_bytes, self.device)
        cfg = _ServerConfig(ctypes.c_void_p(self.arena.data_ptr()), int(arena_bytes), int(lanes_per_pool),
                            int(max_pools), int(epoch_supersteps), float(damping), int(ppr_iters),
                            int(sssp_epoch_supersteps))
        h = ctypes.c_void_p()
        _check(lib.gx_server_create(ctypes.byref(cfg), ctypes.byref(h)))
        self.handle = h
        _live.add(self)
        self.graphs: list[DeviceGraph] = []
        self._buffers: dict[int, np.ndarray] = {}

    def add_graph(self, g: DeviceGraph) -> int:
        gid = ctypes.c_int32()
        _check(lib.gx_server_add_graph(self.handle, g.handle, ctypes.byref(gid)))
        self.graphs.append(g)
        return gid.value

    def submit(self, graph_id: int, algo: int, source: int) -> int:
        V = self.graphs[graph_id].V
        buf = np.empty(V, np.float32 if algo == GX_PPR else np.uint32)
        qid = ctypes.c_int64()
        _check(lib.gx_server_submit(self.handle, int(graph_id), int(algo), int(source), _np_ptr(buf),
                                    ctypes.byref(qid)))
        self._buffers[qid.value] = buf
        return qid.value

    def poll(self, cap: int = 256, wait_ms: int = 0) -> list[Completed]:
        arr = (QueryResult * cap)()
        n = ctypes.c_uint32()
        _check(lib.gx_server_poll(self.handle, arr, cap, ctypes.byref(n), int(wait_ms)))
        out = []
        for i in range(n.value):
            r = arr[i]
            out.append(Completed(r.id, r.graph, r.algo, r.source, r.status, r.submit_s, r.start_s, r.done_s,
                                 r.supersteps, self._buffers.pop(r.id)))
        return out

    def pending(self) -> int:
        n = ctypes.c_int64()
        _check(lib.gx_server_pending(self.handle, ctypes.byref(n)))
        return n.value

    def close(self):
        if getattr(self, "handle", None):
            lib.gx_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


GX_STREAM_PIPELINED, GX_STREAM_SERIAL = 0, 1


def pipeline_plan(k1: float, k2: float, k3: float, a: float, d: int):
    """Lemma "bSizeSelection" with the floor/ceiling rule: (blocks, block size, modelled time)."""
    s, b, t = ctypes.c_int64(), ctypes.c_double(), ctypes.c_double()
    _check(lib.gx_pipeline_plan(ctypes.byref(PipelineCoef(k1, k2, k3, a)), int(d), ctypes.byref(s), ctypes.byref(b),
                                ctypes.byref(t)))
    return s.value, b.value, t.value


class Stream:
    """Streamed supersteps: the triplets in pinned host memory, blocks of them
    through three rotating device buffers per superstep."""

    def __init__(self, host, algo: int, source: int = 0, block_edges_max: int = 1 << 20, ring: int = 3,
                 device="cuda:0"):
        import torch
        self.device = torch.device(device)
        keep = [np.ascontiguousarray(host.row_ptr, np.int32), np.ascontiguousarray(host.col, np.int32),
                None if host.w is None else np.ascontiguousarray(host.w, np.uint32),
                None if getattr(host, "l2g", None) is None else np.ascontiguousarray(host.l2g, np.int32)]
        rp, col, w, l2g = keep
        desc = _GraphDesc(int(host.V), int(host.E), _np_ptr(rp), _np_ptr(col), _np_ptr(w), _np_ptr(l2g), None,
                          GX_NEED_OUT, 0, 0, None)
        nbytes = ctypes.c_size_t()
        _check(lib.gx_stream_bytes(ctypes.byref(desc), int(algo), int(block_edges_max), int(ring),
                                   ctypes.byref(nbytes)))
        with torch.cuda.device(self.device):
            self.mem = _arena(nbytes.value, self.device)
            h = ctypes.c_void_p()
            _check(lib.gx_stream_create(ctypes.byref(desc), int(algo), int(source), ctypes.c_void_p(self.mem.data_ptr()),
                                        nbytes.value, int(block_edges_max), int(ring), ctypes.byref(h)))
        self.handle = h
        self.V, self.algo = int(host.V), int(algo)
        _live.add(self)

    def reset(self):
        _check(lib.gx_stream_reset(self.handle))

    def superstep(self, block_edges: int, serial: bool = False) -> dict:
        st = StreamStats()
        _check(lib.gx_stream_superstep(self.handle, int(block_edges), GX_STREAM_SERIAL if serial else GX_STREAM_PIPELINED,
                                       ctypes.byref(st)))
        return st.as_dict()

    def _dev(self, which: int, dtype_bytes: int):
        import torch
        v, f = ctypes.c_void_p(), ctypes.c_void_p()
        _check(lib.gx_stream_values(self.handle, ctypes.byref(v), ctypes.byref(f)))
        p = (v, f)[which].value
        off = p - self.mem.data_ptr()
        return self.mem[off: off + dtype_bytes * self.V]

    def values_numpy(self) -> np.ndarray:
        import torch
        torch.cuda.synchronize(self.device)
        return self._dev(0, 4).cpu().numpy().view(np.uint32)

    def frontier_numpy(self) -> np.ndarray:
        import torch
        torch.cuda.synchronize(self.device)
        return self._dev(1, 1).cpu().numpy() != 0

    def results_numpy(self) -> np.ndarray:
        """Messages the last superstep uploaded, one per triplet (a copy)."""
        p = ctypes.POINTER(ctypes.c_uint32)()
        n = ctypes.c_int64()
        _check(lib.gx_stream_results(self.handle, ctypes.byref(p), ctypes.byref(n)))
        return np.ctypeslib.as_array(p, shape=(max(n.value, 1),))[: n.value].copy()

    def close(self):
        if getattr(self, "handle", None):
            lib.gx_stream_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def balance_split(c, D: float) -> np.ndarray:
    """Lemma "minmaxcidi": entities per worker, d_j proportional to 1 / c_j."""
    cc = np.ascontiguousarray(c, np.float64)
    out = np.empty(len(cc), np.float64)
    _check(lib.gx_balance_split(_np_ptr(cc), len(cc), float(D), _np_ptr(out)))
    return out


class CpuPart:
    """A part run by the CPU daemon (host threads), exchanging sync sets like
    a State with GX_DELTA_ALL."""

    def __init__(self, host, algo: int, source: int = 0, threads: int = 0):
        self._keep = [np.ascontiguousarray(host.row_ptr, np.int32), np.ascontiguousarray(host.col, np.int32),
                      None if host.w is None else np.ascontiguousarray(host.w, np.uint32),
                      None if getattr(host, "l2g", None) is None else np.ascontiguousarray(host.l2g, np.int32),
                      None if getattr(host, "flags", None) is None else np.ascontiguousarray(host.flags, np.uint8)]
        rp, col, w, l2g, flags = self._keep
        desc = _GraphDesc(int(host.V), int(host.E), _np_ptr(rp), _np_ptr(col), _np_ptr(w), _np_ptr(l2g),
                          _np_ptr(flags), GX_NEED_OUT, 0, 0, None)
        h = ctypes.c_void_p()
        _check(lib.gx_cpu_create(ctypes.byref(desc), int(algo), int(source), int(threads), ctypes.byref(h)))
        self.handle, self.V = h, int(host.V)
        self._keep = None
        _live.add(self)

    def superstep(self):
        st = StepStats()
        _check(lib.gx_cpu_superstep(self.handle, ctypes.byref(st)))
        return st.as_tuple()

    def sync_delta(self):
        gid = np.empty(max(self.V, 1), np.int32)
        val = np.empty(max(self.V, 1), np.uint32)
        n = ctypes.c_uint32()
        _check(lib.gx_cpu_sync_delta(self.handle, _np_ptr(gid), _np_ptr(val), self.V, ctypes.byref(n)))
        return gid[:n.value], val[:n.value]

    def apply_delta(self, gid, val) -> int:
        g = np.ascontiguousarray(gid, np.int32)
        v = np.ascontiguousarray(val, np.uint32)
        act = ctypes.c_int64()
        _check(lib.gx_cpu_apply_delta(self.handle, _np_ptr(g) if len(g) else None, _np_ptr(v) if len(v) else None,
                                      len(g), ctypes.byref(act)))
        return act.value

    def values_numpy(self) -> np.ndarray:
        p = ctypes.POINTER(ctypes.c_uint32)()
        _check(lib.gx_cpu_values(self.handle, ctypes.byref(p)))
        return np.ctypeslib.as_array(p, shape=(max(self.V, 1),))[: self.V].copy()

    def close(self):
        if getattr(self, "handle", None):
            lib.gx_cpu_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
