"""Seeded synthetic inputs shared by the CPU oracle and the device library.

This package only generates input graphs (R-MAT edges, weights, a hash
vertex-cut) and seeded source/seed vertex choices.  It contains none of the
graph algorithms' arithmetic.  The heavy lifting is in ``rmat.c`` (plain C +
OpenMP), loaded through ctypes.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rmat.c")
_LIB = os.path.join(_HERE, "_rmat.so")
_lib = None

# R-MAT quadrant probabilities used by every workload (d = 1 - a - b - c = 0.05).
RMAT_A, RMAT_B, RMAT_C = 0.57, 0.19, 0.19


def build(force: bool = False) -> str:
    """Compile rmat.c into _rmat.so (gcc, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O3", "-march=x86-64-v2", "-fopenmp", "-shared", "-fPIC",
                               "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        lib.gen_rmat_csr.restype = ctypes.c_int64
        lib.gen_rmat_csr.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                                     ctypes.c_double, ctypes.c_uint64, P, P, P]
        lib.gen_rmat_part.restype = ctypes.c_int
        PP = ctypes.POINTER(ctypes.c_void_p)
        lib.gen_rmat_part.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                                      ctypes.c_double, ctypes.c_uint64, ctypes.c_int, ctypes.c_int,
                                      P, P, PP, PP, PP, PP, PP]
        lib.gen_free.restype = None
        lib.gen_free.argtypes = [P]
        lib.gen_rmat_quadrants.restype = None
        lib.gen_rmat_quadrants.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                                           ctypes.c_double, ctypes.c_uint64, P]
        _lib = lib
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


@dataclass
class Graph:
    """A directed graph as out-CSR with rows sorted by destination.

    ``l2g`` / ``flags`` are set for one part of a vertex-cut: local vertex x
    is global vertex l2g[x]; flags bit0 master, bit1 remote_out, bit2
    remote_any.
    """
    V: int
    E: int
    row_ptr: np.ndarray            # int32 [V+1]
    col: np.ndarray                # int32 [E]
    w: np.ndarray                  # uint32 [E], in [1, 255]
    l2g: np.ndarray | None = None  # int32 [V]
    flags: np.ndarray | None = None  # uint8 [V]
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def src(self) -> np.ndarray:
        return np.repeat(np.arange(self.V, dtype=np.int32), np.diff(self.row_ptr))

    def outdeg(self) -> np.ndarray:
        return np.diff(self.row_ptr).astype(np.int32)


def rmat(scale: int, edge_factor: int = 16, seed: int = 1,
         a: float = RMAT_A, b: float = RMAT_B, c: float = RMAT_C, E_raw: int | None = None) -> Graph:
    """Whole R-MAT graph, self-loops and duplicates removed."""
    lib = _load()
    V = 1 << scale
    if E_raw is None:
        E_raw = edge_factor * V
    row_ptr = np.empty(V + 1, np.int32)
    col = np.empty(max(E_raw, 1), np.int32)
    w = np.empty(max(E_raw, 1), np.uint32)
    E = lib.gen_rmat_csr(scale, E_raw, a, b, c, seed, _p(row_ptr), _p(col), _p(w))
    if E < 0:
        raise RuntimeError("gen_rmat_csr failed")
    return Graph(V, int(E), row_ptr, col[:E].copy(), w[:E].copy(),
                 name=f"rmat{scale}_s{seed}", meta=dict(scale=scale, E_raw=E_raw, seed=seed))


def rmat_part(scale: int, edge_factor: int = 16, seed: int = 3, nparts: int = 8, part: int = 0,
              a: float = RMAT_A, b: float = RMAT_B, c: float = RMAT_C, E_raw: int | None = None) -> Graph:
    """One part of a hash vertex-cut of an R-MAT graph (local ids, l2g, flags)."""
    lib = _load()
    if E_raw is None:
        E_raw = edge_factor * (1 << scale)
    Vp = ctypes.c_int64(0)
    Ep = ctypes.c_int64(0)
    ptrs = [ctypes.c_void_p() for _ in range(5)]
    rc = lib.gen_rmat_part(scale, E_raw, a, b, c, seed, nparts, part, ctypes.byref(Vp), ctypes.byref(Ep),
                           *[ctypes.byref(p) for p in ptrs])
    if rc != 0:
        raise RuntimeError("gen_rmat_part failed")
    V, E = Vp.value, Ep.value

    def take(p, n, dt):
        out = np.empty(n, dt)
        if n:
            ctypes.memmove(out.ctypes.data, p.value, n * np.dtype(dt).itemsize)
        lib.gen_free(p)
        return out

    row_ptr = take(ptrs[0], V + 1, np.int32)
    col = take(ptrs[1], E, np.int32)
    w = take(ptrs[2], E, np.uint32)
    l2g = take(ptrs[3], V, np.int32)
    flags = take(ptrs[4], V, np.uint8)
    return Graph(V, E, row_ptr, col, w, l2g, flags,
                 name=f"rmat{scale}_s{seed}_p{part}of{nparts}",
                 meta=dict(scale=scale, E_raw=E_raw, seed=seed, nparts=nparts, part=part))


def cover_isolated(parts: list, V_global: int) -> list:
    """The parts of a vertex-cut with every global vertex that no part holds
    (no edge at all) added to part 0 as a master without edges, so that each
    global vertex lives in exactly one master part.  Local ids stay sorted by
    global id; part 0's rows are re-indexed accordingly."""
    covered = np.zeros(V_global, bool)
    for p in parts:
        covered[p.l2g] = True
    iso = np.nonzero(~covered)[0].astype(np.int32)
    if len(iso) == 0:
        return list(parts)
    p0 = parts[0]
    l2g = np.union1d(p0.l2g, iso).astype(np.int32)
    pos = np.searchsorted(l2g, p0.l2g)
    deg = np.zeros(len(l2g), np.int64)
    deg[pos] = np.diff(p0.row_ptr)
    row_ptr = np.r_[0, np.cumsum(deg)].astype(np.int32)
    flags = np.full(len(l2g), 1, np.uint8)  # master, no remote edge
    flags[pos] = p0.flags
    q = Graph(len(l2g), p0.E, row_ptr, pos[p0.col].astype(np.int32), p0.w.copy(), l2g, flags,
              name=p0.name + "_covered", meta=dict(p0.meta, isolated_added=int(len(iso))))
    return [q] + list(parts[1:])


def _splitmix64(x: np.ndarray) -> np.ndarray:
    """SplitMix64 finaliser (Steele, Lea and Flood 2014), vectorised."""
    z = (x + np.uint64(0x9E3779B97F4A7C15)).astype(np.uint64)
    z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
    z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
    return z ^ (z >> np.uint64(31))


def _subgraph(src, dst, w, name, other_out=None, other_any=None, master=None):
    l2g = np.unique(np.r_[src, dst]).astype(np.int32)
    u = np.searchsorted(l2g, src)
    v = np.searchsorted(l2g, dst)
    order = np.lexsort((v, u))
    u, v, w = u[order], v[order], w[order]
    row_ptr = np.r_[0, np.cumsum(np.bincount(u, minlength=len(l2g)))].astype(np.int32)
    flags = np.zeros(len(l2g), np.uint8)
    if master is not None:
        flags |= master[l2g].astype(np.uint8)
        flags |= (other_out[l2g].astype(np.uint8) << 1) | (other_any[l2g].astype(np.uint8) << 2)
    return Graph(len(l2g), len(u), row_ptr, v.astype(np.int32), w.astype(np.uint32), l2g, flags, name=name)


def split_by_share(g: Graph, share: float, seed: int = 11) -> list:
    """Two parts of a vertex-cut by edge hash: an edge goes to part 1 when the
    SplitMix64 hash of (seed, u, v), scaled to [0, 1), is below `share`,
    else to part 0.  Local ids are sorted global ids; flags mark masters and
    the vertices the other part also holds."""
    src = g.src.astype(np.int64)
    dst = g.col.astype(np.int64)
    key = ((src.astype(np.uint64) << np.uint64(32)) | dst.astype(np.uint64)) ^ np.uint64(seed)
    h = (_splitmix64(key) >> np.uint64(11)).astype(np.float64) / float(1 << 53)
    one = h < share
    out_in, any_in = [], []
    for sel in (~one, one):
        o = np.zeros(g.V, bool)
        o[src[sel]] = True
        a = o.copy()
        a[dst[sel]] = True
        out_in.append(o)
        any_in.append(a)
    # flags: bit 0 master (part 0 when it holds the vertex), bit 1 an out-edge
    # in the other part, bit 2 any edge in the other part
    m0 = any_in[0]
    return [_subgraph(src[~one], dst[~one], g.w[~one], g.name + "_p0", out_in[1], any_in[1], m0),
            _subgraph(src[one], dst[one], g.w[one], g.name + "_p1", out_in[0], any_in[0], ~m0)]


def quadrant_counts(scale: int, n: int, seed: int, a: float = RMAT_A, b: float = RMAT_B,
                    c: float = RMAT_C) -> np.ndarray:
    lib = _load()
    out = np.zeros(4, np.int64)
    lib.gen_rmat_quadrants(scale, n, a, b, c, seed, _p(out))
    return out


def from_edges(V: int, src, dst, w=None, name: str = "custom") -> Graph:
    """Graph from an explicit edge list (self-loops dropped, duplicates merged,
    the smallest weight kept for a duplicated pair)."""
    src = np.asarray(src, np.int64)
    dst = np.asarray(dst, np.int64)
    if w is None:
        w = np.ones(len(src), np.uint32)
    w = np.asarray(w, np.uint32)
    keep = src != dst
    src, dst, w = src[keep], dst[keep], w[keep]
    order = np.lexsort((w, dst, src))
    src, dst, w = src[order], dst[order], w[order]
    if len(src):
        first = np.ones(len(src), bool)
        first[1:] = (src[1:] != src[:-1]) | (dst[1:] != dst[:-1])
        src, dst, w = src[first], dst[first], w[first]
    row_ptr = np.zeros(V + 1, np.int64)
    np.add.at(row_ptr, src + 1, 1)
    row_ptr = np.cumsum(row_ptr).astype(np.int32)
    return Graph(V, len(src), row_ptr, dst.astype(np.int32), w.astype(np.uint32), name=name)


def pick_sources(g: Graph, B: int, seed: int) -> np.ndarray:
    """B distinct vertices, uniform among those with out-degree > 0."""
    cand = np.nonzero(np.diff(g.row_ptr) > 0)[0].astype(np.int32)
    if B > len(cand):
        raise ValueError("not enough vertices with out-degree > 0")
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.choice(cand, size=B, replace=False).astype(np.int32)
