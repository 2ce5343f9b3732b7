"""CPU oracle for the superstep engine -- test infrastructure only.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The device library
(``paper_2203_13005_amd``) never imports it and shares no code with it; the
two meet only in the seeded inputs from ``gen``.

The arithmetic lives in ``oracle.c`` (plain C, PageRank in float64).  Its
single-threaded functions are the reference; ``threads != 1`` selects the
OpenMP timing mode, which runs the same supersteps on all host cores and is
pinned bitwise to the reference by a CPU test.  The functions here drive it
superstep by superstep and hold the independent pins that check it: a dense
linear solve for the PageRank fixed point and a hop-bounded Bellman-Ford
written as whole-array relaxation.  Each function names the passage of the
paper it follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "_oracle.so")
_lib = None

INF = 0xFFFFFFFF


def build(force: bool = False) -> str:
    """Compile oracle.c into _oracle.so with gcc (no device code involved)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        P, I64, I32, D = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double
        sig = {
            "or_out_degree": (None, [I64, I64, P, P]),
            "or_pr_superstep": (None, [I64, I64, P, P, P, D, P, P]),
            "or_ppr_superstep": (None, [I64, I64, P, P, P, D, I32, P, P]),
            "or_min_superstep": (I64, [I64, I64, P, P, P, ctypes.c_int, P, P, P, P, P]),
            "or_sssp": (I64, [I64, I64, P, P, P, I32, I64, P, P, P, P]),
            "or_cc": (I64, [I64, I64, P, P, P, I64, P, P, P, P]),
            "or_delta": (I64, [I64, P, P, P, P, P, P]),
            "or_dijkstra": (ctypes.c_int, [I64, I64, P, P, P, I32, P, P]),
            "or_cc_hops": (I64, [I64, I64, P, P, P]),
            "or_union_find_min": (ctypes.c_int, [I64, I64, P, P, P, P]),
            "or_sssp_omp": (I64, [I64, I64, P, P, P, I32, I64, P, P, P, P, ctypes.c_int]),
            "or_cc_omp": (I64, [I64, I64, P, P, P, I64, P, P, P, P, ctypes.c_int]),
            "or_in_edges": (None, [I64, I64, P, P, P, P]),
            "or_pr_superstep_omp": (None, [I64, P, P, P, D, I32, P, P, ctypes.c_int]),
            "or_sssp_many": (None, [I64, I64, P, P, P, P, I32, P, P, ctypes.c_int]),
            "or_dijkstra_many": (None, [I64, I64, P, P, P, P, I32, P, ctypes.c_int]),
            "or_ppr_many": (ctypes.c_int, [I64, I64, P, P, P, D, P, I32, I32, P, ctypes.c_int]),
            "or_max_threads": (ctypes.c_int, []),
            "or_sym_adjacency": (I64, [I64, I64, P, P, P, P]),
            "or_lp_superstep": (I64, [I64, P, P, P, P]),
            "or_lp": (I64, [I64, I64, P, P, P, I64, P, P]),
        }
        for name, (res, args) in sig.items():
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _lib = lib
    return _lib


def _p(a):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.c_void_p)


def _edges(g):
    src = np.ascontiguousarray(np.repeat(np.arange(g.V, dtype=np.int32), np.diff(g.row_ptr)))
    dst = np.ascontiguousarray(g.col, dtype=np.int32)
    w = np.ascontiguousarray(g.w, dtype=np.uint32)
    return src, dst, w


def out_degree(g) -> np.ndarray:
    src, _, _ = _edges(g)
    deg = np.empty(max(g.V, 1), np.int32)
    _load().or_out_degree(g.V, g.E, _p(src), _p(deg))
    return deg[: g.V]


# --------------------------------------------------------------------------
# PageRank / personalised PageRank (algorithms named in Section "Setup"; the
# iteration follows the template of Section "Algorithm Template").
# --------------------------------------------------------------------------

def max_threads() -> int:
    """Host threads the OpenMP timing mode uses by default."""
    return int(_load().or_max_threads())


class _PrPull:
    """Destination-major edge order for the OpenMP PageRank mode (each
    destination keeps its messages in edge-list order)."""

    def __init__(self, g):
        src, dst, _ = _edges(g)
        self.in_rp = np.empty(g.V + 1, np.int64)
        self.in_src = np.empty(max(g.E, 1), np.int32)
        _load().or_in_edges(g.V, g.E, _p(src), _p(dst), _p(self.in_rp), _p(self.in_src))


def _pr_run(g, T, d, x, seed, history, threads):
    lib = _load()
    deg = out_degree(g)
    hist = [x.copy()] if history else None
    nxt = np.empty_like(x)
    if threads == 1:
        src, dst, _ = _edges(g)
    else:
        pull = _PrPull(g)
    for _ in range(T):
        if threads != 1:
            lib.or_pr_superstep_omp(g.V, _p(pull.in_rp), _p(pull.in_src), _p(deg), d,
                                    -1 if seed is None else int(seed), _p(x), _p(nxt), int(threads))
        elif seed is None:
            lib.or_pr_superstep(g.V, g.E, _p(src), _p(dst), _p(deg), d, _p(x), _p(nxt))
        else:
            lib.or_ppr_superstep(g.V, g.E, _p(src), _p(dst), _p(deg), d, int(seed), _p(x), _p(nxt))
        x, nxt = nxt, x
        if history:
            hist.append(x.copy())
    return (x, hist) if history else x


def pagerank(g, T: int, d: float = 0.85, x0: np.ndarray | None = None,
             history: bool = False, threads: int = 1):
    """x after T supersteps from x0 (default 1/V), float64.  With history=True
    also returns the list of states x_0 .. x_T.  threads != 1: OpenMP timing
    mode (0 = all host threads), bitwise the same result."""
    x = np.full(g.V, 1.0 / g.V) if x0 is None else np.array(x0, np.float64)
    return _pr_run(g, T, d, x, None, history, threads)


def ppr(g, seed: int, T: int, d: float = 0.85, history: bool = False, threads: int = 1):
    """Personalised PageRank from seed after T supersteps, x0 = e_seed."""
    x = np.zeros(g.V)
    x[seed] = 1.0
    return _pr_run(g, T, d, x, seed, history, threads)


# --------------------------------------------------------------------------
# Min-combine algorithms (Bellman-Ford SSSP and label propagation, Section
# "Setup"), run to convergence under the iteration control of Section
# "Iteration Control".
# --------------------------------------------------------------------------

@dataclass
class MinRun:
    state: np.ndarray          # uint32 [V]
    K: int                     # supersteps including the last one with no change (-1: cap hit)
    front: np.ndarray          # |F_k| per superstep
    msgs: np.ndarray           # messages generated per superstep
    changed: np.ndarray        # |F_{k+1}| per superstep


def sssp(g, source: int, max_steps: int = 1 << 30, threads: int = 1) -> MinRun:
    """Bellman-Ford to convergence.  threads != 1: OpenMP timing mode (0 =
    all host threads), bitwise the same result."""
    lib = _load()
    src, dst, w = _edges(g)
    cap = min(max_steps, g.V + 2)
    dist = np.empty(max(g.V, 1), np.uint32)
    fs, ef, ch = (np.zeros(cap, np.int64) for _ in range(3))
    if threads == 1:
        K = lib.or_sssp(g.V, g.E, _p(src), _p(dst), _p(w), int(source), cap, _p(dist), _p(fs), _p(ef), _p(ch))
    else:
        K = lib.or_sssp_omp(g.V, g.E, _p(src), _p(dst), _p(w), int(source), cap, _p(dist), _p(fs), _p(ef),
                            _p(ch), int(threads))
    if K == -2:
        raise MemoryError("oracle sssp")
    n = K if K > 0 else cap
    return MinRun(dist[: g.V], int(K), fs[:n], ef[:n], ch[:n])


def cc(g, max_steps: int = 1 << 30, threads: int = 1) -> MinRun:
    lib = _load()
    src, dst, _ = _edges(g)
    l2g = None if g.l2g is None else np.ascontiguousarray(g.l2g, np.int32)
    cap = min(max_steps, g.V + 2)
    lab = np.empty(max(g.V, 1), np.uint32)
    fs, ef, ch = (np.zeros(cap, np.int64) for _ in range(3))
    if threads == 1:
        K = lib.or_cc(g.V, g.E, _p(src), _p(dst), _p(l2g), cap, _p(lab), _p(fs), _p(ef), _p(ch))
    else:
        K = lib.or_cc_omp(g.V, g.E, _p(src), _p(dst), _p(l2g), cap, _p(lab), _p(fs), _p(ef), _p(ch),
                          int(threads))
    if K == -2:
        raise MemoryError("oracle cc")
    n = K if K > 0 else cap
    return MinRun(lab[: g.V], int(K), fs[:n], ef[:n], ch[:n])


class LpRun:
    def __init__(self, state, K, changed):
        self.state, self.K, self.changed = state, K, changed


def lp(g, max_steps: int = 15) -> LpRun:
    """Label propagation (most frequent neighbour label, smallest on a tie),
    at most max_steps iterations.  K = iterations run when the last one
    changed nothing, -1 when the cap was reached with labels still moving."""
    lib = _load()
    src, dst, _ = _edges(g)
    l2g = None if g.l2g is None else np.ascontiguousarray(g.l2g, np.int32)
    lab = np.empty(max(g.V, 1), np.uint32)
    ch = np.zeros(max(max_steps, 1), np.int64)
    K = lib.or_lp(g.V, g.E, _p(src), _p(dst), _p(l2g), int(max_steps), _p(lab), _p(ch))
    if K == -2:
        raise MemoryError("oracle lp")
    n = K if K > 0 else max_steps
    return LpRun(lab[: g.V], int(K), ch[:n])


def lp_steps(g, max_steps: int = 15):
    """Labels after every LP iteration: list label_0 .. label_n (n = the
    iterations run, stopping after the first that changes nothing)."""
    lib = _load()
    src, dst, _ = _edges(g)
    rp = np.empty(g.V + 1, np.int64)
    nb = np.empty(max(2 * g.E, 1), np.int32)
    if lib.or_sym_adjacency(g.V, g.E, _p(src), _p(dst), _p(rp), _p(nb)) < 0:
        raise MemoryError("oracle lp")
    lab = (np.arange(g.V) if g.l2g is None else np.asarray(g.l2g)).astype(np.uint32)
    out = [lab.copy()]
    for _ in range(max_steps):
        nxt = np.empty(max(g.V, 1), np.uint32)
        c = lib.or_lp_superstep(g.V, _p(rp), _p(nb), _p(lab), _p(nxt))
        if c < 0:
            raise MemoryError("oracle lp")
        lab = nxt[: g.V].copy()
        out.append(lab.copy())
        if c == 0:
            break
    return out


class SymAdjacency:
    """Deduplicated symmetric neighbour lists of a graph (the oracle's own)."""

    def __init__(self, g):
        lib = _load()
        src, dst, _ = _edges(g)
        self.rp = np.empty(g.V + 1, np.int64)
        self.nb = np.empty(max(2 * g.E, 1), np.int32)
        if lib.or_sym_adjacency(g.V, g.E, _p(src), _p(dst), _p(self.rp), _p(self.nb)) < 0:
            raise MemoryError("oracle lp")
        self.V = g.V

    def lp_step(self, labels: np.ndarray) -> np.ndarray:
        """One LP iteration from the given labels."""
        lab = np.ascontiguousarray(labels, np.uint32)
        nxt = np.empty(max(self.V, 1), np.uint32)
        if _load().or_lp_superstep(self.V, _p(self.rp), _p(self.nb), _p(lab), _p(nxt)) < 0:
            raise MemoryError("oracle lp")
        return nxt[: self.V]


def sssp_many(g, sources, threads: int = 0):
    """Independent single-source runs of the reference Bellman-Ford, one per
    host thread (the several sources of Section "Setup", first footnote):
    returns (dist [B, V] uint32, K [B])."""
    lib = _load()
    src, dst, w = _edges(g)
    s = np.ascontiguousarray(sources, np.int32)
    dist = np.empty((len(s), max(g.V, 1)), np.uint32)
    K = np.empty(len(s), np.int64)
    lib.or_sssp_many(g.V, g.E, _p(src), _p(dst), _p(w), _p(s), len(s), _p(dist), _p(K), int(threads))
    return dist[:, : g.V], K


def ppr_many(g, seeds, T: int, d: float = 0.85, threads: int = 0) -> np.ndarray:
    """Personalised PageRank of every seed (reference supersteps, one lane per
    host thread): [B, V] float64, lane b bitwise ppr(g, seeds[b], T, d)."""
    lib = _load()
    src, dst, _ = _edges(g)
    deg = out_degree(g)
    s = np.ascontiguousarray(seeds, np.int32)
    x = np.empty((len(s), max(g.V, 1)), np.float64)
    if lib.or_ppr_many(g.V, g.E, _p(src), _p(dst), _p(deg), d, _p(s), len(s), int(T), _p(x), int(threads)):
        raise MemoryError("oracle ppr_many")
    return x[:, : g.V]


def dijkstra_many(g, sources, threads: int = 0) -> np.ndarray:
    """Dijkstra from every source, one run per host thread: [B, V] uint32."""
    lib = _load()
    src, dst, w = _edges(g)
    s = np.ascontiguousarray(sources, np.int32)
    dist = np.empty((len(s), max(g.V, 1)), np.uint32)
    lib.or_dijkstra_many(g.V, g.E, _p(src), _p(dst), _p(w), _p(s), len(s), _p(dist), int(threads))
    return dist[:, : g.V]


def min_superstep(g, state: np.ndarray, front: np.ndarray, weighted: bool, both_dirs: bool):
    """One Jacobi min superstep; returns (state', front')."""
    lib = _load()
    src, dst, w = _edges(g)
    st = np.ascontiguousarray(state, np.uint32)
    fr = np.ascontiguousarray(front, np.uint8)
    nst = np.empty(max(g.V, 1), np.uint32)
    nfr = np.empty(max(g.V, 1), np.uint8)
    lib.or_min_superstep(g.V, g.E, _p(src), _p(dst), _p(w) if weighted else None, int(both_dirs),
                         _p(st), _p(fr), _p(nst), _p(nfr), None)
    return nst[: g.V], nfr[: g.V].astype(bool)


def sssp_frontiers(g, source: int, max_steps: int = 1 << 30):
    """States and frontiers of every superstep: lists dist_k, F_k (k = 0..K)."""
    dist = np.full(g.V, INF, np.uint32)
    front = np.zeros(g.V, bool)
    dist[source] = 0
    front[source] = True
    dists, fronts = [dist.copy()], [front.copy()]
    for _ in range(max_steps):
        dist, front = min_superstep(g, dist, front, True, False)
        dists.append(dist.copy())
        fronts.append(front.copy())
        if not front.any():
            break
    return dists, fronts


# --------------------------------------------------------------------------
# Sync set (Sections "Synchronization Caching" and "Synchronization
# Skipping").
# --------------------------------------------------------------------------

REMOTE_OUT = 2
REMOTE_ANY = 4


def remote_mask(g, algo: str, mode: str = "remote") -> np.ndarray:
    """Which vertices another node needs: out-edges elsewhere for PageRank and
    SSSP (their values flow along out-edges), any edge elsewhere for CC."""
    if mode == "all" or g.flags is None:
        return np.ones(g.V, np.uint8) if (mode == "all") else np.zeros(g.V, np.uint8)
    bit = REMOTE_ANY if algo == "cc" else REMOTE_OUT
    return ((g.flags & bit) != 0).astype(np.uint8)


def delta(g, remote: np.ndarray, now: np.ndarray, synced: np.ndarray):
    """Lazy upload: (gid, value bits) of remote vertices whose value differs
    from the last uploaded copy, ascending gid.  `synced` is updated in place.
    Returns (gids, vals, skippable)."""
    lib = _load()
    now_b = np.ascontiguousarray(now).view(np.uint32)
    assert synced.dtype == np.uint32 and synced.flags.c_contiguous
    rem = np.ascontiguousarray(remote, np.uint8)
    l2g = None if g.l2g is None else np.ascontiguousarray(g.l2g, np.int32)
    gid = np.empty(max(g.V, 1), np.int32)
    val = np.empty(max(g.V, 1), np.uint32)
    n = lib.or_delta(g.V, _p(rem), _p(l2g), _p(now_b), _p(synced), _p(gid), _p(val))
    return gid[:n].copy(), val[:n].copy(), n == 0


# --------------------------------------------------------------------------
# Independent pins.
# --------------------------------------------------------------------------

def dijkstra(g, source: int, with_hops: bool = False):
    lib = _load()
    src, dst, w = _edges(g)
    dist = np.empty(max(g.V, 1), np.uint32)
    hops = np.empty(max(g.V, 1), np.int32) if with_hops else None
    rc = lib.or_dijkstra(g.V, g.E, _p(src), _p(dst), _p(w), int(source), _p(dist), _p(hops))
    if rc != 0:
        raise RuntimeError("or_dijkstra rc=%d" % rc)
    return (dist[: g.V], hops[: g.V]) if with_hops else dist[: g.V]


def union_find_labels(g) -> np.ndarray:
    lib = _load()
    src, dst, _ = _edges(g)
    l2g = None if g.l2g is None else np.ascontiguousarray(g.l2g, np.int32)
    lab = np.empty(max(g.V, 1), np.uint32)
    if lib.or_union_find_min(g.V, g.E, _p(src), _p(dst), _p(l2g), _p(lab)) != 0:
        raise MemoryError("union find")
    return lab[: g.V]


def cc_max_hops(g) -> int:
    lib = _load()
    src, dst, _ = _edges(g)
    hop = np.empty(max(g.V, 1), np.int32)
    return int(lib.or_cc_hops(g.V, g.E, _p(src), _p(dst), _p(hop)))


def pagerank_fixed_point_dense(g, d: float = 0.85) -> np.ndarray:
    """Solves (I - d M) x = (1-d)/V * 1 with a dense LU (numpy), where
    M[v, u] = 1/outdeg(u) for an edge u->v and 1/V for every v when u has no
    out-edge.  Only for small V."""
    V = g.V
    deg = np.diff(g.row_ptr).astype(np.float64)
    M = np.zeros((V, V))
    src = np.repeat(np.arange(V), np.diff(g.row_ptr))
    M[g.col, src] += 1.0 / deg[src]
    M[:, deg == 0] = 1.0 / V
    return np.linalg.solve(np.eye(V) - d * M, np.full(V, (1.0 - d) / V))


def ppr_fixed_point_dense(g, seed: int, d: float = 0.85) -> np.ndarray:
    """Solves (I - d M_s) x = (1-d) e_s, with dangling columns sending their
    mass to the seed."""
    V = g.V
    deg = np.diff(g.row_ptr).astype(np.float64)
    M = np.zeros((V, V))
    src = np.repeat(np.arange(V), np.diff(g.row_ptr))
    M[g.col, src] += 1.0 / deg[src]
    M[seed, deg == 0] = 1.0
    b = np.zeros(V)
    b[seed] = 1.0 - d
    return np.linalg.solve(np.eye(V) - d * M, b)


def hop_bounded_distances(g, source: int, k: int) -> np.ndarray:
    """Brute force: the shortest distance over paths of at most k edges, by k
    rounds of relaxing EVERY edge from the previous round's values (no
    frontier)."""
    src = np.repeat(np.arange(g.V), np.diff(g.row_ptr))
    d = np.full(g.V, np.iinfo(np.int64).max // 4, np.int64)
    d[source] = 0
    for _ in range(k):
        cand = d[src] + g.w.astype(np.int64)
        nd = d.copy()
        np.minimum.at(nd, g.col, cand)
        d = nd
    out = np.where(d >= np.iinfo(np.int64).max // 4, INF, d)
    return np.minimum(out, INF).astype(np.uint32)


# --------------------------------------------------------------------------
# Pipeline block size (Section "Block Size Selection", Eq.
# "PipelineTimeSimplied2", Lemma "bSizeSelection"): the oracle minimises the
# equation by brute force over the block count.
# --------------------------------------------------------------------------

def pipeline_time(k1: float, k2: float, k3: float, a: float, d: float, s) -> np.ndarray:
    """Eq. "PipelineTimeSimplied2": d entities in s equal blocks of b = d / s;
    download k1 b, computation a + k2 b, upload k3 b per block; the first
    block's download and the last block's upload are not overlapped."""
    s = np.asarray(s, np.float64)
    b = d / s
    tn, tc, tu = k1 * b, a + k2 * b, k3 * b
    return tn + np.maximum(tn, tc) + (s - 2) * np.maximum(np.maximum(tn, tc), tu) + np.maximum(tc, tu) + tu


def pipeline_brute_force(k1: float, k2: float, k3: float, a: float, d: int):
    """(s, T): the block count in [2, d] with the smallest modelled time (the
    smallest such s on a tie)."""
    s = np.arange(2, int(d) + 1, dtype=np.float64)
    t = pipeline_time(k1, k2, k3, a, float(d), s)
    i = int(np.argmin(t))
    return int(s[i]), float(t[i])


# --------------------------------------------------------------------------
# Workload balancing (Section "Beyond-Iteration Optimization: Workload
# Balancing", objective min max_j c_j d_j, Lemma "minmaxcidi"): the oracle
# minimises the objective over integer splits by exhaustive search.
# --------------------------------------------------------------------------

def balance_brute_force(c, D: int):
    """(split, value): the integer split d_1 + ... + d_m = D (d_j >= 0) with the
    smallest max_j c_j d_j, searched exhaustively (m <= 3, small D)."""
    c = [float(x) for x in c]
    m = len(c)
    best, arg = float("inf"), None

    def rec(j, left, cur, acc):
        nonlocal best, arg
        if j == m - 1:
            v = max(acc, c[j] * left)
            if v < best:
                best, arg = v, cur + [left]
            return
        for dj in range(left + 1):
            rec(j + 1, left - dj, cur + [dj], max(acc, c[j] * dj))

    rec(0, int(D), [], 0.0)
    return arg, best
