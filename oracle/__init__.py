"""ORACLE -- test infrastructure only.

ctypes wrapper over oracle.c, the plain single-threaded CPU implementation of
the graph algorithms that the GPU library runs.  Only the tests, the smoke
check and the benchmark's CPU-baseline leg import this package; the GPU
library never does, and the two share no code.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

UNREACHED = np.uint32(0xFFFFFFFF)


def build(force: bool = True) -> str:
    """Compile liboracle.so (plain C, single-threaded, -O2)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-shared", "-fPIC", "-std=c11", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        vp = ctypes.c_void_p
        i32, i64, f64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        lib.or_build_adj.restype = i64
        lib.or_build_adj.argtypes = [i32, i64, vp, vp, vp, vp, vp, vp]
        lib.or_pagerank.restype = ctypes.c_int
        lib.or_pagerank.argtypes = [i32, vp, vp, vp, i32, f64, vp]
        lib.or_prdelta.restype = ctypes.c_int
        lib.or_prdelta.argtypes = [i32, vp, vp, i32, f64, f64, vp, vp]
        lib.or_bfs.restype = i32
        lib.or_bfs.argtypes = [i32, vp, vp, i32, vp, vp]
        lib.or_cc.restype = i32
        lib.or_cc.argtypes = [i32, vp, vp, vp]
        lib.or_cc_union_find.restype = i64
        lib.or_cc_union_find.argtypes = [i32, i64, vp, vp, vp]
        lib.or_dijkstra.restype = ctypes.c_int
        lib.or_dijkstra.argtypes = [i32, vp, vp, vp, i32, vp]
        lib.or_bc.restype = i32
        lib.or_bc.argtypes = [i32, vp, vp, i32, vp, vp]
        lib.or_eigenvector.restype = ctypes.c_int
        lib.or_eigenvector.argtypes = [i32, vp, vp, i32, vp]
        lib.or_bellman_ford.restype = i32
        lib.or_bellman_ford.argtypes = [i32, vp, vp, vp, i32, vp]
        _lib = lib
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data


class Adj:
    """One adjacency direction: off[n+1], idx[m], optional w[m]."""

    def __init__(self, off, idx, w=None):
        self.off = off
        self.idx = idx
        self.w = w

    @property
    def n(self):
        return self.off.shape[0] - 1

    @property
    def m(self):
        return int(self.idx.shape[0])

    def degrees(self):
        return np.diff(self.off).astype(np.int64)


def build_adj(n, src, dst, w=None) -> Adj:
    """Drop self-loops, collapse repeated pairs (smallest weight kept), sort rows."""
    src = np.ascontiguousarray(src, np.int32)
    dst = np.ascontiguousarray(dst, np.int32)
    mr = src.shape[0]
    off = np.empty(n + 1, np.int32)
    idx = np.empty(max(mr, 1), np.int32)
    wout = None
    if w is not None:
        w = np.ascontiguousarray(w, np.uint32)
        wout = np.empty(max(mr, 1), np.uint32)
    m = _load().or_build_adj(n, mr, _ptr(src), _ptr(dst), _ptr(w), _ptr(off), _ptr(idx),
                             _ptr(wout))
    if m < 0:
        raise ValueError("or_build_adj failed (%d)" % m)
    return Adj(off, idx[:m].copy(), None if wout is None else wout[:m].copy())


class Graph:
    """CSR (out-edges) and CSC (in-edges) built by the oracle from raw records."""

    def __init__(self, el):
        self.n = el.n
        self.out = build_adj(el.n, el.src, el.dst, el.w)
        self.inc = build_adj(el.n, el.dst, el.src, el.w)
        self.m = self.out.m


def pagerank(g: Graph, iters=20, alpha=0.85):
    x = np.empty(g.n, np.float64)
    rc = _load().or_pagerank(g.n, _ptr(g.out.off), _ptr(g.inc.off), _ptr(g.inc.idx), iters,
                             alpha, _ptr(x))
    if rc:
        raise ValueError("or_pagerank failed")
    return x


def prdelta(g: Graph, iters=10, alpha=0.85, eps=0.1):
    rank = np.empty(g.n, np.float64)
    active = np.empty(max(iters, 1), np.int64)
    rc = _load().or_prdelta(g.n, _ptr(g.out.off), _ptr(g.out.idx), iters, alpha, eps, _ptr(rank),
                            _ptr(active))
    if rc:
        raise ValueError("or_prdelta failed")
    return rank, active[:iters].copy()


def bfs(g: Graph, s):
    level = np.empty(g.n, np.int32)
    parent = np.empty(g.n, np.int32)
    d = _load().or_bfs(g.n, _ptr(g.out.off), _ptr(g.out.idx), int(s), _ptr(level), _ptr(parent))
    if d < 0:
        raise ValueError("or_bfs failed")
    return level, parent


def cc(g: Graph):
    label = np.empty(g.n, np.int32)
    r = _load().or_cc(g.n, _ptr(g.out.off), _ptr(g.out.idx), _ptr(label))
    if r < 0:
        raise ValueError("or_cc failed")
    return label, int(r)


def cc_union_find(n, src, dst):
    """Weak-component labels (least vertex id) of the raw records src[i] ->
    dst[i] by union-find; returns (label, number of components)."""
    src = np.ascontiguousarray(src, np.int32)
    dst = np.ascontiguousarray(dst, np.int32)
    if src.shape != dst.shape:
        raise ValueError("src and dst differ in length")
    label = np.empty(int(n), np.int32)
    r = _load().or_cc_union_find(int(n), int(src.size), _ptr(src), _ptr(dst), _ptr(label))
    if r < 0:
        raise ValueError("or_cc_union_find failed")
    return label, int(r)


def dijkstra(g: Graph, s):
    if g.out.w is None:
        raise ValueError("graph has no weights")
    dist = np.empty(g.n, np.uint32)
    rc = _load().or_dijkstra(g.n, _ptr(g.out.off), _ptr(g.out.idx), _ptr(g.out.w), int(s),
                             _ptr(dist))
    if rc == -5:
        raise OverflowError("distance does not fit in uint32")
    if rc:
        raise ValueError("or_dijkstra failed")
    return dist


def bellman_ford(g: Graph, s):
    dist = np.empty(g.n, np.uint32)
    r = _load().or_bellman_ford(g.n, _ptr(g.out.off), _ptr(g.out.idx), _ptr(g.out.w), int(s),
                                _ptr(dist))
    if r == -5:
        raise OverflowError("distance does not fit in uint32")
    if r < 0:
        raise ValueError("or_bellman_ford failed")
    return dist, int(r)


def eigenvector(g: Graph, iters=20):
    """Eigenvector centrality by L2-normalised power iteration, fp64."""
    x = np.empty(g.n, np.float64)
    if _load().or_eigenvector(g.n, _ptr(g.inc.off), _ptr(g.inc.idx), int(iters), _ptr(x)):
        raise ValueError("or_eigenvector failed")
    return x


def bc(g: Graph, s):
    """Single-source betweenness dependencies (Brandes) and path counts."""
    delta = np.empty(g.n, np.float64)
    sigma = np.empty(g.n, np.float64)
    r = _load().or_bc(g.n, _ptr(g.out.off), _ptr(g.out.idx), int(s), _ptr(delta), _ptr(sigma))
    if r < 0:
        raise ValueError("or_bc failed")
    return delta, sigma


def check_bfs_parents(g: Graph, s, level, parent):
    """Graph500-style validation of a BFS tree against oracle levels.

    parent[s] == s; parent == -1 exactly where level == -1; for every other
    reached v, parent[v] -> v is an edge and level[parent[v]] == level[v]-1.
    Returns a list of failure strings (empty when valid).
    """
    bad = []
    level = np.asarray(level)
    parent = np.asarray(parent)
    if parent[s] != s:
        bad.append("parent[src] != src")
    unreached = level == -1
    if not np.array_equal(parent == -1, unreached):
        bad.append("parent==-1 does not match unreached set")
    v = np.nonzero(~unreached)[0]
    v = v[v != s]
    p = parent[v].astype(np.int64)
    if np.any((p < 0) | (p >= g.n)):
        bad.append("parent out of range")
        return bad
    if np.any(level[p] != level[v] - 1):
        bad.append("parent level mismatch")
    # edge p -> v must exist: binary search in the sorted CSR row of p
    off, idx = g.out.off, g.out.idx
    lo = off[p].astype(np.int64)
    hi = off[p + 1].astype(np.int64)
    ok = np.zeros(v.shape[0], bool)
    # vectorised lower_bound over each row
    l, h = lo.copy(), hi.copy()
    for _ in range(32):
        act = l < h
        if not act.any():
            break
        mid = (l + h) // 2
        mv = np.where(act, idx[np.minimum(mid, max(idx.shape[0] - 1, 0))], 0)
        go = act & (mv < v)
        l = np.where(go, mid + 1, l)
        h = np.where(act & ~go, mid, h)
    inrow = l < hi
    ok[inrow] = idx[l[inrow]] == v[inrow]
    if not ok.all():
        bad.append("%d parent edges missing" % int((~ok).sum()))
    return bad
