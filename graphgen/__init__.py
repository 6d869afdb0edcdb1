"""Seeded synthetic graph inputs shared by the oracle tests, the GPU tests and
the benchmark.

Only raw edge records come out of here (self-loops and duplicate pairs
included); the adjacency build, de-duplication and every traversal live on the
consumer side.  The random streams are counter based (see graphgen.c), so a
given (generator, parameters, seed) always yields the same records.

Workload recipes (the paper measures on real social, web and road graphs that
are not available here; these stand in for them):

* ``rmat(scale, 16)`` with (a, b, c, d) = (.57, .19, .19, .05) stands in for
  the power-law social/web graphs of the evaluation (dataset table).
* ``grid(4096, 4096, shortcut_frac=0.01)`` with uint32 weights in [1, 1000]
  stands in for the road network (mesh, low uniform degree, huge diameter).
* ``chung_lu(...)`` gives heavy-tailed degree sequences with a chosen exponent.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "graphgen.c")
_LIB = os.path.join(_HERE, "libgraphgen.so")
_lib = None

RMAT_ABC = (0.57, 0.19, 0.19)


def build(force: bool = True) -> str:
    """Compile libgraphgen.so next to its source (gcc, OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c11",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        i32p = ctypes.POINTER(ctypes.c_int32)
        u32p = ctypes.POINTER(ctypes.c_uint32)
        lib.gg_u64.restype = ctypes.c_uint64
        lib.gg_u64.argtypes = [ctypes.c_uint64] * 3
        lib.gg_rmat.restype = ctypes.c_int
        lib.gg_rmat.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                                ctypes.c_double, ctypes.c_uint64, ctypes.c_int, i32p, i32p]
        lib.gg_grid_count.restype = ctypes.c_int64
        lib.gg_grid_count.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int64]
        lib.gg_grid.restype = ctypes.c_int
        lib.gg_grid.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32,
                                ctypes.c_uint32, ctypes.c_uint64, i32p, i32p, ctypes.c_void_p]
        lib.gg_uniform_weights.restype = ctypes.c_int
        lib.gg_uniform_weights.argtypes = [ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint32,
                                           ctypes.c_uint64, u32p]
        lib.gg_chunglu_weights.restype = ctypes.c_double
        lib.gg_chunglu_weights.argtypes = [ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                                           ctypes.c_double, ctypes.c_void_p]
        lib.gg_chunglu.restype = ctypes.c_int
        lib.gg_chunglu.argtypes = [ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                                   ctypes.c_double, ctypes.c_uint64, i32p, i32p]
        lib.gg_uniform.restype = ctypes.c_int
        lib.gg_uniform.argtypes = [ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, i32p, i32p]
        lib.gg_pick_sources.restype = ctypes.c_int64
        lib.gg_pick_sources.argtypes = [ctypes.c_int32, ctypes.c_int64, i32p, i32p, ctypes.c_int64,
                                        ctypes.c_uint64, i32p]
        lib.gg_permutation.restype = None
        lib.gg_permutation.argtypes = [ctypes.c_int32, ctypes.c_uint64, ctypes.c_uint64, i32p]
        _lib = lib
    return _lib


def _p(a, t=ctypes.c_int32):
    return a.ctypes.data_as(ctypes.POINTER(t))


class EdgeList:
    """Raw directed edge records over vertices [0, n)."""

    def __init__(self, n, src, dst, w=None, name=""):
        self.n = int(n)
        self.src = np.ascontiguousarray(src, dtype=np.int32)
        self.dst = np.ascontiguousarray(dst, dtype=np.int32)
        self.w = None if w is None else np.ascontiguousarray(w, dtype=np.uint32)
        self.name = name

    @property
    def m(self):
        return int(self.src.shape[0])

    def __repr__(self):
        return "EdgeList(%s, n=%d, records=%d, weighted=%s)" % (self.name, self.n, self.m,
                                                               self.w is not None)


def u64(seed, stream, idx):
    return int(_load().gg_u64(seed, stream, idx))


def rmat(scale, edge_factor=16, abc=RMAT_ABC, seed=1, permute=True, nsamples=None):
    """R-MAT records: edge_factor * 2^scale samples (or ``nsamples``)."""
    n = 1 << scale
    ns = edge_factor * n if nsamples is None else int(nsamples)
    src = np.empty(ns, np.int32)
    dst = np.empty(ns, np.int32)
    rc = _load().gg_rmat(scale, ns, abc[0], abc[1], abc[2], seed, 1 if permute else 0,
                         _p(src), _p(dst))
    if rc != 0:
        raise RuntimeError("gg_rmat failed (%d)" % rc)
    return EdgeList(n, src, dst, name="rmat%d_ef%d_s%d" % (scale, edge_factor, seed))


def grid(rows, cols, shortcut_frac=0.0, seed=4, weighted=True, wlo=1, whi=1000):
    """2-D 4-neighbour grid (both directions) + floor(frac*n) random shortcut pairs."""
    n = rows * cols
    nshort = int(np.floor(shortcut_frac * n + 1e-9))
    cnt = int(_load().gg_grid_count(rows, cols, nshort))
    src = np.empty(cnt, np.int32)
    dst = np.empty(cnt, np.int32)
    w = np.empty(cnt, np.uint32) if weighted else None
    rc = _load().gg_grid(rows, cols, nshort, wlo, whi, seed, _p(src), _p(dst),
                         None if w is None else w.ctypes.data)
    if rc != 0:
        raise RuntimeError("gg_grid failed (%d)" % rc)
    return EdgeList(n, src, dst, w, name="grid%dx%d_sc%d_s%d" % (rows, cols, nshort, seed))


def uniform_weights(m, seed, lo=1, hi=1000):
    w = np.empty(int(m), np.uint32)
    rc = _load().gg_uniform_weights(int(m), lo, hi, seed, _p(w, ctypes.c_uint32))
    if rc != 0:
        raise RuntimeError("gg_uniform_weights failed")
    return w


def chunglu_weights(n, gamma, dmax, wsum):
    w = np.empty(int(n), np.float64)
    i0 = _load().gg_chunglu_weights(int(n), float(gamma), float(dmax), float(wsum), w.ctypes.data)
    return w, i0


def chung_lu(n, nsamples, gamma, dmax, seed, wsum=None):
    """Chung-Lu records with expected-degree weights summing to ``wsum``
    (default: nsamples)."""
    wsum = float(nsamples if wsum is None else wsum)
    src = np.empty(int(nsamples), np.int32)
    dst = np.empty(int(nsamples), np.int32)
    rc = _load().gg_chunglu(int(n), int(nsamples), float(gamma), float(dmax), wsum, seed,
                            _p(src), _p(dst))
    if rc != 0:
        raise RuntimeError("gg_chunglu failed (%d)" % rc)
    return EdgeList(n, src, dst, name="chunglu_n%d_g%.2f_s%d" % (n, gamma, seed))


def uniform(n, nsamples, seed):
    src = np.empty(int(nsamples), np.int32)
    dst = np.empty(int(nsamples), np.int32)
    rc = _load().gg_uniform(int(n), int(nsamples), seed, _p(src), _p(dst))
    if rc != 0:
        raise RuntimeError("gg_uniform failed")
    return EdgeList(n, src, dst, name="uniform_n%d_s%d" % (n, seed))


def permutation(n, seed, stream=1):
    p = np.empty(int(n), np.int32)
    _load().gg_permutation(int(n), seed, stream, _p(p))
    return p


def pick_sources(el: EdgeList, k, seed):
    """k distinct vertices with at least one non-self-loop out-record."""
    out = np.empty(int(k), np.int32)
    got = _load().gg_pick_sources(el.n, el.m, _p(el.src), _p(el.dst), int(k), seed, _p(out))
    if got < 0:
        raise RuntimeError("gg_pick_sources failed")
    return out[:got].copy()


# ---- small fixed families used by the pins ---------------------------------

def cycle(n):
    v = np.arange(n, dtype=np.int32)
    return EdgeList(n, v, (v + 1) % n, name="cycle%d" % n)


def path(n):
    v = np.arange(n - 1, dtype=np.int32)
    return EdgeList(n, v, v + 1, name="path%d" % n)


def star(n, center=0, out=True):
    leaves = np.array([v for v in range(n) if v != center], dtype=np.int32)
    c = np.full(leaves.shape, center, np.int32)
    return EdgeList(n, c, leaves, name="star%d" % n) if out else EdgeList(n, leaves, c,
                                                                          name="instar%d" % n)


def complete(n):
    s, d = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    s = s.ravel()
    d = d.ravel()
    keep = s != d
    return EdgeList(n, s[keep], d[keep], name="complete%d" % n)


def empty(n):
    z = np.zeros(0, np.int32)
    return EdgeList(n, z, z, name="empty%d" % n)


def from_pairs(n, pairs, w=None, name="pairs"):
    a = np.asarray(pairs, dtype=np.int64).reshape(-1, 2)
    return EdgeList(n, a[:, 0], a[:, 1], w, name=name)
