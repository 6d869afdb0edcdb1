"""Python binding of libgraphit_mi.so (the C ABI in include/graphit_mi.h).

Argument marshalling only: every step of the traversals runs in the HIP
kernels of the library.  Device buffers are torch CUDA tensors (or raw
device addresses as ints); streams are torch streams (default: the current
stream).  The library must be built (``python -m paper_1805_00923_amd.build``
or ``__graft_entry__.build()``); importing this package without it raises.
"""
from __future__ import annotations

import atexit
import ctypes
import os
import sys
import weakref

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "libgraphit_mi.so")

GI_OK = 0
GI_ERR_INVALID_ARG = -1
GI_ERR_OUT_OF_MEMORY = -2
GI_ERR_DEVICE = -3
GI_ERR_UNSUPPORTED = -4
GI_ERR_OVERFLOW = -5

SPARSE_PUSH = 0
DENSE_PUSH = 1
DENSE_PULL = 2
DENSE_PULL_SPARSE_PUSH = 3
DENSE_PUSH_SPARSE_PUSH = 4
LEARNED = 5
DIRECTIONS = {
    "SparsePush": SPARSE_PUSH,
    "DensePush": DENSE_PUSH,
    "DensePull": DENSE_PULL,
    "DensePull-SparsePush": DENSE_PULL_SPARSE_PUSH,
    "DensePush-SparsePush": DENSE_PUSH_SPARSE_PUSH,
    "Learned": LEARNED,
}
ALG_PAGERANK = 0
ALG_BFS = 1
ALG_CC = 2
ALG_SSSP = 3
SEL_FEATURES = 12
SEL_SCHEDULES = 4
SEL_PARAMS = 5252
BITVECTOR = 0
BOOLMAP = 1
FIXED_VERTEX_COUNT = 0
EDGE_AWARE_VERTEX_COUNT = 1
CC_ADJ_AUTO = 0
CC_ADJ_SYMMETRIC = 1
CC_ADJ_DIRECT = 2
ORDER_GIVEN = 0
BARRIER_AGENT = 0
BARRIER_XCD = 1
ORDER_OUT_DEGREE = 1
MAX_TRACE = 4096
NOALLOC_MAX_WORDS = 1 << 21


class GiError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("gi status %d: %s" % (status, msg))
        self.status = status


class Schedule(ctypes.Structure):
    _fields_ = [("direction", ctypes.c_int32), ("dense_frontier", ctypes.c_int32),
                ("num_segments", ctypes.c_int32), ("segment_strategy", ctypes.c_int32),
                ("hybrid_divisor", ctypes.c_int32), ("steps_per_sync", ctypes.c_int32),
                ("pull_block_edges", ctypes.c_int32), ("block_threads", ctypes.c_int32),
                ("sssp_delta", ctypes.c_uint32), ("segments_concurrent", ctypes.c_int32),
                ("cc_adjacency", ctypes.c_int32), ("vertex_order", ctypes.c_int32),
                ("pull_hot_sources", ctypes.c_int32), ("pull_items_per_thread", ctypes.c_int32),
                ("reserved", ctypes.c_int32 * 2)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


class RunStats(ctypes.Structure):
    _fields_ = [("algorithm", ctypes.c_int32), ("steps", ctypes.c_int32),
                ("dense_steps", ctypes.c_int32), ("trace_len", ctypes.c_int32),
                ("edges_examined", ctypes.c_int64),
                ("kernel_ms", ctypes.c_float), ("launches", ctypes.c_int32),
                ("step_direction", ctypes.c_int8 * MAX_TRACE),
                ("step_frontier", ctypes.c_int32 * MAX_TRACE),
                ("step_degree_sum", ctypes.c_int64 * MAX_TRACE),
                ("step_edges", ctypes.c_int64 * MAX_TRACE),
                ("step_segmented", ctypes.c_int8 * MAX_TRACE)]

    def trace(self):
        k = self.trace_len
        return (np.frombuffer(self.step_direction, np.int8)[:k].copy(),
                np.frombuffer(self.step_frontier, np.int32)[:k].copy(),
                np.frombuffer(self.step_degree_sum, np.int64)[:k].copy())

    def step_edges_examined(self):
        return np.frombuffer(self.step_edges, np.int64)[:self.trace_len].copy()

    def step_schedules(self):
        """Selector schedule index per step: the direction (S0..S2), or S3
        for a pull over the source segments."""
        k = self.trace_len
        d = np.frombuffer(self.step_direction, np.int8)[:k].astype(np.int64)
        seg = np.frombuffer(self.step_segmented, np.int8)[:k]
        return np.where(seg != 0, 3, d)


# every symbol the header declares, with its ctypes signature
_vp, _i32, _i64, _u32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32
# gi_alloc_fn / gi_free_fn
_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int32, ctypes.c_void_p)
_FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p)
_SIGS = {
    "gi_last_error": (ctypes.c_char_p, []),
    "gi_abi_version": (_i32, []),
    "gi_build_adjacency": (ctypes.c_int, [_i32, _i64, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "gi_graph_create": (ctypes.c_int, [_i32, _i64, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "gi_graph_create_ex": (ctypes.c_int, [_i32, _i64, _vp, _vp, _vp, _vp, _vp, _vp, _i32, _vp,
                                          ctypes.c_size_t, _vp, _vp]),
    "gi_graph_workspace_size": (ctypes.c_int, [_i32, _i64, _i32, _vp]),
    "gi_set_allocator": (ctypes.c_int, [_ALLOC_FN, _FREE_FN, _vp]),
    "gi_live_allocations": (ctypes.c_int, [_vp, _vp]),
    "gi_sync_status": (ctypes.c_int, [_vp]),
    "gi_graph_destroy": (ctypes.c_int, [_vp]),
    "gi_graph_info": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp]),
    "gi_graph_copy_in_adjacency": (ctypes.c_int, [_vp, _vp, _vp, _vp]),
    "gi_schedule_init": (ctypes.c_int, [_vp]),
    "gi_set_schedule": (ctypes.c_int, [_vp, _vp]),
    "gi_get_schedule": (ctypes.c_int, [_vp, _vp]),
    "gi_hybrid_choose_dense": (_i32, [_i64, _i64, _i64, _i32]),
    "gi_pagerank": (ctypes.c_int, [_vp, _i32, ctypes.c_float, _vp, _vp]),
    "gi_bfs": (ctypes.c_int, [_vp, _i32, _vp, _vp, _vp]),
    "gi_cc": (ctypes.c_int, [_vp, _vp, _vp]),
    "gi_sssp": (ctypes.c_int, [_vp, _i32, _vp, _vp]),
    "gi_get_run_stats": (ctypes.c_int, [_vp, _vp]),
    "gi_set_step_timing": (ctypes.c_int, [_vp, _i32]),
    "gi_prdelta": (ctypes.c_int, [_vp, _i32, ctypes.c_double, ctypes.c_double, _vp, _vp]),
    "gi_bc": (ctypes.c_int, [_vp, _i32, _vp, _vp, _vp]),
    "gi_pagerank_eigenvector": (ctypes.c_int, [_vp, _i32, ctypes.c_float, _vp, _vp, _i32, _vp]),
    "gi_selector_create": (ctypes.c_int, [ctypes.c_uint64, _vp]),
    "gi_selector_destroy": (ctypes.c_int, [_vp]),
    "gi_selector_get_params": (ctypes.c_int, [_vp, _vp, _vp, _vp]),
    "gi_selector_set_params": (ctypes.c_int, [_vp, _vp, _vp, _vp]),
    "gi_selector_get_range": (ctypes.c_int, [_vp, _vp, _vp]),
    "gi_selector_set_range": (ctypes.c_int, [_vp, _vp, _vp]),
    "gi_selector_train": (ctypes.c_int, [_vp, _vp, _vp, _vp, _i64, _i32, ctypes.c_float,
                                         ctypes.c_uint64, _i32, _vp]),
    "gi_selector_gradient": (ctypes.c_int, [_vp, _vp, _vp, _vp, _i32, _vp, _vp]),
    "gi_selector_predict": (ctypes.c_int, [_vp, _vp, _i64, _i32, _vp]),
    "gi_selector_attach": (ctypes.c_int, [_vp, _vp]),
    "gi_get_step_features": (ctypes.c_int, [_vp, _vp, _i32, _vp]),
    "gi_trace_exhaustive": (ctypes.c_int, [_vp, _i32, _i32, _vp, _vp, _vp, _i32, _vp]),
    "gi_batch_create": (ctypes.c_int, [_vp, _i32, _vp, _i32, _vp]),
    "gi_batch_autotune": (ctypes.c_int, [_vp, _i32]),
    "gi_batch_run": (ctypes.c_int, [_vp, _i32, _vp]),
    "gi_batch_launch": (ctypes.c_int, [_vp, _i32, _vp]),
    "gi_batch_wait": (ctypes.c_int, [_vp]),
    "gi_batch_info": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _vp]),
    "gi_batch_task_counters": (ctypes.c_int, [_vp, _vp, _vp]),
    "gi_batch_pr_block_edges": (ctypes.c_int, [_vp, _vp]),
    "gi_batch_destroy": (ctypes.c_int, [_vp]),
    "gi_batch_set_threads": (ctypes.c_int, [_vp, _i32]),
    "gi_batch_get_threads": (ctypes.c_int, [_vp, _vp]),
    "gi_batch_set_trace": (ctypes.c_int, [_vp, _i32]),
    "gi_batch_set_placement": (ctypes.c_int, [_vp, _i32]),
    "gi_batch_get_placement": (ctypes.c_int, [_vp, _vp]),
    "gi_batch_set_barrier_scope": (ctypes.c_int, [_vp, _i32]),
    "gi_batch_get_barrier_scope": (ctypes.c_int, [_vp, _vp]),
    "gi_batch_get_trace": (ctypes.c_int, [_vp, _i32, _vp, _vp, _vp, _i32, _vp]),
    "gi_get_step_times": (ctypes.c_int, [_vp, _vp, _vp, _i32, _vp]),
    "gi_frontier_sparse_to_bitvec": (ctypes.c_int, [_i32, _vp, _i32, _vp, _vp]),
    "gi_frontier_bitvec_to_sparse": (ctypes.c_int, [_i32, _vp, _vp, _vp, _vp]),
    "gi_frontier_bitvec_to_sparse_noalloc": (ctypes.c_int, [_i32, _vp, _vp, _vp, _vp]),
    "gi_frontier_bitvec_to_boolmap": (ctypes.c_int, [_i32, _vp, _vp, _vp]),
    "gi_frontier_boolmap_to_bitvec": (ctypes.c_int, [_i32, _vp, _vp, _vp]),
    "gi_frontier_degree_sum": (ctypes.c_int, [_vp, _vp, _i32, _vp, _vp]),
}


def _load():
    # torch ships its own HIP runtime with the same SONAME as /opt/rocm's; load
    # torch first so that the library binds to the runtime torch uses and the
    # process holds exactly one HIP runtime.
    import torch  # noqa: F401
    if not os.path.exists(LIB_PATH):
        raise ImportError("libgraphit_mi.so is not built (%s); run "
                          "`python -m paper_1805_00923_amd.build`" % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


lib = _load()


def last_error():
    return lib.gi_last_error().decode()


def _check(st):
    if st != GI_OK:
        raise GiError(st, last_error())


# ---- device memory: torch's caching allocator serves the library ---------

def _torch_alloc(nbytes, device, ctx):
    import torch
    try:
        return torch.cuda.caching_allocator_alloc(int(nbytes), int(device))
    except Exception:
        return None  # the library reports GI_ERR_OUT_OF_MEMORY


def _torch_free(ptr, device, ctx):
    if sys.is_finalizing():
        return  # the process is ending; torch may already be gone
    import torch
    try:
        torch.cuda.caching_allocator_delete(ptr)
    except Exception:
        pass


_TORCH_ALLOC = _ALLOC_FN(_torch_alloc)
_TORCH_FREE = _FREE_FN(_torch_free)


def use_torch_allocator(on=True):
    """Take the library's device memory from torch's caching allocator (the
    default for this binding), or from hipMalloc (on=False)."""
    if on:
        _check(lib.gi_set_allocator(_TORCH_ALLOC, _TORCH_FREE, None))
    else:
        _check(lib.gi_set_allocator(_ALLOC_FN(), _FREE_FN(), None))


def live_allocations():
    """(live device allocations of the library, how many came from the
    registered allocator)."""
    c, r = ctypes.c_int64(), ctypes.c_int64()
    _check(lib.gi_live_allocations(ctypes.byref(c), ctypes.byref(r)))
    return c.value, r.value


use_torch_allocator(True)

# objects holding device memory, released before torch shuts down at exit
_LIVE = weakref.WeakSet()


@atexit.register
def _release_at_exit():
    for obj in list(_LIVE):
        try:
            obj.close()
        except Exception:
            pass


def _dptr(x):
    """Device address of a torch CUDA tensor (or an int address)."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    if not x.is_cuda:
        raise ValueError("expected a device (CUDA/HIP) tensor")
    if not x.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return x.data_ptr()


def _stream(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _hptr(a):
    return None if a is None else a.ctypes.data


def hybrid_choose_dense(frontier_size, degree_sum, edges, divisor=20):
    return bool(lib.gi_hybrid_choose_dense(frontier_size, degree_sum, edges, divisor))


def build_adjacency(n, src, dst, w=None):
    """Host adjacency build (self-loops dropped, repeats merged keeping the
    smallest weight, rows sorted).  Returns (off, idx, w_or_None)."""
    src = np.ascontiguousarray(src, np.int32)
    dst = np.ascontiguousarray(dst, np.int32)
    nrec = src.shape[0]
    off = np.empty(n + 1, np.int32)
    idx = np.empty(max(nrec, 1), np.int32)
    wout = None
    if w is not None:
        w = np.ascontiguousarray(w, np.uint32)
        wout = np.empty(max(nrec, 1), np.uint32)
    m = ctypes.c_int64(0)
    _check(lib.gi_build_adjacency(n, nrec, _hptr(src), _hptr(dst), _hptr(w), _hptr(off),
                                  _hptr(idx), _hptr(wout), ctypes.byref(m)))
    m = m.value
    return off, idx[:m].copy(), (None if wout is None else wout[:m].copy())


def default_schedule(**kw):
    s = Schedule()
    _check(lib.gi_schedule_init(ctypes.byref(s)))
    for k, v in kw.items():
        if k == "direction" and isinstance(v, str):
            v = DIRECTIONS[v]
        if k == "dense_frontier" and isinstance(v, str):
            v = {"bitvector": BITVECTOR, "boolmap": BOOLMAP, "bool-array": BOOLMAP}[v]
        setattr(s, k, v)
    return s


PTR_HOST = 0
PTR_DEVICE = 1


def workspace_size(n, m, weighted=False):
    """Bytes gi_graph_create_ex takes from a caller's workspace."""
    b = ctypes.c_size_t()
    _check(lib.gi_graph_workspace_size(int(n), int(m), int(bool(weighted)), ctypes.byref(b)))
    return b.value


class Graph:
    """A graph on the device (CSR + CSC, optional uint32 weights).

    workspace: an optional torch CUDA tensor of at least workspace_size(n, m,
    weighted) bytes holding the graph's core arrays (kept alive with the
    graph); stream: the stream of the adjacency copies."""

    def __init__(self, n, out_off, out_idx, out_w=None, in_off=None, in_idx=None, in_w=None,
                 workspace=None, stream=None):
        self._h = ctypes.c_void_p(None)
        out_off = np.ascontiguousarray(out_off, np.int32)
        out_idx = np.ascontiguousarray(out_idx, np.int32)
        out_w = None if out_w is None else np.ascontiguousarray(out_w, np.uint32)
        in_off = None if in_off is None else np.ascontiguousarray(in_off, np.int32)
        in_idx = None if in_idx is None else np.ascontiguousarray(in_idx, np.int32)
        in_w = None if in_w is None else np.ascontiguousarray(in_w, np.uint32)
        m = int(out_idx.shape[0])
        self._create(int(n), m, PTR_HOST, _hptr(out_off), _hptr(out_idx), _hptr(out_w),
                     _hptr(in_off), _hptr(in_idx), _hptr(in_w), workspace, stream)
        self.weighted = out_w is not None
        self.out_off = out_off  # host copy of the row offsets (out-degrees)

    def _create(self, n, m, kind, oo, oi, ow, io, ii, iw, workspace, stream):
        ws, wsb = None, 0
        if workspace is not None:
            ws, wsb = _dptr(workspace), workspace.numel() * workspace.element_size()
        # host arrays: copies on the NULL stream unless one is given; device
        # arrays: read in the order of torch's current stream by default
        st = _stream(stream) if (stream is not None or kind == PTR_DEVICE) else None
        _check(lib.gi_graph_create_ex(n, m, oo, oi, ow, io, ii, iw, kind, ws, wsb, st,
                                      ctypes.byref(self._h)))
        self._workspace = workspace  # kept alive with the graph
        self.n = n
        self.m = m
        _LIVE.add(self)

    @classmethod
    def from_tensors(cls, n, out_off, out_idx, out_w=None, in_off=None, in_idx=None, in_w=None,
                     workspace=None, stream=None):
        """A graph from adjacency arrays in device memory (torch CUDA tensors,
        int32 offsets and ids, int32 or uint32 weights)."""
        import torch
        ok = {torch.int32} | ({torch.uint32} if hasattr(torch, "uint32") else set())
        for t in (out_off, out_idx, out_w, in_off, in_idx, in_w):
            if t is not None and (not t.is_cuda or not t.is_contiguous() or t.dtype not in ok):
                raise ValueError("adjacency tensors must be contiguous 32-bit CUDA tensors")
        g = cls.__new__(cls)
        g._h = ctypes.c_void_p(None)
        m = int(out_idx.numel())
        g._create(int(n), m, PTR_DEVICE, _dptr(out_off), _dptr(out_idx), _dptr(out_w),
                  _dptr(in_off), _dptr(in_idx), _dptr(in_w), workspace, stream)
        g.weighted = out_w is not None
        g.out_off = out_off.cpu().numpy()
        return g

    def sync(self):
        """gi_sync_status: wait for the last enqueued run, raise on a device
        error."""
        _check(lib.gi_sync_status(self._h))

    @classmethod
    def from_edges(cls, n, src, dst, w=None, build_in=True):
        off, idx, ww = build_adjacency(n, src, dst, w)
        if build_in:
            ioff, iidx, iw = build_adjacency(n, dst, src, w)
            return cls(n, off, idx, ww, ioff, iidx, iw)
        return cls(n, off, idx, ww)

    def close(self):
        if self._h:
            lib.gi_graph_destroy(self._h)
            self._h = ctypes.c_void_p(None)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self):
        n, m, mo, mi = ctypes.c_int32(), ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int32()
        _check(lib.gi_graph_info(self._h, ctypes.byref(n), ctypes.byref(m), ctypes.byref(mo),
                                 ctypes.byref(mi)))
        return {"n": n.value, "m": m.value, "max_out_degree": mo.value, "max_in_degree": mi.value}

    def in_adjacency(self):
        off = np.empty(self.n + 1, np.int32)
        idx = np.empty(max(self.m, 1), np.int32)
        w = np.empty(max(self.m, 1), np.uint32) if self.weighted else None
        _check(lib.gi_graph_copy_in_adjacency(self._h, _hptr(off), _hptr(idx), _hptr(w)))
        return off, idx[:self.m], (None if w is None else w[:self.m])

    def set_schedule(self, sched=None, **kw):
        s = sched if sched is not None else default_schedule(**kw)
        _check(lib.gi_set_schedule(self._h, ctypes.byref(s)))
        return s

    def schedule(self):
        s = Schedule()
        _check(lib.gi_get_schedule(self._h, ctypes.byref(s)))
        return s

    def stats(self):
        r = RunStats()
        _check(lib.gi_get_run_stats(self._h, ctypes.byref(r)))
        return r

    def attach_selector(self, sel):
        """Attach a copy of a Selector's weights (None detaches)."""
        _check(lib.gi_selector_attach(self._h, None if sel is None else sel._h))

    def step_features(self):
        """float32 [steps, 12]: selector features of the last BFS/CC call."""
        cnt = ctypes.c_int32()
        _check(lib.gi_get_step_features(self._h, None, 0, ctypes.byref(cnt)))
        out = np.zeros((max(cnt.value, 1), SEL_FEATURES), np.float32)
        _check(lib.gi_get_step_features(self._h, out.ctypes.data, cnt.value, ctypes.byref(cnt)))
        return out[:cnt.value]

    def trace_exhaustive(self, algorithm, src=0, cap=MAX_TRACE):
        """Per-step features, whole-step times of S0..S3 (ms) and validity
        mask of one run per offered schedule."""
        f = np.zeros((cap, SEL_FEATURES), np.float32)
        t = np.zeros((cap, SEL_SCHEDULES), np.float32)
        v = np.zeros((cap, SEL_SCHEDULES), np.uint8)
        cnt = ctypes.c_int32()
        _check(lib.gi_trace_exhaustive(self._h, int(algorithm), int(src), f.ctypes.data,
                                       t.ctypes.data, v.ctypes.data, cap, ctypes.byref(cnt)))
        k = min(cnt.value, cap)
        return f[:k], t[:k], v[:k]

    def set_step_timing(self, enable=True):
        _check(lib.gi_set_step_timing(self._h, 1 if enable else 0))

    def step_times(self):
        """(step_ms, main_ms) float32 arrays of the last call's steps."""
        cnt = ctypes.c_int32()
        _check(lib.gi_get_step_times(self._h, None, None, 0, ctypes.byref(cnt)))
        k = cnt.value
        a = np.zeros(max(k, 1), np.float32)
        b = np.zeros(max(k, 1), np.float32)
        _check(lib.gi_get_step_times(self._h, a.ctypes.data, b.ctypes.data, k, ctypes.byref(cnt)))
        return a[:k], b[:k]

    # ---- algorithms: outputs are device tensors supplied by the caller ----
    def pagerank_eigenvector(self, ranks, eigen, iters=20, damping=0.85, fused=True,
                             stream=None):
        _check(lib.gi_pagerank_eigenvector(self._h, int(iters), float(damping), _dptr(ranks),
                                           _dptr(eigen), 1 if fused else 0, _stream(stream)))
        return ranks, eigen

    def bc(self, src, dependency, sigma=None, stream=None):
        """Single-source betweenness dependencies (float64 device tensors)."""
        _check(lib.gi_bc(self._h, int(src), _dptr(dependency), _dptr(sigma), _stream(stream)))
        return dependency

    def prdelta(self, ranks, rounds=10, damping=0.85, eps=0.1, stream=None):
        """PageRankDelta into a float64 device tensor of n entries."""
        _check(lib.gi_prdelta(self._h, int(rounds), float(damping), float(eps), _dptr(ranks),
                              _stream(stream)))
        return ranks

    def pagerank(self, ranks, iters=20, damping=0.85, stream=None):
        _check(lib.gi_pagerank(self._h, int(iters), float(damping), _dptr(ranks), _stream(stream)))
        return ranks

    def bfs(self, src, level, parent=None, stream=None):
        _check(lib.gi_bfs(self._h, int(src), _dptr(level), _dptr(parent), _stream(stream)))
        return level

    def cc(self, label, stream=None):
        _check(lib.gi_cc(self._h, _dptr(label), _stream(stream)))
        return label

    def sssp(self, src, dist, stream=None):
        _check(lib.gi_sssp(self._h, int(src), _dptr(dist), _stream(stream)))
        return dist

    def frontier_degree_sum(self, ids, count, out, stream=None):
        _check(lib.gi_frontier_degree_sum(self._h, _dptr(ids), int(count), _dptr(out),
                                          _stream(stream)))
        return out


def sparse_to_bitvec(n, ids, count, bv, stream=None):
    _check(lib.gi_frontier_sparse_to_bitvec(int(n), _dptr(ids), int(count), _dptr(bv),
                                            _stream(stream)))
    return bv


def bitvec_to_sparse(n, bv, ids, count_dev, stream=None):
    _check(lib.gi_frontier_bitvec_to_sparse(int(n), _dptr(bv), _dptr(ids), _dptr(count_dev),
                                            _stream(stream)))
    return ids


def bitvec_to_sparse_noalloc(n, bv, ids, count_dev, stream=None):
    """gi_frontier_bitvec_to_sparse_noalloc: the same conversion with the
    library's fixed scratch (no device allocation)."""
    _check(lib.gi_frontier_bitvec_to_sparse_noalloc(int(n), _dptr(bv), _dptr(ids),
                                                    _dptr(count_dev), _stream(stream)))
    return ids


def bitvec_to_boolmap(n, bv, bm, stream=None):
    _check(lib.gi_frontier_bitvec_to_boolmap(int(n), _dptr(bv), _dptr(bm), _stream(stream)))
    return bm


def boolmap_to_bitvec(n, bm, bv, stream=None):
    _check(lib.gi_frontier_boolmap_to_bitvec(int(n), _dptr(bm), _dptr(bv), _stream(stream)))
    return bv


class Selector:
    """Learned schedule selector (MLP 12 -> 64 -> 64 -> 4) trained and
    evaluated by the library's device kernels."""

    def __init__(self, seed=1):
        self._h = ctypes.c_void_p(None)
        _check(lib.gi_selector_create(int(seed), ctypes.byref(self._h)))
        _LIVE.add(self)

    def close(self):
        if self._h:
            lib.gi_selector_destroy(self._h)
            self._h = ctypes.c_void_p(None)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def params(self):
        p = np.zeros(SEL_PARAMS, np.float32)
        mu = np.zeros(SEL_FEATURES, np.float32)
        sd = np.zeros(SEL_FEATURES, np.float32)
        _check(lib.gi_selector_get_params(self._h, p.ctypes.data, mu.ctypes.data, sd.ctypes.data))
        return p, mu, sd

    def set_params(self, params=None, mu=None, sd=None):
        arrs = [None if a is None else np.ascontiguousarray(a, np.float32) for a in (params, mu, sd)]
        _check(lib.gi_selector_set_params(self._h, *[_hptr(a) for a in arrs]))

    def range(self):
        """(lo, hi): the per-feature range inference clamps to."""
        lo = np.zeros(SEL_FEATURES, np.float32)
        hi = np.zeros(SEL_FEATURES, np.float32)
        _check(lib.gi_selector_get_range(self._h, lo.ctypes.data, hi.ctypes.data))
        return lo, hi

    def set_range(self, lo=None, hi=None):
        arrs = [None if a is None else np.ascontiguousarray(a, np.float32) for a in (lo, hi)]
        _check(lib.gi_selector_set_range(self._h, *[_hptr(a) for a in arrs]))

    @staticmethod
    def _records(feats, log_ms, valid):
        f = np.ascontiguousarray(feats, np.float32).reshape(-1, SEL_FEATURES)
        y = np.ascontiguousarray(log_ms, np.float32).reshape(-1, SEL_SCHEDULES)
        v = np.ascontiguousarray(valid, np.uint8).reshape(-1, SEL_SCHEDULES)
        if not (f.shape[0] == y.shape[0] == v.shape[0]):
            raise ValueError("record arrays disagree in length")
        return f, y, v

    def train(self, feats, log_ms, valid, epochs=200, lr=1e-3, seed=7, standardise=True):
        f, y, v = self._records(feats, log_ms, valid)
        loss = np.zeros(epochs, np.float32)
        _check(lib.gi_selector_train(self._h, f.ctypes.data, y.ctypes.data, v.ctypes.data,
                                     f.shape[0], int(epochs), float(lr), int(seed),
                                     1 if standardise else 0, loss.ctypes.data))
        return loss

    def gradient(self, feats, log_ms, valid):
        f, y, v = self._records(feats, log_ms, valid)
        g = np.zeros(SEL_PARAMS, np.float32)
        loss = ctypes.c_float()
        _check(lib.gi_selector_gradient(self._h, f.ctypes.data, y.ctypes.data, v.ctypes.data,
                                        f.shape[0], g.ctypes.data, ctypes.byref(loss)))
        return g, float(loss.value)

    def predict(self, feats, bf16=False):
        f = np.ascontiguousarray(feats, np.float32).reshape(-1, SEL_FEATURES)
        out = np.zeros((f.shape[0], SEL_SCHEDULES), np.float32)
        _check(lib.gi_selector_predict(self._h, f.ctypes.data, f.shape[0], 1 if bf16 else 0,
                                       out.ctypes.data))
        return out


class Task(ctypes.Structure):
    _fields_ = [("graph", ctypes.c_int32), ("algorithm", ctypes.c_int32), ("src", ctypes.c_int32),
                ("iters", ctypes.c_int32), ("damping", ctypes.c_float),
                ("workgroups", ctypes.c_int32), ("out", ctypes.c_void_p),
                ("parent", ctypes.c_void_p), ("sssp_delta", ctypes.c_uint32),
                ("hybrid_divisor", ctypes.c_int32)]


class Batch:
    """Batched persistent execution of BFS / PageRank / SSSP tasks.

    tasks: sequence of dicts with keys graph (index), algorithm (ALG_BFS,
    ALG_PAGERANK or ALG_SSSP), out (device tensor of n int32, float32 or
    int32-as-uint32 distances), and src / iters / damping / workgroups /
    parent / sssp_delta / hybrid_divisor as needed."""

    def __init__(self, graphs, tasks):
        self.graphs = list(graphs)
        self._outs = [(t["out"], t.get("parent")) for t in tasks]   # keep the tensors alive
        arr = (Task * len(tasks))()
        for i, t in enumerate(tasks):
            arr[i] = Task(int(t["graph"]), int(t["algorithm"]), int(t.get("src", 0)),
                          int(t.get("iters", 20)), float(t.get("damping", 0.85)),
                          int(t.get("workgroups", 0)), _dptr(t["out"]), _dptr(t.get("parent")),
                          int(t.get("sssp_delta", 0)), int(t.get("hybrid_divisor", 0)))
        hs = (ctypes.c_void_p * len(self.graphs))(*[g._h.value for g in self.graphs])
        self._h = ctypes.c_void_p(None)
        self.ntasks = len(tasks)
        _check(lib.gi_batch_create(hs, len(self.graphs), arr, len(tasks), ctypes.byref(self._h)))
        _LIVE.add(self)

    def close(self):
        if self._h:
            lib.gi_batch_destroy(self._h)
            self._h = ctypes.c_void_p(None)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def autotune(self, reps=3):
        _check(lib.gi_batch_autotune(self._h, int(reps)))

    def set_threads(self, threads):
        """Pin the workgroup size (256, 512 or 1024); 0 lets the autotuner choose."""
        _check(lib.gi_batch_set_threads(self._h, int(threads)))

    def threads(self):
        t = ctypes.c_int32(0)
        _check(lib.gi_batch_get_threads(self._h, ctypes.byref(t)))
        return t.value

    def set_placement(self, xcd_local):
        """1: keep each task's workgroups on one XCD when they fit; 0: spread."""
        _check(lib.gi_batch_set_placement(self._h, 1 if xcd_local else 0))

    def placement(self):
        x = ctypes.c_int32(0)
        _check(lib.gi_batch_get_placement(self._h, ctypes.byref(x)))
        return x.value

    def set_barrier_scope(self, scope):
        """BARRIER_XCD (default): tasks on one XCD only invalidate L1 at their
        barriers; BARRIER_AGENT: every barrier writes back and invalidates
        the L2."""
        _check(lib.gi_batch_set_barrier_scope(self._h, int(scope)))

    def barrier_scope(self):
        x = ctypes.c_int32(0)
        _check(lib.gi_batch_get_barrier_scope(self._h, ctypes.byref(x)))
        return x.value

    def set_trace(self, cap):
        """Keep up to cap per-step records per task from the next run on."""
        _check(lib.gi_batch_set_trace(self._h, int(cap)))

    def trace(self, task, cap=4096):
        """(start_ns, pull, frontier) arrays of task's steps in the last run,
        the last record marking its end."""
        t = np.zeros(cap, np.int64)
        p = np.zeros(cap, np.int32)
        f = np.zeros(cap, np.int64)
        c = ctypes.c_int32(0)
        _check(lib.gi_batch_get_trace(self._h, int(task), t.ctypes.data, p.ctypes.data,
                                      f.ctypes.data, int(cap), ctypes.byref(c)))
        k = c.value
        return t[:k], p[:k], f[:k]

    def run(self, use_graph=True, stream=None):
        _check(lib.gi_batch_run(self._h, 1 if use_graph else 0, _stream(stream)))

    def launch(self, use_graph=True, stream=None):
        """Enqueue a run and return at once; wait() completes it."""
        _check(lib.gi_batch_launch(self._h, 1 if use_graph else 0, _stream(stream)))

    def wait(self):
        _check(lib.gi_batch_wait(self._h))

    def info(self):
        ms = ctypes.c_float()
        grid = ctypes.c_int32()
        wg = np.zeros(self.ntasks, np.int32)
        lv = np.zeros(self.ntasks, np.int32)
        tm = np.zeros(self.ntasks, np.float32)
        _check(lib.gi_batch_info(self._h, ctypes.byref(ms), ctypes.byref(grid), wg.ctypes.data,
                                 lv.ctypes.data, tm.ctypes.data))
        return {"ms": ms.value, "grid": grid.value, "workgroups": wg, "levels": lv,
                "task_ms": tm}

    def edges(self):
        """Edges each task relaxed in the last run (SSSP tasks; 0 for others)."""
        e = np.zeros(self.ntasks, np.int64)
        _check(lib.gi_batch_task_counters(self._h, e.ctypes.data, None))
        return e

    def pr_block_edges(self):
        """Per graph: the PageRank block size (edges) the batch uses; 0 for
        graphs without PageRank tasks."""
        e = np.zeros(len(self.graphs), np.int32)
        _check(lib.gi_batch_pr_block_edges(self._h, e.ctypes.data))
        return e

    def barrier_ms(self):
        """Per task: mean time a workgroup spent in task barriers in the last
        run (ms; 0 for one-workgroup tasks)."""
        t = np.zeros(self.ntasks, np.float32)
        _check(lib.gi_batch_task_counters(self._h, None, t.ctypes.data))
        return t
