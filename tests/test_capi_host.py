"""Host-side checks of the C ABI that need no GPU: the library loads and
exports every symbol the header declares, the host adjacency build matches
the oracle bit for bit, and argument errors are reported before any device
work."""
import ctypes
import os
import re

import numpy as np
import pytest

import graphgen as gg
import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _gi():
    import paper_1805_00923_amd as gi
    return gi


def header_symbols():
    txt = open(os.path.join(ROOT, "include", "graphit_mi.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(gi_[a-z0-9_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    gi = _gi()
    syms = header_symbols()
    assert len(syms) >= 20
    for s in syms:
        assert hasattr(gi.lib, s), s
        assert s in gi._SIGS, "binding lacks a signature for " + s
    assert gi.lib.gi_abi_version() == 1


@pytest.mark.parametrize("seed", range(6))
def test_host_ingest_matches_oracle(seed):
    gi = _gi()
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 300))
    el = gg.uniform(n, int(rng.integers(0, 6 * n)), seed=seed)
    w = gg.uniform_weights(el.m, seed + 50, 1, 7)  # small range => many repeated pairs with ties
    og = oracle.build_adj(n, el.src, el.dst, w)
    off, idx, ww = gi.build_adjacency(n, el.src, el.dst, w)
    assert np.array_equal(off, og.off)
    assert np.array_equal(idx, og.idx)
    assert np.array_equal(ww, og.w)


def test_host_ingest_rmat_and_grid():
    gi = _gi()
    for el in (gg.rmat(12, seed=3), gg.grid(40, 50, 0.05, seed=9)):
        og = oracle.build_adj(el.n, el.dst, el.src, el.w)   # CSC
        off, idx, ww = gi.build_adjacency(el.n, el.dst, el.src, el.w)
        assert np.array_equal(off, og.off) and np.array_equal(idx, og.idx)
        if el.w is not None:
            assert np.array_equal(ww, og.w)


def test_host_ingest_weighted_rmat16_with_repeats():
    """Rows split over all worker threads, repeated pairs with different
    weights (the smallest survives), self-loops dropped."""
    gi = _gi()
    el = gg.rmat(16, seed=8)
    src = np.concatenate([el.src, el.dst[::3], np.arange(0, el.n, 97, dtype=np.int32)])
    dst = np.concatenate([el.dst, el.src[::3], np.arange(0, el.n, 97, dtype=np.int32)])
    w = gg.uniform_weights(len(src), 12, 1, 50)
    og = oracle.build_adj(el.n, src, dst, w)
    off, idx, ww = gi.build_adjacency(el.n, src, dst, w)
    assert np.array_equal(off, og.off) and np.array_equal(idx, og.idx)
    assert np.array_equal(ww, og.w)


def test_ingest_reports_first_bad_record():
    gi = _gi()
    src = np.zeros(100000, np.int32)
    dst = np.ones(100000, np.int32)
    src[77777] = 9
    dst[99998] = -1
    with pytest.raises(gi.GiError) as e:
        gi.build_adjacency(4, src, dst)
    assert e.value.status == gi.GI_ERR_INVALID_ARG and "77777" in str(e.value)


def test_ingest_rejects_bad_records():
    gi = _gi()
    with pytest.raises(gi.GiError) as e:
        gi.build_adjacency(4, np.array([0, 4]), np.array([1, 2]))
    assert e.value.status == gi.GI_ERR_INVALID_ARG
    with pytest.raises(gi.GiError):
        gi.build_adjacency(0, np.zeros(0), np.zeros(0))


def _create(n, m, off, idx, ioff=None, iidx=None):
    gi = _gi()
    h = ctypes.c_void_p()
    p = lambda a: None if a is None else a.ctypes.data
    st = gi.lib.gi_graph_create(n, m, p(off), p(idx), None, p(ioff), p(iidx), None, ctypes.byref(h))
    return st, gi.last_error()


def test_graph_create_validates_before_device_work():
    gi = _gi()
    off = np.array([0, 1, 2, 2], np.int32)
    idx = np.array([1, 2], np.int32)
    # bad offsets
    st, msg = _create(3, 2, np.array([0, 2, 1, 2], np.int32), idx)
    assert st == gi.GI_ERR_INVALID_ARG and "decrease" in msg
    # neighbour out of range
    st, _ = _create(3, 2, off, np.array([1, 3], np.int32))
    assert st == gi.GI_ERR_INVALID_ARG
    # unsorted row
    st, msg = _create(2, 2, np.array([0, 2, 2], np.int32), np.array([1, 1], np.int32))
    assert st == gi.GI_ERR_INVALID_ARG and "ascending" in msg
    # m beyond int32 offsets
    st, _ = _create(3, 2 ** 31, off, idx)
    assert st == gi.GI_ERR_OVERFLOW
    # n < 1
    st, _ = _create(0, 0, np.array([0], np.int32), idx)
    assert st == gi.GI_ERR_INVALID_ARG
    # CSC that is not the transpose
    st, msg = _create(3, 2, off, idx, np.array([0, 0, 1, 2], np.int32),
                      np.array([1, 0], np.int32))
    assert st == gi.GI_ERR_INVALID_ARG


def test_graph_create_names_the_first_bad_in_edge():
    """In-adjacency checked by worker threads over row ranges: the error
    names the first bad in-edge in row order, for a missing edge and for a
    weight that differs between the two adjacencies."""
    gi = _gi()
    el = gg.rmat(12, seed=5)
    w = gg.uniform_weights(el.m, 3, 1, 100)
    off, idx, ww = gi.build_adjacency(el.n, el.src, el.dst, w)
    ioff, iidx, iw = gi.build_adjacency(el.n, el.dst, el.src, w)
    m = len(idx)
    rows = np.repeat(np.arange(el.n), np.diff(ioff))
    late = int(np.nonzero(rows > 3 * el.n // 4)[0][0])      # an in-edge in a late row
    early = int(np.nonzero(rows > el.n // 3)[0][0])         # and one in an earlier row
    p = lambda a: a.ctypes.data
    h = ctypes.c_void_p()
    bad = iidx.copy()
    for k in (late, early):
        v, u = int(rows[k]), int(iidx[k])
        # a source that is not an in-neighbour of v keeps the degrees equal
        bad[k] = next(x for x in range(el.n) if x != u and x not in set(iidx[ioff[v]:ioff[v + 1]]))
    st = gi.lib.gi_graph_create(el.n, m, p(off), p(idx), None, p(ioff), p(bad), None,
                                ctypes.byref(h))
    v, u = int(rows[early]), int(bad[early])
    assert st == gi.GI_ERR_INVALID_ARG
    assert "in-edge %d->%d is not an out-edge" % (u, v) in gi.last_error()
    badw = iw.copy()
    badw[late] += 1
    st = gi.lib.gi_graph_create(el.n, m, p(off), p(idx), p(ww), p(ioff), p(iidx), p(badw),
                                ctypes.byref(h))
    v, u = int(rows[late]), int(iidx[late])
    assert st == gi.GI_ERR_INVALID_ARG
    assert "weight of %d->%d differs" % (u, v) in gi.last_error()


def test_null_handles_rejected():
    gi = _gi()
    assert gi.lib.gi_bfs(None, 0, None, None, None) == gi.GI_ERR_INVALID_ARG
    assert gi.lib.gi_pagerank(None, 20, 0.85, None, None) == gi.GI_ERR_INVALID_ARG
    assert gi.lib.gi_cc(None, None, None) == gi.GI_ERR_INVALID_ARG
    assert gi.lib.gi_sssp(None, 0, None, None) == gi.GI_ERR_INVALID_ARG
    assert gi.lib.gi_set_schedule(None, None) == gi.GI_ERR_INVALID_ARG
    assert gi.lib.gi_graph_destroy(None) == gi.GI_OK
    assert gi.lib.gi_frontier_sparse_to_bitvec(0, None, 0, None, None) == gi.GI_ERR_INVALID_ARG


def test_default_schedule():
    gi = _gi()
    s = gi.default_schedule()
    assert s.direction == gi.DENSE_PULL_SPARSE_PUSH
    assert s.hybrid_divisor == 20 and s.num_segments == 1 and s.steps_per_sync == 0


def test_hybrid_rule_as_written():
    """Dense side iff |F| + sum outdeg(F) > m / divisor (section 2)."""
    gi = _gi()
    m = 1000
    for nf in range(0, 60, 7):
        for d in range(0, 80, 9):
            assert gi.hybrid_choose_dense(nf, d, m, 20) == ((nf + d) * 20 > m)
    assert not gi.hybrid_choose_dense(25, 25, 1000, 20)   # exactly m/20 stays sparse
    assert gi.hybrid_choose_dense(25, 26, 1000, 20)


def test_allocator_registration_and_exit_release():
    """The binding registers torch's caching allocator with the library and,
    at interpreter exit, closes every object still holding device memory
    before torch shuts down (a close after that could reach a torch or HIP
    runtime already torn down)."""
    gi = _gi()
    c = ctypes.c_int64()
    assert gi.lib.gi_live_allocations(ctypes.byref(c), None) == gi.GI_OK and c.value >= 0
    # only one of the two functions is refused; NULL, NULL goes back to hipMalloc
    assert gi.lib.gi_set_allocator(gi._TORCH_ALLOC, gi._FREE_FN(), None) == gi.GI_ERR_INVALID_ARG
    gi.use_torch_allocator(False)
    gi.use_torch_allocator(True)

    class Holder:
        closed = 0

        def close(self):
            Holder.closed += 1

    h = Holder()
    gi._LIVE.add(h)
    gi._release_at_exit()
    assert Holder.closed == 1
    gi._LIVE.discard(h)
    # the release callback does nothing while the interpreter finalizes
    import sys
    assert hasattr(sys, "is_finalizing")


def test_workspace_size_arguments():
    gi = _gi()
    b = ctypes.c_size_t()
    assert gi.lib.gi_graph_workspace_size(0, 0, 0, ctypes.byref(b)) == gi.GI_ERR_INVALID_ARG
    assert gi.lib.gi_graph_workspace_size(10, -1, 0, ctypes.byref(b)) == gi.GI_ERR_INVALID_ARG
    assert gi.lib.gi_graph_workspace_size(10, 2**31, 0, ctypes.byref(b)) == gi.GI_ERR_OVERFLOW
    small = gi.workspace_size(1000, 5000)
    assert small % 256 == 0 and small >= 4 * (2 * 1001 + 2 * 5000)
    assert gi.workspace_size(1000, 5000, weighted=True) >= small + 2 * 4 * 5000
    # a NULL handle is refused before anything else
    h = ctypes.c_void_p(None)
    assert gi.lib.gi_graph_create_ex(10, 0, None, None, None, None, None, None, 5, None, 0,
                                     None, ctypes.byref(h)) == gi.GI_ERR_INVALID_ARG
    assert gi.lib.gi_sync_status(None) == gi.GI_ERR_INVALID_ARG
