"""The C-ABI boundary with torch owning the memory: a graph built from torch
CUDA tensors (device-pointer ingest) whose core arrays live in a torch-
allocated workspace, every other library allocation taken from torch's
caching allocator, PageRank returning after enqueue, and the refusals."""
import ctypes

import numpy as np
import pytest

import graphgen as gg
import oracle
from gpu_util import PR_RTOL, pr_max_rel, say, torch_dev

pytestmark = pytest.mark.gpu


def _gi():
    import paper_1805_00923_amd as gi
    return gi


def _tensors(el, torch, dev):
    gi = _gi()
    off, idx, _ = gi.build_adjacency(el.n, el.src, el.dst)
    ioff, iidx, _ = gi.build_adjacency(el.n, el.dst, el.src)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.int32)).to(dev)
    return (off, idx, ioff, iidx), (t(off), t(idx), t(ioff), t(iidx))


@pytest.mark.parametrize("with_in", [True, False])
def test_graph_from_torch_tensors_in_a_torch_workspace(with_in):
    gi = _gi()
    torch, dev = torch_dev()
    el = gg.rmat(14, seed=31)
    og = oracle.Graph(el)
    host, (off, idx, ioff, iidx) = _tensors(el, torch, dev)
    m = int(idx.numel())
    nbytes = gi.workspace_size(el.n, m)
    ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    base_live, _ = gi.live_allocations()
    say("boundary: rmat14 from device tensors, workspace %d bytes, in-adjacency %s" %
        (nbytes, with_in))
    g = gi.Graph.from_tensors(el.n, off, idx, None, ioff if with_in else None,
                              iidx if with_in else None, None, workspace=ws)
    # the device CSC equals the host-built one
    co, ci, _ = g.in_adjacency()
    assert np.array_equal(co, host[2]) and np.array_equal(ci, host[3])
    # everything the library allocated beyond the workspace came from torch
    live, from_torch = gi.live_allocations()
    assert live > base_live and from_torch == live
    src = int(gg.pick_sources(el, 1, 7)[0])
    level = torch.full((el.n,), -7, dtype=torch.int32, device=dev)
    parent = torch.full((el.n,), -7, dtype=torch.int32, device=dev)
    g.bfs(src, level, parent)
    torch.cuda.synchronize()
    ref, _ = oracle.bfs(og, src)
    lv = level.cpu().numpy()
    assert np.array_equal(lv, ref)
    assert oracle.check_bfs_parents(og, src, lv, parent.cpu().numpy()) == []
    ref_pr = oracle.pagerank(og, 20, 0.85)
    for sched in (dict(), dict(vertex_order=1)):
        g.set_schedule(**sched)
        x = torch.full((el.n,), -1.0, dtype=torch.float32, device=dev)
        g.pagerank(x, 20, 0.85)
        g.sync()
        assert pr_max_rel(x.cpu().numpy(), ref_pr) <= PR_RTOL, sched
    g.close()
    live_after, _ = gi.live_allocations()
    assert live_after == base_live  # every allocation went back where it came from
    del ws


def test_every_library_allocation_comes_from_torch():
    gi = _gi()
    torch, dev = torch_dev()
    el = gg.rmat(12, seed=32)
    base_live, base_torch = gi.live_allocations()
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated(dev)
    g = gi.Graph.from_edges(el.n, el.src, el.dst)
    g.set_schedule(vertex_order=1)
    x = torch.empty(el.n, dtype=torch.float32, device=dev)
    g.pagerank(x, 3, 0.85)  # builds the ordered copy on first use
    g.sync()
    live, from_torch = gi.live_allocations()
    assert live - base_live == from_torch - base_torch > 0
    # torch accounts for the library's memory
    assert torch.cuda.memory_allocated(dev) > before
    g.close()
    assert gi.live_allocations() == (base_live, base_torch)


def test_pagerank_returns_after_enqueue_and_stats_wait():
    gi = _gi()
    torch, dev = torch_dev()
    el = gg.rmat(15, seed=33)
    og = oracle.Graph(el)
    g = gi.Graph.from_edges(el.n, el.src, el.dst)
    s = torch.cuda.Stream()
    x = torch.full((el.n,), -1.0, dtype=torch.float32, device=dev)
    say("boundary: async pagerank on a side stream")
    with torch.cuda.stream(s):
        g.pagerank(x, 20, 0.85, stream=s)
    st = g.stats()  # waits for the run, then reads its time
    assert st.kernel_ms > 0 and st.steps == 20
    g.sync()
    s.synchronize()
    assert pr_max_rel(x.cpu().numpy(), oracle.pagerank(og, 20, 0.85)) <= PR_RTOL
    g.close()


def test_pagerank_ordered_replays_from_a_graph():
    """A degree-ordered PageRank call that repeats the previous call's
    arguments replays the run from a HIP graph: every replay, with the
    program's own eager work and synchronizations in between, on the default
    stream and on a side stream, matches the oracle and the direct run; a
    changed argument (output, iterations) or step timing runs directly."""
    gi = _gi()
    torch, dev = torch_dev()
    el = gg.rmat(14, seed=34)
    og = oracle.Graph(el)
    ref = oracle.pagerank(og, 20, 0.85)
    g = gi.Graph.from_edges(el.n, el.src, el.dst)
    g.set_schedule(vertex_order=1)
    x = torch.full((el.n,), -1.0, dtype=torch.float32, device=dev)
    g.pagerank(x, 20, 0.85)  # direct (new arguments)
    g.sync()
    direct = x.cpu().numpy()
    assert pr_max_rel(direct, ref) <= PR_RTOL
    launches = g.stats().launches
    side = torch.cuda.Stream()
    lv = torch.empty(el.n, dtype=torch.int32, device=dev)
    for rep in range(4):
        say("boundary: ordered pagerank replay %d" % rep)
        x.fill_(-3.0)  # eager work on the stream before the replay
        if rep % 2:
            with torch.cuda.stream(side):
                side.wait_stream(torch.cuda.current_stream())
                g.pagerank(x, 20, 0.85, stream=side)
            torch.cuda.current_stream().wait_stream(side)
        else:
            g.pagerank(x, 20, 0.85)
        y = x.clone()  # read on the caller's stream after the run
        st = g.stats()
        assert st.kernel_ms > 0 and st.steps == 20 and st.launches == launches
        torch.cuda.synchronize()
        got = y.cpu().numpy()
        assert pr_max_rel(got, ref) <= PR_RTOL, rep
        assert np.max(np.abs(got - direct) / np.maximum(np.abs(direct), 1e-30)) <= 1e-5, rep
        g.bfs(int(rep), lv)  # other work of the graph between replays
        torch.cuda.synchronize()
    # changed arguments: a direct run, then replays of the new arguments
    z = torch.full((el.n,), -1.0, dtype=torch.float32, device=dev)
    ref7 = oracle.pagerank(og, 7, 0.85)
    for _ in range(3):
        z.fill_(-2.0)
        g.pagerank(z, 7, 0.85)
        g.sync()
        assert pr_max_rel(z.cpu().numpy(), ref7) <= PR_RTOL
    g.set_step_timing(True)
    x.fill_(-4.0)
    g.pagerank(x, 20, 0.85)
    g.sync()
    assert len(g.step_times()[0]) == 20
    assert pr_max_rel(x.cpu().numpy(), ref) <= PR_RTOL
    g.close()


def test_workspace_refusals():
    gi = _gi()
    torch, dev = torch_dev()
    el = gg.rmat(10, seed=34)
    _, (off, idx, ioff, iidx) = _tensors(el, torch, dev)
    m = int(idx.numel())
    need = gi.workspace_size(el.n, m)
    small = torch.empty(need // 2, dtype=torch.uint8, device=dev)
    with pytest.raises(gi.GiError) as e:
        gi.Graph.from_tensors(el.n, off, idx, None, ioff, iidx, None, workspace=small)
    assert e.value.status == gi.GI_ERR_INVALID_ARG and "workspace" in str(e.value)
    big = torch.empty(need + 512, dtype=torch.uint8, device=dev)
    with pytest.raises(gi.GiError) as e:  # misaligned by 4 bytes
        h = ctypes.c_void_p(None)
        gi._check(gi.lib.gi_graph_create_ex(el.n, m, off.data_ptr(), idx.data_ptr(), None, None,
                                            None, None, gi.PTR_DEVICE, big.data_ptr() + 4,
                                            need, None, ctypes.byref(h)))
    assert e.value.status == gi.GI_ERR_INVALID_ARG
    with pytest.raises(gi.GiError) as e:
        h = ctypes.c_void_p(None)
        gi._check(gi.lib.gi_graph_create_ex(el.n, m, off.data_ptr(), idx.data_ptr(), None, None,
                                            None, None, 7, None, 0, None, ctypes.byref(h)))
    assert e.value.status == gi.GI_ERR_INVALID_ARG
    # an exactly sized workspace is enough
    exact = torch.empty(need, dtype=torch.uint8, device=dev)
    g = gi.Graph.from_tensors(el.n, off, idx, None, ioff, iidx, None, workspace=exact)
    g.close()
