"""Parity at the full benchmark sizes, in the launch configuration bench.py
times (default hybrid schedule, bitvector frontier, adaptive batching,
per-step timing on): RMAT scale 22 BFS from sampled sources and CC, checked
exactly against the oracle; PageRank on RMAT scale 22 within 1e-6; and
delta-stepping on the 4096 x 4096 grid (1% shortcuts, and none) against
Dijkstra from sampled sources, on the plain path and as the benchmark's
batched SSSP tasks."""
import numpy as np
import pytest

import graphgen as gg
import oracle
from gpu_util import (PR_RTOL, device_graph, pr_max_rel, run_bfs, run_cc, run_pr, run_sssp,
                      say)

pytestmark = pytest.mark.gpu

_G = {}


def rmat22():
    if "rmat22" not in _G:
        say("building rmat22")
        el = gg.rmat(22, 16, seed=2)
        g = device_graph(el)
        og = oracle.Graph(el)
        _G["rmat22"] = (el, g, og)
    return _G["rmat22"]


def test_rmat22_bfs_sampled_sources():
    el, g, og = rmat22()
    g.set_schedule(direction=3, dense_frontier=0, hybrid_divisor=20)  # bitvector
    g.set_step_timing(True)
    srcs = gg.pick_sources(el, 64, 3)
    # first, middle and last of the 64 benchmark sources
    for s in (srcs[0], srcs[31], srcs[63]):
        say("rmat22 bfs src=%d" % s)
        lv, par = run_bfs(g, s)
        ref = oracle.bfs(og, int(s))[0]
        assert np.array_equal(lv, ref)
        assert oracle.check_bfs_parents(og, int(s), lv, par) == []
        assert g.stats().dense_steps > 0
    g.set_step_timing(False)


def test_rmat22_batched_bfs_all_sources():
    """The benchmark's batched launch: 64 sources, levels of three checked
    against the oracle, parents of all validated on those three, levels of
    all equal to the plain path's."""
    import torch
    import paper_1805_00923_amd as gi
    el, g, og = rmat22()
    g.set_schedule(direction=3, dense_frontier=0, hybrid_divisor=20)
    srcs = gg.pick_sources(el, 64, 3)
    outs = [(torch.empty(g.n, dtype=torch.int32, device="cuda:0"),
             torch.empty(g.n, dtype=torch.int32, device="cuda:0")) for _ in srcs]
    b = gi.Batch([g], [dict(graph=0, algorithm=gi.ALG_BFS, src=int(s), out=o, parent=p)
                       for s, (o, p) in zip(srcs, outs)])
    say("rmat22 batched autotune")
    b.autotune(reps=1)
    say("rmat22 batched run")
    b.run(use_graph=True)
    for i in (0, 31, 63):
        lv = outs[i][0].cpu().numpy()
        assert np.array_equal(lv, oracle.bfs(og, int(srcs[i]))[0]), i
        assert oracle.check_bfs_parents(og, int(srcs[i]), lv, outs[i][1].cpu().numpy()) == [], i
    ref = torch.empty(g.n, dtype=torch.int32, device="cuda:0")
    for i in range(0, 64, 7):
        g.bfs(int(srcs[i]), ref)
        assert torch.equal(ref, outs[i][0]), i
    b.close()


def test_rmat22_cc():
    el, g, og = rmat22()
    g.set_schedule(direction=3, dense_frontier=0, hybrid_divisor=20)  # bitvector
    say("rmat22 cc")
    lab = run_cc(g)
    ref, rounds = oracle.cc(og)
    assert np.array_equal(lab, ref)
    assert g.stats().steps == rounds


@pytest.mark.parametrize("sched", [dict(direction=d) for d in range(5)] + [
    dict(direction=3, dense_frontier=1), dict(num_segments=8, segment_strategy=1, hybrid_divisor=4)],
    ids=lambda c: "_".join("%s%s" % (k[:8], v) for k, v in c.items()))
def test_rmat22_cc_direct(sched):
    """CC without the symmetric copy (the form graphs with 2m > 2^31 - 1
    take) at RMAT-22 under every direction, both frontier kinds and the
    benchmark's segmented schedule."""
    import paper_1805_00923_amd as gi
    el, g, og = rmat22()
    if "rmat22_cc" not in _G:
        _G["rmat22_cc"] = oracle.cc(og)
    ref, rounds = _G["rmat22_cc"]
    g.set_schedule(cc_adjacency=gi.CC_ADJ_DIRECT, **sched)
    say("rmat22 cc direct %s" % sched)
    lab = run_cc(g)
    assert np.array_equal(lab, ref)
    assert g.stats().steps == rounds
    g.set_schedule()


def test_rmat22_pagerank():
    el, g, og = rmat22()
    g.set_schedule()
    say("rmat22 pagerank")
    x = run_pr(g, 20)
    assert pr_max_rel(x, oracle.pagerank(og, 20, 0.85)) <= PR_RTOL
    g.set_schedule(num_segments=8)
    say("rmat22 pagerank 8 segments")
    x = run_pr(g, 20)
    assert pr_max_rel(x, oracle.pagerank(og, 20, 0.85)) <= PR_RTOL
    g.set_schedule(num_segments=8, segments_concurrent=1)
    say("rmat22 pagerank 8 concurrent segments")
    x = run_pr(g, 20)
    assert pr_max_rel(x, oracle.pagerank(og, 20, 0.85)) <= PR_RTOL
    for cfg in (dict(vertex_order=1), dict(vertex_order=1, block_threads=1024),
                dict(vertex_order=1, block_threads=512, pull_items_per_thread=16)):
        g.set_schedule(**cfg)
        say("rmat22 pagerank %s" % cfg)
        x = run_pr(g, 20)
        assert pr_max_rel(x, oracle.pagerank(og, 20, 0.85)) <= PR_RTOL, cfg
    g.set_schedule()
    _G.pop("rmat22", None)


def test_grid4096_sssp_sampled_sources():
    say("building grid4096")
    el = gg.grid(4096, 4096, 0.01, seed=4)
    g = device_graph(el)
    og = oracle.Graph(el)
    srcs = gg.pick_sources(el, 4, 5)
    for delta in (4096,):
        g.set_schedule(sssp_delta=delta)
        g.set_step_timing(True)
        for s in srcs[:2]:
            say("grid4096 sssp src=%d delta=%d" % (s, delta))
            d = run_sssp(g, s)
            assert np.array_equal(d, oracle.dijkstra(og, int(s)))
    g.set_step_timing(False)


@pytest.mark.parametrize("frac", [0.01, 0.0])
def test_grid4096_batched_sssp(frac):
    """The benchmark's batched SSSP launch (4 sources as SSSP tasks,
    autotuned): distances of two sources bit-exact against Dijkstra, all four
    equal to the plain path's; with no shortcuts the diameter is 8190 hops
    and each task runs thousands of delta-stepping phases."""
    import torch
    import paper_1805_00923_amd as gi
    say("building grid4096 frac=%g" % frac)
    el = gg.grid(4096, 4096, frac, seed=4)
    g = device_graph(el)
    og = oracle.Graph(el)
    srcs = gg.pick_sources(el, 4, 5)
    outs = [torch.empty(g.n, dtype=torch.int32, device="cuda:0") for _ in srcs]
    b = gi.Batch([g], [dict(graph=0, algorithm=gi.ALG_SSSP, src=int(s), sssp_delta=8192,
                            out=o) for s, o in zip(srcs, outs)])
    say("grid4096 batched sssp autotune")
    b.autotune(reps=1)
    say("grid4096 batched sssp run")
    b.run(use_graph=True)
    torch.cuda.synchronize()
    for i in (0, 3):
        say("grid4096 dijkstra src=%d" % srcs[i])
        d = outs[i].cpu().numpy().view(np.uint32)
        assert np.array_equal(d, oracle.dijkstra(og, int(srcs[i]))), i
    g.set_schedule(sssp_delta=8192)
    for i, s in enumerate(srcs):
        say("grid4096 plain sssp src=%d" % s)
        assert np.array_equal(run_sssp(g, s), outs[i].cpu().numpy().view(np.uint32)), i
    g.set_schedule()
    b.close()
    g.close()
