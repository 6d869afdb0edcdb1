"""GPU parity: every traversal schedule of the library against the oracle.

BFS levels, CC labels (and round counts) and SSSP distances must match the
oracle exactly; BFS parents must form a valid BFS tree; PageRank must be
within 1e-6 max relative error of the FP64 oracle.  Inputs are seeded
synthetic graphs: small families that reach every code path (long rows,
empty rows, ragged bit-vector tails, many levels) and the full-size
workloads.
"""
import itertools

import numpy as np
import pytest

import graphgen as gg
import oracle
from gpu_util import (PR_RTOL, device_graph, pr_max_rel, run_bfs, run_cc, run_pr, run_sssp,
                      say, torch_dev)

pytestmark = pytest.mark.gpu


def _gi():
    import paper_1805_00923_amd as gi
    return gi


def families():
    fam = [
        gg.cycle(100), gg.path(300), gg.star(500), gg.star(400, out=False), gg.complete(40),
        gg.empty(17), gg.empty(1), gg.grid(30, 41, 0.0, weighted=False),
        gg.uniform(2000, 9000, seed=3), gg.uniform(129, 40, seed=4),
        gg.rmat(8, seed=21), gg.rmat(11, seed=22), gg.rmat(13, seed=23),
        # more than 256 bitvector words: several compaction workgroups
        gg.rmat(15, seed=24), gg.uniform(300000, 1200000, seed=25),
    ]
    # a hub with more in- and out-edges than any block or wave holds
    n = 5000
    hub_src = np.concatenate([np.zeros(n - 1, np.int32), np.arange(1, n, dtype=np.int32)])
    hub_dst = np.concatenate([np.arange(1, n, dtype=np.int32), np.zeros(n - 1, np.int32)])
    extra = gg.uniform(n, 3 * n, seed=5)
    fam.append(gg.EdgeList(n, np.concatenate([hub_src, extra.src]),
                           np.concatenate([hub_dst, extra.dst]), name="hub5000"))
    return fam


_FAM = None
_ORACLE = {}


def fam_graphs():
    global _FAM
    if _FAM is None:
        _FAM = [(el, device_graph(el), oracle.Graph(el)) for el in families()]
    return _FAM


def sources_of(el, k=3):
    s = gg.pick_sources(el, k, 3)
    return [0] if s.size == 0 else list(s)


TRAVERSAL_SCHEDULES = [
    dict(direction=d, dense_frontier=f, steps_per_sync=p)
    for d, f, p in itertools.product(range(5), (0, 1), (0, 1))
]


def sched_name(s):
    return "dir%d_fr%d_sync%d" % (s["direction"], s["dense_frontier"], s["steps_per_sync"])


# ------------------------------------------------------------------ PageRank

def test_pagerank_families_default():
    for el, g, og in fam_graphs():
        for iters in (0, 1, 20):
            say("pr %s iters=%d" % (el.name, iters))
            g.set_schedule()
            x = run_pr(g, iters)
            ref = oracle.pagerank(og, iters)
            assert pr_max_rel(x, ref) <= PR_RTOL, (el.name, iters)


@pytest.mark.parametrize("cfg", [
    dict(), dict(pull_block_edges=64), dict(pull_block_edges=256),
    dict(pull_block_edges=8192, block_threads=512), dict(block_threads=64),
    dict(block_threads=128), dict(num_segments=2), dict(num_segments=3, segment_strategy=1),
    dict(num_segments=8, pull_block_edges=128), dict(num_segments=64, segment_strategy=1),
    dict(num_segments=8, segments_concurrent=1),
    dict(num_segments=3, segment_strategy=1, segments_concurrent=1, pull_block_edges=256),
    # degree-ordered pull: LDS sources none, a few, default; every tile shape
    dict(vertex_order=1), dict(vertex_order=1, pull_hot_sources=0),
    dict(vertex_order=1, pull_hot_sources=64, pull_items_per_thread=4),
    dict(vertex_order=1, pull_items_per_thread=16, block_threads=512),
    dict(vertex_order=1, block_threads=1024, pull_items_per_thread=8),
    dict(vertex_order=1, block_threads=1024, pull_items_per_thread=4, pull_hot_sources=0),
    dict(vertex_order=1, block_threads=512, pull_items_per_thread=4, pull_hot_sources=100000),
], ids=lambda c: "_".join("%s%s" % (k[:8], v) for k, v in c.items()))
def test_pagerank_schedules(cfg):
    for el, g, og in fam_graphs():
        say("pr %s %s" % (el.name, cfg))
        g.set_schedule(**cfg)
        x = run_pr(g, 20)
        assert pr_max_rel(x, oracle.pagerank(og, 20)) <= PR_RTOL, el.name
    for el, g, _ in fam_graphs():
        g.set_schedule()


def test_pagerank_rmat16_workload():
    """The PageRank workload: RMAT scale 16, edge factor 16, 20 iterations."""
    el = gg.rmat(16, seed=1)
    og = oracle.Graph(el)
    g = device_graph(el)
    ref = oracle.pagerank(og, 20, 0.85)
    for cfg in (dict(), dict(num_segments=4), dict(num_segments=4, segment_strategy=1),
                dict(num_segments=8, segments_concurrent=1),
                dict(num_segments=16, segments_concurrent=1),
                dict(num_segments=8, segments_concurrent=1, segment_strategy=1),
                dict(vertex_order=1), dict(vertex_order=1, block_threads=1024),
                dict(vertex_order=1, pull_items_per_thread=16)):
        say("pr rmat16 %s" % cfg)
        g.set_schedule(**cfg)
        x = run_pr(g, 20)
        err = pr_max_rel(x, ref)
        assert err <= PR_RTOL, (cfg, err)
    g.close()


# ----------------------------------------------------------------------- BFS

@pytest.mark.parametrize("sched", TRAVERSAL_SCHEDULES, ids=sched_name)
def test_bfs_all_schedules(sched):
    for el, g, og in fam_graphs():
        g.set_schedule(**sched)
        for s in sources_of(el):
            say("bfs %s src=%d %s" % (el.name, s, sched))
            lv, par = run_bfs(g, s)
            ref, _ = oracle.bfs(og, s)
            assert np.array_equal(lv, ref), (el.name, s)
            assert oracle.check_bfs_parents(og, s, lv, par) == [], (el.name, s)
            st = g.stats()
            assert st.steps == int(ref.max()) + 1
    for el, g, _ in fam_graphs():
        g.set_schedule()


def by_name(name):
    return next(x for x in fam_graphs() if x[0].name == name)


def test_bfs_without_parent_and_divisors():
    el, g, og = by_name("rmat13_ef16_s23")
    for div in (1, 5, 20, 1000, 1 << 30):
        g.set_schedule(hybrid_divisor=div)
        for s in sources_of(el, 4):
            say("bfs %s src=%d div=%d" % (el.name, s, div))
            lv, _ = run_bfs(g, s, with_parent=False)
            assert np.array_equal(lv, oracle.bfs(og, s)[0])
    g.set_schedule()


def test_bfs_hybrid_switches_direction():
    """On a power-law graph the hybrid schedule must actually use both sides."""
    el, g, og = by_name("rmat13_ef16_s23")
    g.set_schedule(direction=3)
    s = sources_of(el, 1)[0]
    lv, _ = run_bfs(g, s)
    st = g.stats()
    dirs, fs, ds = st.trace()
    assert 0 < st.dense_steps < st.steps
    # the recorded choice follows the rule |F| + D_F > m/20
    for d, f, dd in zip(dirs, fs, ds):
        dense = (int(f) + int(dd)) * 20 > g.m
        assert d == (2 if dense else 0)


# ------------------------------------------------------------------------ CC

@pytest.mark.parametrize("sched", TRAVERSAL_SCHEDULES, ids=sched_name)
def test_cc_all_schedules(sched):
    for el, g, og in fam_graphs():
        say("cc %s %s" % (el.name, sched))
        g.set_schedule(**sched)
        lab = run_cc(g)
        ref, rounds = oracle.cc(og)
        assert np.array_equal(lab, ref), el.name
        assert g.stats().steps == rounds, el.name
    for el, g, _ in fam_graphs():
        g.set_schedule()


@pytest.mark.parametrize("cfg", [
    dict(num_segments=8), dict(num_segments=3, segment_strategy=1),
    dict(num_segments=8, dense_frontier=1), dict(num_segments=2, direction=2),
    dict(num_segments=64, hybrid_divisor=2), dict(num_segments=4096),
], ids=lambda c: "_".join("%s%s" % (k[:8], v) for k, v in c.items()))
def test_cc_segmented_pull(cfg):
    """The segmented CC pull (source segments, per-segment minima merged
    after the step) gives the oracle's labels and round count."""
    for el, g, og in fam_graphs():
        say("cc segmented %s %s" % (el.name, cfg))
        g.set_schedule(**cfg)
        lab = run_cc(g)
        ref, rounds = oracle.cc(og)
        assert np.array_equal(lab, ref), el.name
        assert g.stats().steps == rounds, el.name
        lab = run_cc(g)  # partial minima were reset by the merge
        assert np.array_equal(lab, ref), el.name
    for el, g, _ in fam_graphs():
        g.set_schedule()


DIRECT_CC_SCHEDULES = [dict(direction=d, dense_frontier=f) for d in range(5) for f in (0, 1)] + [
    dict(num_segments=8), dict(num_segments=3, segment_strategy=1, direction=2),
    dict(num_segments=64, hybrid_divisor=2, dense_frontier=1)]


@pytest.mark.parametrize("sched", DIRECT_CC_SCHEDULES,
                         ids=lambda c: "_".join("%s%s" % (k[:8], v) for k, v in c.items()))
def test_cc_direct_adjacency(sched):
    """CC over the CSR and CSC rows directly (no symmetric copy: push
    expands both rows of a frontier vertex, pull reduces the out-row and
    in-row blocks separately and merges them by atomic minimum) gives the
    oracle's labels and round count under every direction, frontier kind
    and segmentation."""
    gi = _gi()
    for el, g, og in fam_graphs():
        say("cc direct %s %s" % (el.name, sched))
        g.set_schedule(cc_adjacency=gi.CC_ADJ_DIRECT, **sched)
        lab = run_cc(g)
        ref, rounds = oracle.cc(og)
        assert np.array_equal(lab, ref), el.name
        assert g.stats().steps == rounds, el.name
    for el, g, _ in fam_graphs():
        g.set_schedule()


# ---------------------------------------------------------------------- SSSP

def weighted_families():
    fam = [gg.grid(40, 50, 0.01, seed=4), gg.grid(64, 64, 0.0, seed=7),
           gg.grid(200, 300, 0.01, seed=6)]
    for sc, seed in ((10, 31), (13, 32)):
        el = gg.rmat(sc, seed=seed)
        el.w = gg.uniform_weights(el.m, seed, 1, 1000)
        fam.append(el)
    el = gg.rmat(11, seed=33)
    el.w = np.ones(el.m, np.uint32)
    fam.append(el)
    el = gg.path(2000)
    el.w = gg.uniform_weights(el.m, 5, 1, 1000)
    fam.append(el)
    return fam


@pytest.mark.parametrize("delta", [1, 7, 100, 1000, 1 << 20])
def test_sssp_matches_dijkstra(delta):
    for el in weighted_families():
        g = device_graph(el)
        og = oracle.Graph(el)
        g.set_schedule(sssp_delta=delta)
        for s in sources_of(el, 2):
            say("sssp %s src=%d delta=%d" % (el.name, s, delta))
            d = run_sssp(g, s)
            ref = oracle.dijkstra(og, s)
            assert np.array_equal(d, ref), (el.name, s, delta)
        g.close()


def test_sssp_unit_weights_equal_bfs():
    el = gg.rmat(12, seed=8)
    el.w = np.ones(el.m, np.uint32)
    g = device_graph(el)
    og = oracle.Graph(el)
    s = sources_of(el, 1)[0]
    d = run_sssp(g, s)
    lv, _ = run_bfs(g, s)
    assert np.array_equal(d, np.where(lv < 0, 0xFFFFFFFF, lv).astype(np.uint32))
    g.close()


def test_sssp_overflow_reported():
    gi = _gi()
    el = gg.path(5)
    el.w = np.full(el.m, 0x7FFFFFFF, np.uint32)
    g = device_graph(el)
    with pytest.raises(gi.GiError) as e:
        run_sssp(g, 0)
    assert e.value.status == gi.GI_ERR_OVERFLOW
    g.close()


# ------------------------------------------------------ frontier primitives

@pytest.mark.parametrize("n", [1, 63, 64, 65, 1000, 100003])
def test_frontier_conversions(n):
    gi = _gi()
    torch, dev = torch_dev()
    rng = np.random.default_rng(n)
    for frac in (0.0, 0.01, 0.5, 1.0):
        say("frontier n=%d frac=%g" % (n, frac))
        members = np.nonzero(rng.random(n) < frac)[0].astype(np.int32) if frac < 1 else \
            np.arange(n, dtype=np.int32)
        ids = torch.from_numpy(rng.permutation(members).astype(np.int32)).to(dev)
        W = (n + 63) // 64
        bv = torch.full((W,), -1, dtype=torch.int64, device=dev)
        gi.sparse_to_bitvec(n, ids if members.size else 0, members.size, bv)
        bm = torch.full((n,), 7, dtype=torch.uint8, device=dev)
        gi.bitvec_to_boolmap(n, bv, bm)
        bv2 = torch.full((W,), -1, dtype=torch.int64, device=dev)
        gi.boolmap_to_bitvec(n, bm, bv2)
        out = torch.full((n,), -1, dtype=torch.int32, device=dev)
        cnt = torch.zeros((1,), dtype=torch.int32, device=dev)
        gi.bitvec_to_sparse(n, bv2, out, cnt)
        torch.cuda.synchronize()
        expect_bm = np.zeros(n, np.uint8)
        expect_bm[members] = 1
        assert np.array_equal(bm.cpu().numpy(), expect_bm)
        assert np.array_equal(bv.cpu().numpy(), bv2.cpu().numpy())
        bits = np.unpackbits(bv.cpu().numpy().view(np.uint8), bitorder="little")[:n]
        assert np.array_equal(bits, expect_bm)
        k = int(cnt.item())
        assert k == members.size
        assert np.array_equal(out.cpu().numpy()[:k], np.sort(members))


def test_frontier_degree_sum():
    torch, dev = torch_dev()
    el, g, og = by_name("rmat13_ef16_s23")
    ids = np.array(sources_of(el, 3) + [0, 1, 2], np.int32)
    out = torch.zeros((2,), dtype=torch.int64, device=dev)
    g.frontier_degree_sum(torch.from_numpy(ids).to(dev), ids.size, out)
    torch.cuda.synchronize()
    deg = og.out.degrees()
    assert out.cpu().numpy().tolist() == [ids.size, int(deg[ids].sum())]


# --------------------------------------------------------------- errors

def test_schedule_errors_and_bad_arguments():
    gi = _gi()
    el, g, og = fam_graphs()[0]
    for bad in (dict(direction=9), dict(dense_frontier=5), dict(num_segments=0),
                dict(steps_per_sync=-1), dict(hybrid_divisor=0),
                dict(block_threads=100), dict(pull_block_edges=10)):
        with pytest.raises(gi.GiError) as e:
            g.set_schedule(**bad)
        assert e.value.status == gi.GI_ERR_UNSUPPORTED, bad
    torch, dev = torch_dev()
    lv = torch.zeros((g.n,), dtype=torch.int32, device=dev)
    with pytest.raises(gi.GiError) as e:
        g.bfs(g.n, lv)
    assert e.value.status == gi.GI_ERR_INVALID_ARG
    with pytest.raises(gi.GiError) as e:
        g.sssp(0, lv)     # unweighted graph
    assert e.value.status == gi.GI_ERR_INVALID_ARG
    with pytest.raises(gi.GiError) as e:
        g.pagerank(torch.zeros((g.n,), dtype=torch.float32, device=dev), -1)
    assert e.value.status == gi.GI_ERR_INVALID_ARG
    g.set_schedule()


# ------------------------------------------------------------- step timing

def test_step_timing_covers_every_step_and_changes_nothing():
    el, g, og = by_name("rmat13_ef16_s23")
    s = sources_of(el, 1)[0]
    ref = oracle.bfs(og, s)[0]
    g.set_schedule(direction=3)
    g.set_step_timing(True)
    try:
        for rep in range(3):   # the first batch size adapts after the first run
            say("timed bfs rep %d" % rep)
            lv, par = run_bfs(g, s)
            assert np.array_equal(lv, ref)
            assert oracle.check_bfs_parents(og, s, lv, par) == []
            st = g.stats()
            step_ms, main_ms = g.step_times()
            assert len(step_ms) >= st.trace_len > 0
            assert np.all(main_ms >= 0) and np.all(step_ms >= main_ms - 1e-3)
        ranks = run_pr(g, 7)
        assert pr_max_rel(ranks, oracle.pagerank(og, 7, 0.85)) <= PR_RTOL
        step_ms, main_ms = g.step_times()
        assert len(main_ms) == 7 and np.all(main_ms > 0)
        lab = run_cc(g)
        assert np.array_equal(lab, oracle.cc(og)[0])
        assert len(g.step_times()[1]) >= g.stats().trace_len
    finally:
        g.set_step_timing(False)
        g.set_schedule()
    g.bfs(int(s), __import__("torch").empty(g.n, dtype=__import__("torch").int32, device="cuda:0"))
    assert len(g.step_times()[0]) == 0


@pytest.mark.parametrize("leaves", [100_000, 300_000])
def test_pagerank_ordered_split_rows(leaves):
    """A row split over many tiles: an in-star (every leaf points to the
    centre) plus a cycle over the leaves.  The centre's row spans leaves /
    (64 u) tiles (about 195 to 1,170 here), whose parts meet in one FP64
    slot that the split pass turns into the row's update; the slot is left
    clear for the next run."""
    import numpy as np
    gi = _gi()
    n = leaves + 1
    src = np.concatenate([np.arange(1, n), np.arange(1, n)]).astype(np.int32)
    dst = np.concatenate([np.zeros(leaves), np.roll(np.arange(1, n), 1)]).astype(np.int32)
    el = gg.EdgeList(n, src, dst)
    g = device_graph(el)
    og = oracle.Graph(el)
    ref = oracle.pagerank(og, 20, 0.85)
    for u in (4, 8):
        g.set_schedule(vertex_order=1, block_threads=256, pull_items_per_thread=u)
        say("ordered pagerank in-star leaves=%d u=%d" % (leaves, u))
        x = run_pr(g, 20)
        assert pr_max_rel(x, ref) <= PR_RTOL, u
        x = run_pr(g, 20)   # the slots were left clear for the next run
        assert pr_max_rel(x, ref) <= PR_RTOL, u
    g.set_schedule()


def test_pagerank_ordered_schedule_checks():
    """Combinations the degree-ordered pull does not offer are refused."""
    gi = _gi()
    el, g, og = fam_graphs()[8]
    bad = [dict(vertex_order=2), dict(vertex_order=1, num_segments=4),
           dict(vertex_order=1, block_threads=128), dict(vertex_order=1, pull_items_per_thread=5),
           dict(vertex_order=1, block_threads=1024, pull_items_per_thread=16),
           dict(vertex_order=1, pull_hot_sources=-2), dict(pull_hot_sources=64),
           dict(pull_items_per_thread=8)]
    for cfg in bad:
        with pytest.raises(gi.GiError) as e:
            g.set_schedule(**cfg)
        assert e.value.status == gi.GI_ERR_UNSUPPORTED, cfg
    g.set_schedule()
    x = run_pr(g, 20)
    assert pr_max_rel(x, oracle.pagerank(og, 20)) <= PR_RTOL
