"""The batched workload's own pool, as the benchmark builds and tunes it:
256 instances (even: BFS, odd: 20-iteration PageRank) over R-MAT scales
10-18 (seeds 100 + scale) and 4-neighbour grids 64^2 ... 1024^2, BFS sources
seeded per instance (seed 200 + i), one autotuned persistent launch replayed
from a HIP graph.  Every BFS level array equals the oracle's, every
PageRank vector is within the PageRank tolerance of the FP64 oracle."""
import numpy as np
import pytest

import graphgen as gg
import oracle
from gpu_util import PR_RTOL, pr_max_rel, say

pytestmark = pytest.mark.gpu


def test_batched_pool_matches_oracle():
    import torch
    import paper_1805_00923_amd as gi
    els = [gg.rmat(s, 16, seed=100 + s) for s in range(10, 19)]
    els += [gg.grid(d, d, 0.0, weighted=False) for d in (64, 128, 256, 512, 1024)]
    graphs = [gi.Graph.from_edges(el.n, el.src, el.dst) for el in els]
    tasks = []
    for i in range(256):
        gidx = i % len(graphs)
        g, el = graphs[gidx], els[gidx]
        if i % 2 == 0:
            src = int(gg.pick_sources(el, 1, 200 + i)[0])
            tasks.append(dict(graph=gidx, algorithm=gi.ALG_BFS, src=src,
                              out=torch.full((g.n,), -7, dtype=torch.int32, device="cuda:0")))
        else:
            tasks.append(dict(graph=gidx, algorithm=gi.ALG_PAGERANK, iters=20, damping=0.85,
                              out=torch.full((g.n,), -1.0, dtype=torch.float32,
                                             device="cuda:0")))
    b = gi.Batch(graphs, tasks)
    say("pool batch autotune (256 instances)")
    b.autotune(reps=1)
    caps = b.pr_block_edges()
    say("pool batch run: %d threads, grid %d, PageRank blocks %s" %
        (b.threads(), b.info()["grid"], caps.tolist()))
    with_pr = {t["graph"] for t in tasks if t["algorithm"] == gi.ALG_PAGERANK}
    for i in range(len(graphs)):
        assert (caps[i] in (256, 512, 1024, 2048, 4096)) if i in with_pr else caps[i] == 0
    b.run(use_graph=True)
    b.run(use_graph=True)
    torch.cuda.synchronize()
    ogs = {}
    prs = {}
    for i, t in enumerate(tasks):
        gidx = t["graph"]
        if gidx not in ogs:
            say("oracle graph %s" % els[gidx].name)
            ogs[gidx] = oracle.Graph(els[gidx])
        og = ogs[gidx]
        got = t["out"].cpu().numpy()
        if t["algorithm"] == gi.ALG_BFS:
            assert np.array_equal(got, oracle.bfs(og, t["src"])[0]), (i, els[gidx].name)
        else:
            if gidx not in prs:
                prs[gidx] = oracle.pagerank(og, 20, 0.85)
            assert pr_max_rel(got, prs[gidx]) <= PR_RTOL, (i, els[gidx].name)
    b.close()
