"""GPU parity of single-source betweenness (Brandes dependencies) against
the fp64 oracle: path counts and dependencies to 1e-9 relative (FP64 atomic
sums differ from the oracle's order only by rounding), levels equal to the
BFS oracle's."""
import numpy as np
import pytest

import graphgen as gg
import oracle
from gpu_util import device_graph, say

pytestmark = pytest.mark.gpu


def hub_graph(n=6000, seed=64):
    """A vertex with n-1 in- and out-edges: longer than a pull block, so its
    in-row is summed in chunks."""
    src = np.concatenate([np.zeros(n - 1, np.int32), np.arange(1, n, dtype=np.int32)])
    dst = np.concatenate([np.arange(1, n, dtype=np.int32), np.zeros(n - 1, np.int32)])
    extra = gg.uniform(n, 3 * n, seed=seed)
    return gg.EdgeList(n, np.concatenate([src, extra.src]), np.concatenate([dst, extra.dst]),
                       name="hub%d" % n)


def fams():
    return [gg.rmat(8, seed=61), gg.rmat(12, seed=62), gg.rmat(14, seed=65),
            gg.grid(30, 41, 0.0, weighted=False), gg.uniform(3000, 9000, seed=63),
            gg.path(200), gg.star(300), gg.complete(30), gg.empty(5), hub_graph(),
            gg.from_pairs(4, [(0, 1), (0, 2), (1, 3), (2, 3)])]


@pytest.mark.parametrize("divisor", [20, 1, 100000])
def test_bc_matches_oracle(divisor):
    """Default direction rule, all-push (divisor 1) and nearly all-pull."""
    import torch
    for el in fams():
        g = device_graph(el)
        g.set_schedule(hybrid_divisor=divisor)
        og = oracle.Graph(el)
        for s in list(gg.pick_sources(el, 3, 7)) or [0]:
            say("bc %s src=%d" % (el.name, s))
            dep = torch.full((g.n,), -1.0, dtype=torch.float64, device="cuda:0")
            sig = torch.full((g.n,), -1.0, dtype=torch.float64, device="cuda:0")
            g.bc(int(s), dep, sig)
            torch.cuda.synchronize()
            d_ref, s_ref = oracle.bc(og, int(s))
            d, sg = dep.cpu().numpy(), sig.cpu().numpy()
            assert np.allclose(sg, s_ref, rtol=1e-12, atol=0), el.name
            assert np.allclose(d, d_ref, rtol=1e-9, atol=1e-9), el.name
            lv = oracle.bfs(og, int(s))[0]
            assert g.stats().steps == lv.max() + 1
            dirs, fr, ds = g.stats().trace()
            assert list(fr) == [int((lv == k).sum()) for k in range(lv.max() + 1)]
            outdeg = np.diff(og.out.off)
            assert list(ds) == [int(outdeg[lv == k].sum()) for k in range(lv.max() + 1)]
            # level 0 pushes; later levels pull by the hybrid rule
            assert dirs[0] == 0
            assert all(int(d) == (2 if (int(f) + int(dd)) * divisor > g.m else 0)
                       for d, f, dd in zip(dirs[1:], fr[1:], ds[1:])), el.name
        g.set_schedule()


def test_bc_sum_over_sources_on_a_cycle():
    """Directed n-cycle: from every source the dependency of the vertex j
    steps ahead is n-1-j; summed over all sources every vertex has
    sum_{j=1}^{n-1} (n-1-j) = (n-1)(n-2)/2."""
    import torch
    n = 40
    g = device_graph(gg.cycle(n))
    tot = torch.zeros(n, dtype=torch.float64, device="cuda:0")
    dep = torch.empty(n, dtype=torch.float64, device="cuda:0")
    for s in range(n):
        g.bc(s, dep)
        tot += dep
    assert np.allclose(tot.cpu().numpy(), (n - 1) * (n - 2) / 2)


def test_bc_bad_source():
    import torch
    import paper_1805_00923_amd as gi
    g = device_graph(gg.path(10))
    dep = torch.empty(10, dtype=torch.float64, device="cuda:0")
    with pytest.raises(gi.GiError):
        g.bc(10, dep)
