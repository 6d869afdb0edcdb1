"""GPU parity of PageRank + eigenvector centrality, fused and unfused, against
the fp64 oracle: PageRank within 1e-6 relative (as gi_pagerank), eigenvector
centrality within EC_TOL of the largest entry.

EC tolerance: x is stored in FP32 (relative rounding 2^-24 per entry and
iteration) and summed in FP64; twenty iterations of a map whose output is
renormalised to unit length add at most about 20 * 2^-24 * ||x|| = 1.2e-6 of
the unit norm, so 1e-5 of the largest entry leaves an order of magnitude of
room while catching any dropped or misplaced term (each is at least 1/n of
the norm on these graphs)."""
import numpy as np
import pytest

import graphgen as gg
import oracle
from gpu_util import PR_RTOL, device_graph, pr_max_rel, say

pytestmark = pytest.mark.gpu

EC_TOL = 1e-5
_G = None


def graphs():
    global _G
    if _G is None:
        n = 5000
        # a hub whose in-row is longer than one block of the fused kernel
        hub_src = np.concatenate([np.arange(1, n, dtype=np.int32), np.zeros(n - 1, np.int32)])
        hub_dst = np.concatenate([np.zeros(n - 1, np.int32), np.arange(1, n, dtype=np.int32)])
        extra = gg.uniform(n, 3 * n, seed=61)
        hub = gg.EdgeList(n, np.concatenate([hub_src, extra.src]),
                          np.concatenate([hub_dst, extra.dst]), name="hub5000")
        els = [gg.rmat(10, seed=62), gg.rmat(14, seed=63), gg.grid(30, 41, 0.0, weighted=False),
               gg.uniform(3000, 12000, seed=64), gg.star(300), gg.star(300, out=False),
               gg.cycle(50), gg.path(200), gg.complete(40), gg.empty(9), gg.empty(1), hub]
        _G = [(el, device_graph(el), oracle.Graph(el)) for el in els]
    return _G


def run(g, iters, fused):
    import torch
    r = torch.full((g.n,), -1.0, dtype=torch.float32, device="cuda:0")
    e = torch.full((g.n,), -1.0, dtype=torch.float32, device="cuda:0")
    g.pagerank_eigenvector(r, e, iters, 0.85, fused)
    torch.cuda.synchronize()
    return r.cpu().numpy(), e.cpu().numpy()


def ec_err(x, ref):
    scale = max(float(np.max(np.abs(ref))), 1e-300)
    return float(np.max(np.abs(x.astype(np.float64) - ref))) / scale


@pytest.mark.parametrize("fused", [True, False], ids=["fused", "unfused"])
@pytest.mark.parametrize("iters", [0, 1, 3, 20])
def test_prec_matches_oracle(fused, iters):
    for el, g, og in graphs():
        say("prec %s iters=%d fused=%d" % (el.name, iters, fused))
        r, e = run(g, iters, fused)
        pr = oracle.pagerank(og, iters, 0.85)
        ec = oracle.eigenvector(og, iters)
        assert pr_max_rel(r, pr) <= PR_RTOL, el.name
        if np.all(ec == 0.0):
            assert np.all(e == 0.0), el.name
        else:
            assert ec_err(e, ec) <= EC_TOL, (el.name, ec_err(e, ec))
        assert g.stats().algorithm == 6


@pytest.mark.parametrize("iters", [0, 1, 3, 20])
def test_prec_fused_degree_ordered_matches_oracle(iters):
    """The fused pass over the degree-ordered in-adjacency (vertex_order = 1)
    returns the ranks and the eigenvector under the caller's vertex ids,
    within the same tolerances, and agrees with the id-order fused pass."""
    for el, g, og in graphs():
        say("prec ordered %s iters=%d" % (el.name, iters))
        ri, ei = run(g, iters, True)
        g.set_schedule(vertex_order=1)
        try:
            r, e = run(g, iters, True)
        finally:
            g.set_schedule(vertex_order=0)
        pr = oracle.pagerank(og, iters, 0.85)
        ec = oracle.eigenvector(og, iters)
        assert pr_max_rel(r, pr) <= PR_RTOL, el.name
        assert np.max(np.abs(r - ri) / np.maximum(np.abs(ri), 1e-30)) <= 2 * PR_RTOL, el.name
        if np.all(ec == 0.0):
            assert np.all(e == 0.0), el.name
        else:
            assert ec_err(e, ec) <= EC_TOL, (el.name, ec_err(e, ec))
            assert ec_err(e, ei.astype(np.float64)) <= EC_TOL, el.name


def test_prec_fused_equals_unfused_and_pagerank():
    """The fused pass changes the memory layout, not the values: both
    variants agree to FP32 rounding, and the PageRank part agrees with
    gi_pagerank."""
    import torch
    for el, g, og in graphs():
        say("prec fused-vs-unfused %s" % el.name)
        rf, ef = run(g, 20, True)
        ru, eu = run(g, 20, False)
        out = torch.empty(g.n, dtype=torch.float32, device="cuda:0")
        g.pagerank(out, 20, 0.85)
        torch.cuda.synchronize()
        rp = out.cpu().numpy().astype(np.float64)
        assert np.max(np.abs(rf - ru) / rp) <= 2 * PR_RTOL, el.name
        assert np.max(np.abs(rf - rp) / rp) <= 2 * PR_RTOL, el.name
        scale = max(float(np.max(np.abs(eu))), 1e-30)
        assert np.max(np.abs(ef.astype(np.float64) - eu)) <= 1e-6 * scale, el.name


def test_prec_repeated_calls_and_errors():
    """Buffers persist across calls (a shorter run after a longer one still
    starts from x_0), and bad arguments are rejected."""
    import torch
    import paper_1805_00923_amd as gi
    el, g, og = graphs()[1]
    run(g, 20, True)
    r, e = run(g, 2, True)
    assert ec_err(e, oracle.eigenvector(og, 2)) <= EC_TOL
    assert pr_max_rel(r, oracle.pagerank(og, 2, 0.85)) <= PR_RTOL
    x = torch.zeros(g.n, dtype=torch.float32, device="cuda:0")
    with pytest.raises(gi.GiError):
        g.pagerank_eigenvector(x, x.clone(), -1)
    with pytest.raises(gi.GiError):
        g.pagerank_eigenvector(x, x.clone(), 5, 1.5)
