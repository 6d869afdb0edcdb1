"""GPU parity of PageRankDelta against the fp64 oracle (the GraphIt program
in SparsePush order): ranks to 1e-9 relative, the active set of every round
of the same size, under every direction; with epsilon = 0 it equals the
PageRank power iteration."""
import numpy as np
import pytest

import graphgen as gg
import oracle
from gpu_util import device_graph, say

pytestmark = pytest.mark.gpu

_G = None


def graphs():
    global _G
    if _G is None:
        els = [gg.rmat(10, seed=51), gg.rmat(13, seed=52), gg.grid(30, 41, 0.0, weighted=False),
               gg.uniform(3000, 12000, seed=53), gg.star(300), gg.cycle(50), gg.empty(9)]
        _G = [(el, device_graph(el), oracle.Graph(el)) for el in els]
    return _G


def run(g, rounds, eps):
    import torch
    x = torch.full((g.n,), -1.0, dtype=torch.float64, device="cuda:0")
    g.prdelta(x, rounds, 0.85, eps)
    torch.cuda.synchronize()
    return x.cpu().numpy()


@pytest.mark.parametrize("direction", [0, 1, 2, 3, 4])
@pytest.mark.parametrize("eps", [0.1, 0.01])
def test_prdelta_matches_oracle(direction, eps):
    for el, g, og in graphs():
        say("prdelta %s dir=%d eps=%g" % (el.name, direction, eps))
        g.set_schedule(direction=direction)
        x = run(g, 10, eps)
        ref, active = oracle.prdelta(og, 10, 0.85, eps)
        assert np.all(np.abs(x - ref) <= 1e-12 + 1e-9 * np.abs(ref)), el.name
        st = g.stats()
        fr = st.trace()[1]
        # round k+1's frontier is the active set after round k
        k = len(fr)
        assert fr[0] == g.n
        assert list(fr[1:]) == list(active[:k - 1]), el.name
        assert k == 10 or active[k - 1] == 0
    for _, g, _ in graphs():
        g.set_schedule()


def test_prdelta_eps0_is_pagerank():
    for el, g, og in graphs():
        say("prdelta eps=0 %s" % el.name)
        x = run(g, 20, 0.0)
        ref = oracle.pagerank(og, 20, 0.85)
        assert np.all(np.abs(x - ref) <= 1e-12 * np.abs(ref)), el.name


def test_prdelta_zero_rounds_and_errors():
    import torch
    import paper_1805_00923_amd as gi
    el, g, og = graphs()[0]
    assert np.all(run(g, 0, 0.1) == 0.0)
    x = torch.zeros(g.n, dtype=torch.float64, device="cuda:0")
    with pytest.raises(gi.GiError):
        g.prdelta(x, -1)
    with pytest.raises(gi.GiError):
        g.prdelta(x, 5, 1.5)
    with pytest.raises(gi.GiError):
        g.prdelta(x, 5, 0.85, -0.1)
