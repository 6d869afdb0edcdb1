"""Connected components on the selector's held-out graph at full size
(Chung-Lu, degree exponent 2.0, 41,000,000 vertices, 1.5 billion samples,
about 1.32 billion edges, 2m beyond 32-bit offsets: the direct form), checked
once against the oracle's union-find over the raw records.  Opt-in, as it
spends minutes of host time on generation, ingest and the oracle:
GI_HELDOUT_FULL=1."""
import os
import time

import numpy as np
import pytest

import graphgen as gg
import oracle
from gpu_util import say

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(os.environ.get("GI_HELDOUT_FULL") != "1",
                                 reason="opt-in (GI_HELDOUT_FULL=1): minutes of host work")]


def test_heldout_full_cc_matches_union_find():
    import torch
    import paper_1805_00923_amd as gi
    t0 = time.time()
    el = gg.chung_lu(41_000_000, 1_500_000_000, 2.0, 1e6, seed=999)
    say("held-out records generated in %.0fs" % (time.time() - t0))
    off, idx, _ = gi.build_adjacency(el.n, el.src, el.dst)
    ioff, iidx, _ = gi.build_adjacency(el.n, el.dst, el.src)
    g = gi.Graph(el.n, off, idx, None, ioff, iidx, None)
    del off, idx, ioff, iidx
    say("held-out graph n=%d m=%d built in %.0fs" % (g.n, g.m, time.time() - t0))
    assert 2 * g.m > 2**31 - 1
    lab = torch.empty(g.n, dtype=torch.int32, device="cuda:0")
    g.cc(lab)
    torch.cuda.synchronize()
    say("device cc: %d rounds, %.1f ms" % (g.stats().steps, g.stats().kernel_ms))
    got = lab.cpu().numpy()
    g.close()
    t1 = time.time()
    ref, comps = oracle.cc_union_find(el.n, el.src, el.dst)
    say("oracle union-find: %d components in %.0fs" % (comps, time.time() - t1))
    assert np.array_equal(got, ref)
