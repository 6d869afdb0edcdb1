"""Helpers for the GPU parity tests: device graphs built through the library's
own ingest, device output buffers, and the comparison rules.

PageRank tolerance: max_v |x_gpu - x| / x <= 1e-6 against the FP64 oracle
(x >= (1-alpha)/n > 0 so the ratio is defined).  BFS levels, CC labels and
SSSP distances are integers and must match exactly; BFS parents are checked
for validity, since several BFS trees are correct.
"""
import sys

import numpy as np

PR_RTOL = 1e-6


def torch_dev():
    import torch
    return torch, torch.device("cuda:0")


def say(msg):
    print("[case] " + msg, flush=True)
    sys.stdout.flush()


def device_graph(el):
    import paper_1805_00923_amd as gi
    return gi.Graph.from_edges(el.n, el.src, el.dst, el.w)


def run_pr(g, iters=20, alpha=0.85):
    torch, dev = torch_dev()
    out = torch.full((g.n,), -1.0, dtype=torch.float32, device=dev)
    g.pagerank(out, iters, alpha)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def run_bfs(g, s, with_parent=True):
    torch, dev = torch_dev()
    level = torch.full((g.n,), -7, dtype=torch.int32, device=dev)
    parent = torch.full((g.n,), -7, dtype=torch.int32, device=dev) if with_parent else None
    g.bfs(int(s), level, parent)
    torch.cuda.synchronize()
    return level.cpu().numpy(), (parent.cpu().numpy() if with_parent else None)


def run_cc(g):
    torch, dev = torch_dev()
    lab = torch.full((g.n,), -7, dtype=torch.int32, device=dev)
    g.cc(lab)
    torch.cuda.synchronize()
    return lab.cpu().numpy()


def run_sssp(g, s):
    torch, dev = torch_dev()
    dist = torch.zeros((g.n,), dtype=torch.int32, device=dev)
    g.sssp(int(s), dist)
    torch.cuda.synchronize()
    return dist.cpu().numpy().view(np.uint32)


def pr_max_rel(x_gpu, x_ref):
    return float(np.max(np.abs(x_gpu.astype(np.float64) - x_ref) / x_ref))
