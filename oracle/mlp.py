"""ORACLE -- test infrastructure only.

Plain fp64 reference of the schedule selector network: a multilayer
perceptron 12 -> 64 -> 64 -> 4 with ReLU, trained by mean squared error on
log step time over the valid schedules, with Adam (Kingma and Ba, "Adam: A
Method for Stochastic Optimization", ICLR 2015, Algorithm 1 with bias
correction).  The forward pass is three matrix products; the backward pass
is the chain rule written out layer by layer.  Pinned by finite differences
and closed forms in tests/test_oracle_mlp_pins.py.

Parameter vector layout (row-major): W1[12][64] b1[64] W2[64][64] b2[64]
W3[64][4] b3[4].  Features are standardised, (x - mu) / sd, before W1; at
inference they may first be clamped to the training records' range.
Also: the per-step selector features of BFS and CC, recomputed from the
oracle's own traversal.
"""
import numpy as np

F, H, S = 12, 64, 4
SIZES = [("W1", (F, H)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("W3", (H, S)), ("b3", (S,))]
NPARAMS = sum(int(np.prod(s)) for _, s in SIZES)


def unpack(p):
    p = np.asarray(p, np.float64)
    out, o = {}, 0
    for name, shape in SIZES:
        k = int(np.prod(shape))
        out[name] = p[o:o + k].reshape(shape)
        o += k
    return out


def pack(d):
    return np.concatenate([np.asarray(d[name], np.float64).ravel() for name, _ in SIZES])


def forward(p, mu, sd, x, lo=None, hi=None):
    """Predicted log-times [N, 4] and the intermediate activations.  With
    lo/hi given, each raw feature is first clamped to [lo, hi] (the range
    of the training records), so that inputs outside it are read as its
    nearest edge instead of being extrapolated."""
    w = unpack(p)
    x = np.asarray(x, np.float64)
    if lo is not None:
        x = np.maximum(x, np.asarray(lo, np.float64))
    if hi is not None:
        x = np.minimum(x, np.asarray(hi, np.float64))
    xn = (x - np.asarray(mu, np.float64)) / np.asarray(sd, np.float64)
    z1 = xn @ w["W1"] + w["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ w["W2"] + w["b2"]
    h2 = np.maximum(z2, 0.0)
    y = h2 @ w["W3"] + w["b3"]
    return y, (xn, z1, h1, z2, h2)


def loss_and_grad(p, mu, sd, x, t, valid):
    """L = (1/V) sum over valid (record, schedule) of (y - t)^2, V = number of
    valid pairs; returns (L, dL/dp)."""
    w = unpack(p)
    y, (xn, z1, h1, z2, h2) = forward(p, mu, sd, x)
    v = np.asarray(valid, bool)
    nv = int(v.sum())
    diff = np.where(v, y - np.asarray(t, np.float64), 0.0)
    loss = float((diff ** 2).sum() / nv)
    dy = 2.0 * diff / nv
    g = {}
    g["W3"] = h2.T @ dy
    g["b3"] = dy.sum(0)
    dz2 = (dy @ w["W3"].T) * (z2 > 0)
    g["W2"] = h1.T @ dz2
    g["b2"] = dz2.sum(0)
    dz1 = (dz2 @ w["W2"].T) * (z1 > 0)
    g["W1"] = xn.T @ dz1
    g["b1"] = dz1.sum(0)
    return loss, pack(g)


def adam_step(p, g, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update at step t (1-based); returns (p, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def bf16_round(a):
    """Round float32 values to bfloat16 (nearest, ties to even), returned as
    float64."""
    u = np.asarray(a, np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (u.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def graph_features(deg, n, edges, alg):
    """Graph-level features: log2 n, log2 E, E/n, log2(1 + max degree),
    coefficient of variation of the degrees, algorithm id."""
    deg = np.asarray(deg, np.float64)
    mean = deg.mean()
    cv = deg.std() / mean if mean > 0 else 0.0
    return [np.log2(n), np.log2(max(edges, 1)), edges / n, np.log2(1 + deg.max()), cv, alg]


def bfs_step_features(g, level):
    """Features of each BFS step from the oracle's levels: step k meets
    F_k = {v : level v = k}."""
    outdeg = np.diff(g.out.off).astype(np.int64)
    n, m = g.n, g.m
    gf = graph_features(outdeg, n, m, 0.0)
    rows, visited, prev = [], 0, 0
    for k in range(int(level.max()) + 1):
        f = level == k
        nf = int(f.sum())
        d = int(outdeg[f].sum())
        visited += nf
        rows.append(gf[:5] + [nf / n, d / m, 1.0 - visited / n, np.log2(1 + nf), np.log2(1 + d),
                              min(64.0, nf / max(prev, 1)), gf[5]])
        prev = nf
    return np.array(rows)


def cc_step_features(g, frontiers):
    """Features of each CC round from the frontiers of the synchronous label
    propagation (list of boolean vertex masks)."""
    deg = (np.diff(g.out.off) + np.diff(g.inc.off)).astype(np.int64)
    n, e = g.n, 2 * g.m
    gf = graph_features(deg, n, e, 0.5)
    rows, prev = [], 0
    for f in frontiers:
        nf = int(f.sum())
        d = int(deg[f].sum())
        rows.append(gf[:5] + [nf / n, d / max(e, 1), d / max(e, 1), np.log2(1 + nf),
                              np.log2(1 + d), min(64.0, nf / max(prev, 1)), gf[5]])
        prev = nf
    return np.array(rows)


def cc_frontiers(g):
    """Frontier of every round of synchronous label propagation (edges both
    ways), F_0 = V, up to the last non-empty one."""
    n = g.n
    src = np.repeat(np.arange(n), np.diff(g.out.off))
    dst = g.out.idx.astype(np.int64)
    a = np.concatenate([src, dst])
    b = np.concatenate([dst, src])
    lab = np.arange(n, dtype=np.int64)
    f = np.ones(n, bool)
    out = []
    while f.any():
        out.append(f.copy())
        act = f[a] | f[b]
        new = lab.copy()
        np.minimum.at(new, b[act], lab[a[act]])
        f = new < lab
        lab = new
    return out
