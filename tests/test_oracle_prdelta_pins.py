"""Pins of the oracle's PageRankDelta filter (epsilon > 0) and of the CC
selector features, each checked against planted mistakes.

PageRankDelta is the GraphIt program of section 3 (the running example of
sections 2 and 3): Rank starts at 0 and Delta at 1/n; every round the active
vertices push Delta/OutDegree along their out-edges into DeltaSum; each
vertex then sets Delta = alpha*DeltaSum (plus (1-alpha)/n in the first
round, after which 1/n is taken off again), adds Delta to Rank, and stays
active when |Delta| > epsilon*Rank, Rank being the value after the update.

The pins:
- an exact rational (Fraction) run of that program on every directed graph
  with at most 3 vertices, for several epsilon, against the oracle's ranks
  and per-round active counts;
- closed forms: a directed cycle is inactive after round 1 with Rank = 1/n
  for any epsilon > 0; a star whose centre has a negative Delta (so the
  absolute value decides) reaches PageRank's second iterate; an edgeless
  graph whose Delta equals epsilon*Rank exactly stays inactive; a large
  epsilon that only the updated Rank can meet.
The CC features (one row per synchronous label-propagation round) are
pinned by hand on a path and a star.

Each planted mistake (no absolute value, >= in place of >, the Rank before
the update, the first round's 1/n not taken off, for CC features E = m in
place of 2m or out-degrees only) is compiled or executed here, on the CPU,
and must fail at least one pin.
"""
import ctypes
import inspect
import os
import subprocess
from fractions import Fraction

import numpy as np
import pytest

import graphgen as gg
import oracle
from oracle import mlp

ALPHA = 0.85
EPS_LIST = (0.0, 0.01, 0.1, 0.5, 2.0, 10.0)
ROUNDS = 6


# ------------------------------------------------- PageRankDelta, exact ----

def all_graphs(n):
    pairs = [(u, v) for u in range(n) for v in range(n) if u != v]
    for mask in range(1 << len(pairs)):
        yield [pairs[i] for i in range(len(pairs)) if mask >> i & 1]


def exact_prdelta(n, edges, rounds, alpha, eps):
    """The section 3 program in exact rational arithmetic.  alpha and eps
    are taken at the exact value of the doubles the oracle receives.
    Returns ranks, active counts and, per round, whether some vertex sat
    within 1e-9 (relative) of the threshold (a decision that rounding could
    flip)."""
    a = Fraction(alpha)
    ep = Fraction(eps)
    inv_n = Fraction(1, n)
    outdeg = [0] * n
    for u, _ in edges:
        outdeg[u] += 1
    rank = [Fraction(0)] * n
    delta = [inv_n] * n
    active = [True] * n
    counts, near = [], []
    for r in range(1, rounds + 1):
        dsum = [Fraction(0)] * n
        for u, v in edges:
            if active[u]:
                dsum[v] += delta[u] / outdeg[u]
        close = False
        for v in range(n):
            delta[v] = a * dsum[v] + ((1 - a) * inv_n if r == 1 else 0)
            rank[v] += delta[v]
            if r == 1:
                delta[v] -= inv_n
            gap = abs(delta[v]) - ep * rank[v]
            if eps > 0 and abs(gap) <= Fraction(1, 10 ** 9) * rank[v]:
                close = True
            active[v] = abs(delta[v]) > ep * rank[v]
        counts.append(sum(active))
        near.append(close)
    return [float(x) for x in rank], counts, near


def run_oracle_prdelta(fn, el, rounds, alpha, eps):
    g = oracle.Graph(el)
    rank = np.empty(g.n, np.float64)
    active = np.empty(rounds, np.int64)
    rc = fn(g.n, g.out.off.ctypes.data, g.out.idx.ctypes.data, rounds, alpha, eps,
            rank.ctypes.data, active.ctypes.data)
    assert rc == 0
    return rank, active


def prdelta_pin_failures(fn):
    """Every PageRankDelta pin against the or_prdelta entry point fn;
    returns the list of failures (empty when all hold)."""
    bad = []
    # exhaustive, exact
    for n in (1, 2, 3):
        for edges in all_graphs(n):
            el = gg.from_pairs(n, edges) if edges else gg.empty(n)
            for eps in EPS_LIST:
                xr, xc, near = exact_prdelta(n, edges, ROUNDS, ALPHA, eps)
                r, c = run_oracle_prdelta(fn, el, ROUNDS, ALPHA, eps)
                if not np.allclose(r, xr, rtol=1e-12, atol=0):
                    bad.append("ranks n=%d %s eps=%g" % (n, edges, eps))
                    continue
                if eps > 0:
                    for k in range(ROUNDS):
                        if near[k]:
                            break
                        if c[k] != xc[k]:
                            bad.append("active n=%d %s eps=%g round %d: %d != %d"
                                       % (n, edges, eps, k + 1, c[k], xc[k]))
                            break
    # directed cycle: Delta is 0 after round 1, Rank = 1/n, nothing active
    for n in (3, 7, 64):
        for eps in (0.01, 0.1, 1.0):
            r, c = run_oracle_prdelta(fn, gg.cycle(n), 4, ALPHA, eps)
            if not (np.allclose(r, 1.0 / n, rtol=1e-14) and list(c) == [0, 0, 0, 0]):
                bad.append("cycle n=%d eps=%g: active %s" % (n, eps, list(c)))
    # out-star (centre 0 -> leaves): the centre has no in-edges, so its
    # Delta after round 1 is -alpha/n and only |Delta| keeps it active; its
    # round-2 push then gives the leaves PageRank's second iterate
    # (1-a)/n + a (1-a)/(n (n-1)), the centre keeps (1-a)/n.
    for n in (4, 6, 11):
        r, c = run_oracle_prdelta(fn, gg.star(n), 2, ALPHA, 0.1)
        leaf = (1 - ALPHA) / n + ALPHA * (1 - ALPHA) / (n * (n - 1))
        if c[0] != n:
            bad.append("star n=%d: %d active after round 1, expected %d" % (n, c[0], n))
        if not (abs(r[0] - (1 - ALPHA) / n) < 1e-16 and np.allclose(r[1:], leaf, rtol=1e-13)):
            bad.append("star n=%d: ranks after round 2 are not PageRank's second iterate" % n)
    # edgeless, alpha = 1/2, n = 4, eps = 1: after round 1 Delta = -1/8 and
    # Rank = 1/8 exactly (powers of two), |Delta| = eps*Rank, which is not
    # above the threshold: no vertex stays active
    r, c = run_oracle_prdelta(fn, gg.empty(4), 1, 0.5, 1.0)
    if not (np.all(r == 0.125) and c[0] == 0):
        bad.append("tie: %d active at |Delta| == eps*Rank" % c[0])
    # edgeless, eps = 10: |Delta| = a/n against 10 (1-a)/n after the update
    # (not active), but against 0 before it (active)
    r, c = run_oracle_prdelta(fn, gg.empty(5), 1, ALPHA, 10.0)
    if c[0] != 0:
        bad.append("eps=10 edgeless: %d active, the threshold must use the updated Rank" % c[0])
    return bad


def _bind(lib):
    f = lib.or_prdelta
    vp = ctypes.c_void_p
    f.restype = ctypes.c_int
    f.argtypes = [ctypes.c_int32, vp, vp, ctypes.c_int32, ctypes.c_double, ctypes.c_double, vp, vp]
    return f


def test_prdelta_pins_hold():
    oracle.build(force=False)
    bad = prdelta_pin_failures(_bind(ctypes.CDLL(oracle._LIB)))
    assert bad == []


def test_prdelta_exhaustive_has_no_near_ties():
    """The exhaustive comparison checks every decision: no vertex of the
    enumerated graphs sits within rounding distance of the threshold."""
    skipped = 0
    for n in (1, 2, 3):
        for edges in all_graphs(n):
            for eps in EPS_LIST[1:]:
                skipped += any(exact_prdelta(n, edges, ROUNDS, ALPHA, eps)[2])
    assert skipped == 0


# Planted mistakes: (what, text in oracle.c, replacement).  Each is applied
# to a copy of the oracle source, compiled, and must fail a pin.
MUTANTS = [
    ("no absolute value", "double ad = delta[v] < 0 ? -delta[v] : delta[v];",
     "double ad = delta[v];"),
    (">= in place of >", "in_f[v] = ad > eps * rank[v];", "in_f[v] = ad >= eps * rank[v];"),
    ("Rank before the update",
     "in_f[v] = ad > eps * rank[v];",
     "in_f[v] = ad > eps * (rank[v] - delta[v] - (round == 1 ? inv_n : 0.0));"),
    ("first round keeps 1/n", "        delta[v] -= inv_n;\n", "\n"),
]


@pytest.mark.parametrize("what,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_prdelta_planted_mistake_fails_a_pin(tmp_path, what, old, new):
    src = open(os.path.join(os.path.dirname(oracle.__file__), "oracle.c")).read()
    assert src.count(old) == 1, "mutation site not found: %s" % what
    mpath = tmp_path / "oracle_mut.c"
    mpath.write_text(src.replace(old, new))
    so = tmp_path / "liboracle_mut.so"
    subprocess.check_call(["gcc", "-O2", "-shared", "-fPIC", "-std=c11", "-o", str(so), str(mpath),
                           "-lm"])
    bad = prdelta_pin_failures(_bind(ctypes.CDLL(str(so))))
    assert bad, "planted mistake '%s' passed every pin" % what


# ------------------------------------------------------ CC features -------

def cc_feature_pin_failures(features):
    """Hand-computed CC round features on a path and a star; features is
    mlp.cc_step_features or a planted variant."""
    bad = []
    # path 0 -> 1 -> ... -> n-1: degrees (out + in) are 1, 2, ..., 2, 1;
    # E = 2(n-1).  After round k every label is max(0, v - k), so round k
    # meets F_k = {k, ..., n-1}: |F_k| = n - k, degree sum 2(n-1) for k = 0
    # and 2(n-k) - 1 after.
    n = 9
    g = oracle.Graph(gg.path(n))
    fr = mlp.cc_frontiers(g)
    if len(fr) != n or any(set(np.nonzero(f)[0]) != set(range(k, n)) for k, f in enumerate(fr)):
        return ["path frontiers"]
    f = features(g, fr)
    deg = np.array([1] + [2] * (n - 2) + [1], float)
    E = 2 * (n - 1)
    for k in range(n):
        nf = n - k
        d = E if k == 0 else 2 * (n - k) - 1
        prev = n - k + 1 if k > 0 else 0
        want = [np.log2(n), np.log2(E), E / n, np.log2(3.0), deg.std() / deg.mean(),
                nf / n, d / E, d / E, np.log2(1 + nf), np.log2(1 + d),
                min(64.0, nf / max(prev, 1)), 0.5]
        if not np.allclose(f[k], want, rtol=1e-12, atol=1e-15):
            bad.append("path round %d: %s != %s" % (k, list(f[k]), want))
    # out-star centre 0 -> n-1 leaves: degrees n-1 and 1, E = 2(n-1); round
    # 0 meets V, round 1 the leaves (their label drops to 0), then nothing.
    n = 7
    g = oracle.Graph(gg.star(n))
    fr = mlp.cc_frontiers(g)
    if len(fr) != 2:
        return bad + ["star rounds"]
    f = features(g, fr)
    deg = np.array([n - 1] + [1] * (n - 1), float)
    E = 2 * (n - 1)
    rows = [(n, E, 0), (n - 1, n - 1, n)]
    for k, (nf, d, prev) in enumerate(rows):
        want = [np.log2(n), np.log2(E), E / n, np.log2(n), deg.std() / deg.mean(),
                nf / n, d / E, d / E, np.log2(1 + nf), np.log2(1 + d),
                min(64.0, nf / max(prev, 1)), 0.5]
        if not np.allclose(f[k], want, rtol=1e-12, atol=1e-15):
            bad.append("star round %d: %s != %s" % (k, list(f[k]), want))
    return bad


def test_cc_features_by_hand():
    assert cc_feature_pin_failures(mlp.cc_step_features) == []


CC_MUTANTS = [
    ("E = m", "n, e = g.n, 2 * g.m", "n, e = g.n, g.m"),
    ("out-degree only", "deg = (np.diff(g.out.off) + np.diff(g.inc.off))", "deg = (np.diff(g.out.off))"),
    ("ratio to the current frontier", "min(64.0, nf / max(prev, 1))", "min(64.0, prev / max(nf, 1))"),
]


@pytest.mark.parametrize("what,old,new", CC_MUTANTS, ids=[m[0] for m in CC_MUTANTS])
def test_cc_features_planted_mistake_fails(what, old, new):
    src = inspect.getsource(mlp.cc_step_features)
    assert src.count(old) == 1, "mutation site not found: %s" % what
    ns = dict(vars(mlp))
    exec(compile(src.replace(old, new), "<mutant>", "exec"), ns)
    assert cc_feature_pin_failures(ns["cc_step_features"]), \
        "planted mistake '%s' passed the CC feature pins" % what
