"""The seeded input generators against their recipes (CPU only): R-MAT
quadrant frequencies at every recursion level and the id permutation being
a relabelling; the grid's records, symmetric weights and shortcut count;
the Chung-Lu weight sequence (largest weight, total, power-law ratios) and
sampled degrees that follow it; determinism per seed; source picking."""
import numpy as np
import pytest

import graphgen as gg


def test_rmat_quadrant_frequencies_at_every_level():
    scale, ns = 8, 200_000
    el = gg.rmat(scale, nsamples=ns, seed=11, permute=False)
    a, b, c = gg.RMAT_ABC
    want = {(0, 0): a, (0, 1): b, (1, 0): c, (1, 1): 1.0 - a - b - c}
    for level in range(scale):
        bit = 1 << (scale - 1 - level)
        sb = (el.src & bit) != 0
        db = (el.dst & bit) != 0
        for (s, d), p in want.items():
            frac = float(np.mean((sb == bool(s)) & (db == bool(d))))
            # binomial standard deviation at most 0.0011; 5 of them
            assert abs(frac - p) < 0.0056, (level, s, d, frac, p)


def test_rmat_permutation_is_a_relabelling():
    plain = gg.rmat(10, seed=7, permute=False)
    perm = gg.rmat(10, seed=7, permute=True)
    n = plain.n
    mapping = np.full(n, -1, np.int64)
    for x, y in ((plain.src, perm.src), (plain.dst, perm.dst)):
        for u, v in zip(x.tolist(), y.tolist()):
            assert mapping[u] in (-1, v)
            mapping[u] = v
    used = mapping[mapping >= 0]
    assert len(np.unique(used)) == len(used)          # injective
    assert not np.array_equal(plain.src, perm.src)     # and not the identity


def test_generators_are_deterministic_per_seed():
    a = gg.rmat(9, seed=3)
    b = gg.rmat(9, seed=3)
    c = gg.rmat(9, seed=4)
    assert np.array_equal(a.src, b.src) and np.array_equal(a.dst, b.dst)
    assert not np.array_equal(a.src, c.src)
    g1 = gg.grid(20, 30, 0.05, seed=9)
    g2 = gg.grid(20, 30, 0.05, seed=9)
    assert np.array_equal(g1.src, g2.src) and np.array_equal(g1.w, g2.w)
    l1 = gg.chung_lu(3000, 20000, 2.2, 200.0, seed=5)
    l2 = gg.chung_lu(3000, 20000, 2.2, 200.0, seed=5)
    assert np.array_equal(l1.src, l2.src) and np.array_equal(l1.dst, l2.dst)


def test_grid_records_and_symmetric_weights():
    r, c = 5, 7
    el = gg.grid(r, c, 0.0, seed=4)
    assert el.m == 2 * (2 * r * c - r - c)
    w = {}
    for u, v, x in zip(el.src.tolist(), el.dst.tolist(), el.w.tolist()):
        (ru, cu), (rv, cv) = divmod(u, c), divmod(v, c)
        assert abs(ru - rv) + abs(cu - cv) == 1
        assert 1 <= x <= 1000
        w[(u, v)] = x
    for (u, v), x in w.items():
        assert w[(v, u)] == x
    assert len(w) == el.m


def test_grid_shortcut_count():
    r = c = 64
    el = gg.grid(r, c, 0.01, seed=4)
    nshort = int(np.floor(0.01 * r * c))
    assert el.m == 2 * (2 * r * c - r - c) + 2 * nshort
    far = [(u, v) for u, v in zip(el.src.tolist(), el.dst.tolist())
           if abs(u // c - v // c) + abs(u % c - v % c) != 1]
    assert all(u != v for u, v in far)
    assert len(far) <= 2 * nshort


def test_chunglu_weight_sequence():
    n, gamma, dmax, wsum = 10_000, 2.5, 500.0, 200_000.0
    w, i0 = gg.chunglu_weights(n, gamma, dmax, wsum)
    beta = 1.0 / (gamma - 1.0)
    assert w[0] == pytest.approx(dmax, rel=1e-9)
    assert w.sum() == pytest.approx(wsum, rel=1e-6)
    assert np.all(np.diff(w) < 0)
    for i, j in ((0, 10), (5, 500), (100, 9999)):
        assert w[i] / w[j] == pytest.approx(((j + i0) / (i + i0)) ** beta, rel=1e-12)


def test_chunglu_degrees_follow_the_weights():
    n, ns, gamma, dmax = 2000, 400_000, 2.5, 300.0
    el = gg.chung_lu(n, ns, gamma, dmax, seed=21)
    w, _ = gg.chunglu_weights(n, gamma, dmax, float(ns))
    expect = np.sort(w / w.sum() * ns)[::-1]
    got = np.sort(np.bincount(el.src, minlength=n))[::-1]
    # the largest degrees: Poisson counts around their expectations
    for k in range(5):
        assert abs(got[k] - expect[k]) < 6.0 * np.sqrt(expect[k]) + 10, (k, got[k], expect[k])
    # and the whole sorted sequence
    assert np.abs(got - expect).sum() / ns < 0.05


def test_pick_sources_distinct_with_out_records():
    el = gg.rmat(10, seed=2)
    s = gg.pick_sources(el, 64, 3)
    assert len(s) == 64 and len(np.unique(s)) == 64
    has_out = np.zeros(el.n, bool)
    has_out[el.src[el.src != el.dst]] = True
    assert np.all(has_out[s])
    assert np.array_equal(s, gg.pick_sources(el, 64, 3))
