"""Pins of the fp64 selector-network oracle (oracle/mlp.py) to things other
than itself: central finite differences of the loss, closed forms for a
network with zero weights, the first Adam step's closed form, bfloat16
rounding of known values, and the step features of small graphs whose
frontiers are known by hand."""
import numpy as np
import pytest

import graphgen as gg
import oracle
from oracle import mlp


def rand_problem(seed, n=9, frac_valid=0.7):
    rng = np.random.default_rng(seed)
    p = rng.normal(0.0, 0.3, mlp.NPARAMS)
    mu = rng.normal(0.0, 1.0, mlp.F)
    sd = rng.uniform(0.5, 2.0, mlp.F)
    x = rng.normal(0.0, 2.0, (n, mlp.F))
    t = rng.normal(0.0, 1.0, (n, mlp.S))
    v = rng.random((n, mlp.S)) < frac_valid
    v[:, 0] = True
    return p, mu, sd, x, t, v


@pytest.mark.parametrize("seed", range(3))
def test_gradient_matches_finite_differences(seed):
    p, mu, sd, x, t, v = rand_problem(seed)
    _, g = mlp.loss_and_grad(p, mu, sd, x, t, v)
    rng = np.random.default_rng(100 + seed)
    idx = rng.choice(mlp.NPARAMS, 200, replace=False)
    # every block of the layout is probed
    idx = np.concatenate([idx, [0, 767, 768, 831, 832, 4927, 4928, 4991, 4992, 5247, 5248, 5251]])
    h = 1e-6
    for i in idx:
        e = np.zeros_like(p)
        e[i] = h
        lp, _ = mlp.loss_and_grad(p + e, mu, sd, x, t, v)
        lm, _ = mlp.loss_and_grad(p - e, mu, sd, x, t, v)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)) + 1e-8, (i, fd, g[i])


def test_zero_weights_closed_form():
    """W = 0, b1 = b2 = 0, b3 = c: y = c everywhere; L = mean over valid of
    (c - t)^2; dL/db3[s] = (2/V) sum over valid rows of (c_s - t); every other
    gradient is zero."""
    rng = np.random.default_rng(5)
    d = {name: np.zeros(shape) for name, shape in mlp.SIZES}
    c = np.array([0.5, -1.0, 2.0, 0.25])
    d["b3"] = c
    p = mlp.pack(d)
    x = rng.normal(size=(7, 12))
    t = rng.normal(size=(7, 4))
    v = rng.random((7, 4)) < 0.6
    v[0, 0] = True
    y, _ = mlp.forward(p, np.zeros(12), np.ones(12), x)
    assert np.all(y == c)
    loss, g = mlp.loss_and_grad(p, np.zeros(12), np.ones(12), x, t, v)
    V = v.sum()
    assert loss == pytest.approx(((c - t) ** 2)[v].sum() / V, rel=1e-14)
    gd = mlp.unpack(g)
    for s in range(4):
        assert gd["b3"][s] == pytest.approx(2.0 * ((c[s] - t[:, s])[v[:, s]]).sum() / V, rel=1e-13)
    for name in ("W1", "b1", "W2", "b2", "W3"):
        assert np.all(gd[name] == 0.0)


def test_clamped_input_closed_form():
    """One path through the network, W1[3,0] = W2[0,0] = 1 and W3[0,:] = 1,
    zero biases: y_s = max((clamp(x_3, lo, hi) - mu_3) / sd_3, 0).  The
    clamp applies to the raw feature, before standardisation, and leaves
    features inside the range untouched."""
    d = {name: np.zeros(shape) for name, shape in mlp.SIZES}
    d["W1"][3, 0] = 1.0
    d["W2"][0, 0] = 1.0
    d["W3"][0, :] = 1.0
    p = mlp.pack(d)
    mu = np.zeros(12)
    sd = np.ones(12)
    mu[3], sd[3] = 1.0, 2.0
    lo, hi = np.full(12, -np.inf), np.full(12, np.inf)
    lo[3], hi[3] = 2.0, 9.0
    x = np.zeros((5, 12))
    x[:, 3] = [-4.0, 2.0, 5.0, 9.0, 30.0]
    x[:, 5] = 1e6   # other features do not reach the output
    y, _ = mlp.forward(p, mu, sd, x, lo, hi)
    want = np.maximum((np.clip(x[:, 3], 2.0, 9.0) - 1.0) / 2.0, 0.0)
    assert np.array_equal(y, np.repeat(want[:, None], 4, 1))
    assert list(want) == [0.5, 0.5, 2.0, 4.0, 4.0]
    # no range: the plain network
    y0, _ = mlp.forward(p, mu, sd, x)
    assert list(y0[:, 0]) == [0.0, 0.5, 2.0, 4.0, 14.5]


def test_first_adam_step_is_lr_times_sign():
    """After one step from zero moments, bias correction gives m_hat = g and
    v_hat = g^2, so the update is lr * g / (|g| + eps)."""
    g = np.array([3.0, -0.25, 1e-3, -7.5, 0.0])
    p = np.zeros(5)
    p1, m, v = mlp.adam_step(p, g, np.zeros(5), np.zeros(5), 1, lr=0.01, eps=1e-8)
    assert np.allclose(p1, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=0)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_bf16_rounding_known_values():
    vals = np.array([1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, -2.5, 1 + 2 ** -7, 3.0 + 2 ** -9],
                    np.float32)
    want = [1.0, 1.0, 1 + 2 ** -6, -2.5, 1 + 2 ** -7, 3.0]
    assert list(mlp.bf16_round(vals)) == want


def test_bfs_features_on_a_path():
    """Path 0 -> 1 -> ... -> 9 from 0: one vertex per level, out-degree 1
    except the last."""
    el = gg.path(10)
    g = oracle.Graph(el)
    lv, _ = oracle.bfs(g, 0)
    f = mlp.bfs_step_features(g, lv)
    assert f.shape == (10, 12)
    n, m = 10, 9
    deg = np.array([1] * 9 + [0], float)
    for k in range(10):
        assert f[k, 0] == pytest.approx(np.log2(10)) and f[k, 1] == pytest.approx(np.log2(9))
        assert f[k, 2] == pytest.approx(0.9) and f[k, 3] == pytest.approx(1.0)
        assert f[k, 4] == pytest.approx(deg.std() / deg.mean())
        assert f[k, 5] == pytest.approx(0.1)
        assert f[k, 6] == pytest.approx((1.0 if k < 9 else 0.0) / 9)
        assert f[k, 7] == pytest.approx(1.0 - (k + 1) / 10)
        assert f[k, 8] == pytest.approx(1.0)
        assert f[k, 10] == pytest.approx(1.0) and f[k, 11] == 0.0


@pytest.mark.parametrize("el", [gg.rmat(9, seed=3), gg.grid(12, 17, 0.0, weighted=False),
                                gg.uniform(300, 500, seed=2), gg.path(40)],
                         ids=["rmat9", "grid", "uniform", "path"])
def test_cc_frontiers_match_the_label_propagation_oracle(el):
    """The round frontiers replayed here end in the oracle's labels and have
    its round count."""
    g = oracle.Graph(el)
    fr = mlp.cc_frontiers(g)
    lab, rounds = oracle.cc(g)
    assert len(fr) == rounds
    assert fr[0].all()
    f = mlp.cc_step_features(g, fr)
    assert f.shape == (rounds, 12)
    assert np.all(f[:, 11] == 0.5)
