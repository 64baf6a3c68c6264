"""Pins of the FP64 rank-network oracle: central finite differences of the
loss, closed forms for degenerate networks, the feature definition."""
import numpy as np

from oracle import mlp


def _data(m=24, seed=1):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((m, mlp.NIN))
    y = rng.uniform(0.0, 1.0, m)
    return X, y


def test_gradient_matches_central_differences():
    X, y = _data()
    w = mlp.init(seed=3)
    w[mlp.NPARAM - 1] = 0.3     # b3
    L, g = mlp.grad(w, X, y, alpha=4.0)
    assert abs(L - mlp.loss(w, X, y, 4.0)) < 1e-14
    rng = np.random.default_rng(7)
    idx = np.concatenate([rng.choice(mlp.NPARAM, 200, replace=False), [mlp.NPARAM - 1]])
    h = 1e-6
    for i in idx:
        wp, wm = w.copy(), w.copy()
        wp[i] += h
        wm[i] -= h
        fd = (mlp.loss(wp, X, y, 4.0) - mlp.loss(wm, X, y, 4.0)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])), (i, fd, g[i])


def test_degenerate_networks():
    X, y = _data(10)
    # all weights zero: out = b3 everywhere; dL/db3 = mean(2 w (b3 - y))
    w = np.zeros(mlp.NPARAM)
    w[-1] = 0.5
    out, _ = mlp.forward(w, X)
    assert np.all(out == 0.5)
    L, g = mlp.grad(w, X, y, alpha=3.0)
    d = 0.5 - y
    wt = np.where(d < 0, 3.0, 1.0)
    assert abs(L - np.mean(wt * d * d)) < 1e-15
    assert abs(g[-1] - np.mean(2 * wt * d)) < 1e-15
    assert np.all(g[:-1] == 0.0)   # every hidden unit is dead
    # alpha = 1 is the plain mean squared error
    w = mlp.init(seed=5)
    out, _ = mlp.forward(w, X)
    assert abs(mlp.loss(w, X, y, 1.0) - np.mean((out - y) ** 2)) < 1e-14


def test_linear_path_closed_form():
    # one active hidden chain: out = relu(relu(x W1 + b1) W2 + b2) W3 + b3 with
    # positive weights on a single path equals the product of the path weights
    p = mlp.unpack(np.zeros(mlp.NPARAM))
    p = {k: v.copy() for k, v in p.items()}
    p["W1"][0, 5] = 2.0
    p["W2"][5, 7] = 3.0
    p["W3"][7] = 0.25
    p["b3"][0] = 0.1
    w = mlp.pack(p)
    X = np.zeros((3, mlp.NIN))
    X[:, 0] = [1.0, 2.0, -1.0]
    out, _ = mlp.forward(w, X)
    assert np.allclose(out, [0.1 + 1.5, 0.1 + 3.0, 0.1])


def test_features():
    f = mlp.features([4.0, 0.4, 0.04, 0.0], k=5, K=20, step=250)
    assert np.allclose(f[:3], [0.0, -1.0, -2.0])
    assert f[3] == -30.0 and np.all(f[4:32] == -30.0)
    assert f[32] == 0.25 and f[33] == 0.25
    assert np.all(mlp.features([], 0, 4, 0)[:32] == -30.0)
    assert mlp.features([1.0], 1, 2, 50000)[33] == 10.0
    w = np.zeros(mlp.NPARAM)
    w[-1] = 0.37
    assert list(mlp.predict_rank(w, np.zeros((2, mlp.NIN)), 64)) == [24, 24]
