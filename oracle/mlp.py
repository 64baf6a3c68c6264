"""Truncation-rank network, plainly, in FP64.  TEST INFRASTRUCTURE.

A three-layer perceptron maps a bond's singular-value features to the rank
the truncation rule of Sec. 4.3 keeps (discard sigma_i < eps sigma_max, cap at
chi_max).  Features of bond k in rounding j at step t (34 values):

    f_i  = log10(sigma_i / sigma_1), i = 1..32, the leading singular values of
           the same bond and rounding at step t-1 (-30 where absent or zero);
    f_33 = k / K;   f_34 = min(t, 10^4) / 1000.

Network: h1 = relu(x W1 + b1) (128), h2 = relu(h1 W2 + b2) (128),
out = h2 W3 + b3, read as rank / chi_max.  Loss: mean of w (out - y)^2 with
w = alpha where out < y (an under-predicted rank costs an exact fallback) and
w = 1 otherwise.  Parameters are one flat vector in the order W1 (34 x 128,
row-major, input by output), b1, W2 (128 x 128), b2, W3 (128), b3.
"""
import numpy as np

NIN, NH = 34, 128
SHAPES = [("W1", (NIN, NH)), ("b1", (NH,)), ("W2", (NH, NH)), ("b2", (NH,)), ("W3", (NH,)), ("b3", (1,))]
NPARAM = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(w):
    w = np.asarray(w, dtype=np.float64)
    assert w.size == NPARAM
    out, o = {}, 0
    for name, shape in SHAPES:
        sz = int(np.prod(shape))
        out[name] = w[o:o + sz].reshape(shape)
        o += sz
    return out


def pack(p):
    return np.concatenate([np.ravel(p[name]) for name, _ in SHAPES])


def init(seed=0):
    """He-scaled normal weights, zero biases."""
    rng = np.random.default_rng(seed)
    p = {"W1": rng.standard_normal((NIN, NH)) * np.sqrt(2.0 / NIN), "b1": np.zeros(NH),
         "W2": rng.standard_normal((NH, NH)) * np.sqrt(2.0 / NH), "b2": np.zeros(NH),
         "W3": rng.standard_normal(NH) * np.sqrt(1.0 / NH), "b3": np.zeros(1)}
    return pack(p)


def features(sigma, k, K, step):
    """The 34 inputs of one bond (sigma: leading singular values, any length)."""
    f = np.full(NIN, -30.0)
    s = np.asarray(sigma, dtype=np.float64)[:32]
    if s.size and s[0] > 0:
        with np.errstate(divide="ignore"):
            v = np.log10(s / s[0])
        v[~np.isfinite(v)] = -30.0
        f[:s.size] = np.maximum(v, -30.0)
    f[32] = k / K
    f[33] = min(step, 10000) / 1000.0
    return f


def forward(w, X):
    p = unpack(w)
    X = np.asarray(X, dtype=np.float64)
    z1 = X @ p["W1"] + p["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ p["W2"] + p["b2"]
    h2 = np.maximum(z2, 0.0)
    out = h2 @ p["W3"] + p["b3"][0]
    return out, (X, z1, h1, z2, h2)


def loss(w, X, y, alpha):
    out, _ = forward(w, X)
    d = out - np.asarray(y, dtype=np.float64)
    wt = np.where(d < 0.0, alpha, 1.0)
    return float(np.mean(wt * d * d))


def grad(w, X, y, alpha):
    """Loss and its gradient (flat, same order as the parameters), by the chain rule."""
    p = unpack(w)
    out, (X, z1, h1, z2, h2) = forward(w, X)
    m = X.shape[0]
    d = out - np.asarray(y, dtype=np.float64)
    wt = np.where(d < 0.0, alpha, 1.0)
    L = float(np.mean(wt * d * d))
    dout = 2.0 * wt * d / m
    g = {"W3": h2.T @ dout, "b3": np.array([dout.sum()])}
    dz2 = np.outer(dout, p["W3"]) * (z2 > 0.0)
    g["W2"] = h1.T @ dz2
    g["b2"] = dz2.sum(axis=0)
    dz1 = (dz2 @ p["W2"].T) * (z1 > 0.0)
    g["W1"] = X.T @ dz1
    g["b1"] = dz1.sum(axis=0)
    return L, pack(g)


def predict_rank(w, X, chi):
    """Rank the network proposes: ceil(out * chi), clamped to [1, chi]."""
    out, _ = forward(w, X)
    return np.clip(np.ceil(out * chi), 1, chi).astype(int)
