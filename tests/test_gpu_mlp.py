"""The rank network's GPU kernels (FP32 forward, backward, Adam) against the
FP64 oracle (itself pinned by central differences).

FP32 bounds: a gradient entry is a sum of products of O(1) values over
m samples and 128 hidden units, so the normwise relative error of the whole
gradient is a small multiple of 6e-8 times the depth of the sums; 1e-4 is
asserted normwise, and the loss to 1e-5.
"""
import sys

import numpy as np
import pytest

from oracle import mlp

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def mpsw():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    from paper_2609_01904_amd import mpsw as m
    m.load()
    return m


def _data(m, seed):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((m, mlp.NIN)).astype(np.float32)
    X[:, :32] = -np.abs(X[:, :32]) * 3.0   # log10 sigma ratios are <= 0
    y = rng.uniform(0.05, 1.0, m).astype(np.float32)
    return X, y


@pytest.mark.parametrize("m", [1, 31, 100, 257])
def test_gradient_matches_oracle(mpsw, m):
    _say("mlp grad", m)
    X, y = _data(m, seed=m)
    w = mlp.init(seed=11).astype(np.float32)
    w[-1] = 0.4
    Lg, gg = mpsw.mlp_grad(X, y, w, alpha=4.0)
    Lo, go = mlp.grad(w.astype(np.float64), X.astype(np.float64), y.astype(np.float64), 4.0)
    assert abs(Lg - Lo) <= 1e-5 * max(Lo, 1e-12), (Lg, Lo)
    err = np.linalg.norm(gg - go) / np.linalg.norm(go)
    _say(f"m={m}: loss {Lg:.6e} vs {Lo:.6e}; gradient rel err {err:.2e}")
    assert err < 1e-4, err
    out = mpsw.mlp_forward(X, w)
    ref, _ = mlp.forward(w.astype(np.float64), X.astype(np.float64))
    assert np.max(np.abs(out - ref)) <= 1e-5 * max(1.0, np.max(np.abs(ref)))


def test_training_fits_and_matches_oracle_forward(mpsw):
    # a smooth target of the features: rank fraction falls with the spectrum's decay
    rng = np.random.default_rng(5)
    m = 2000
    decay = rng.uniform(0.05, 1.0, m)
    X = np.full((m, mlp.NIN), -30.0, dtype=np.float32)
    for i in range(32):
        X[:, i] = np.maximum(-decay * i, -30.0)
    X[:, 32] = rng.uniform(0, 1, m)
    X[:, 33] = rng.uniform(0, 2, m)
    y = np.clip(1.0 / (1.0 + 8.0 * decay), 0.0, 1.0).astype(np.float32)
    w0 = mlp.init(seed=2).astype(np.float32)
    L0 = mlp.loss(w0.astype(np.float64), X.astype(np.float64), y.astype(np.float64), 4.0)
    w = mpsw.mlp_train(X, y, w0, epochs=300, lr=3e-3, alpha=4.0)
    L1 = mlp.loss(w.astype(np.float64), X.astype(np.float64), y.astype(np.float64), 4.0)
    _say(f"training loss {L0:.4e} -> {L1:.4e}")
    assert L1 < 0.01 * L0 and L1 < 0.05
    out = mpsw.mlp_forward(X, w)
    ref, _ = mlp.forward(w.astype(np.float64), X.astype(np.float64))
    assert np.max(np.abs(out - ref)) <= 1e-4
