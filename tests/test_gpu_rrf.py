"""Learned-rank rounding: rank network + randomized range finder + exact
fallback, through the C ABI.

The fallback enforces the truncation tolerance per bond, so a learned-rank
run stays within the truncation error of the exact run: every accepted sketch
keeps all singular values above eps sigma_1 and misses less than that, so the
per-bond difference is a few eps sigma_1.  The exact run is the judge.
"""
import sys

import numpy as np
import pytest

from oracle import mlp
from oracle import stepper as S
import synth

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


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def constant_model(frac):
    """A network whose output is the constant `frac` (rank = ceil(frac chi))."""
    w = np.zeros(mlp.NPARAM, dtype=np.float32)
    w[-1] = frac
    return w


def _run(mpsw, n, chi, eps, steps, rank_mode, model=None, seed=7):
    cfg = synth.get_config("C2", n=n, steps=steps)
    N = 1 << n
    st = mpsw.State(mpsw.make_config(n, chi, eps, cfg["lam"], rank_mode=rank_mode, seed=seed))
    st.set_velocity_dense(cfg["c2"], cfg["eps_c"])
    if model is not None:
        st.set_rank_model(model)
    st.set_source(0, N // 2, 1, synth.ricker(steps, cfg["dt"], 40.0))
    return st, cfg


@pytest.mark.parametrize("frac", [0.02, 0.15])
def test_learned_rank_within_truncation_error_of_exact(mpsw, frac):
    n, chi, eps, steps = 6, 64, 1e-7, 60
    ex, cfg = _run(mpsw, n, chi, eps, steps, mpsw.MPSW_RANK_EXACT)
    ln, _ = _run(mpsw, n, chi, eps, steps, mpsw.MPSW_RANK_LEARNED, constant_model(frac))
    for t in range(0, steps, 10):
        ex.step(10)
        ln.step(10)
        a, b = ex.to_dense(0, 0), ln.to_dense(0, 0)
        st = ln.stats(0)
        _say(f"frac {frac} step {t + 10}: rel-L2 learned vs exact {rel(b, a):.2e}; "
             f"sketches {st['sketches']} fallbacks {st['fallbacks']}")
        assert rel(b, a) < 1e-5
    st = ln.stats(0)
    if frac < 0.05:
        # width 1 + 8 is below the ranks once the field has spread: sketches
        # are rejected and the exact SVD takes over (a rejected bond then
        # waits 1, 2, 4, ... steps before it is sketched again)
        assert st["sketches"] > 0
        assert st["fallbacks"] >= 10
    # the exact run itself against the FP64 oracle
    ds = S.DenseStepper(n, cfg["lam"], eps, chi, ex.to_dense(0, 2), src=((1 << n) // 2, 1),
                        wavelet=synth.ricker(steps, cfg["dt"], 40.0))
    for _ in range(steps):
        ds.step()
    assert rel(ex.to_dense(0, 0), ds.dense()) < 1e-10
    assert rel(ln.to_dense(0, 0), ds.dense()) < 1e-5
    ex.close()
    ln.close()


def test_all_rejected_sketches_reproduce_exact_bitwise(mpsw):
    # eps = 1e-12 keeps every singular value the sketch of width 1 + 8 = 9 sees,
    # so no sketch can show that the kept rank is below its width: every one is
    # rejected, the bond matrix is restored and the exact SVD reproduces the
    # exact-rank run bit for bit
    n, chi, eps, steps = 6, 16, 1e-12, 25
    ex, _ = _run(mpsw, n, chi, eps, steps, mpsw.MPSW_RANK_EXACT)
    ln, _ = _run(mpsw, n, chi, eps, steps, mpsw.MPSW_RANK_LEARNED, constant_model(0.01))
    up, u = synth.random_fields(n, seed=4, smooth=False)   # white noise: every bond at full rank
    for st in (ex, ln):
        st.set_fields(0, up, u)
    ex.step(steps)
    ln.step(steps)
    st = ln.stats(0)
    _say("all-rejected case: sketches", st["sketches"], "fallbacks", st["fallbacks"])
    assert st["sketches"] > 0 and st["fallbacks"] == st["sketches"]
    assert np.array_equal(ex.to_dense(0, 0), ln.to_dense(0, 0))
    assert ex.bonds(0, 0) == ln.bonds(0, 0)
    ex.close()
    ln.close()


def _log_training_data(mpsw, n, chi, eps, steps):
    """(features, labels): spectra of the previous step -> exact ranks."""
    st, _ = _run(mpsw, n, chi, eps, steps, mpsw.MPSW_RANK_EXACT)
    K = 2 * n
    X, y = [], []
    prev = None
    for t in range(steps):
        st.step(1)
        logs = [st.sigma_log(0, j) for j in range(3)]
        ranks = [st.bonds(0, 3), st.bonds(0, 4), st.bonds(0, 0)]   # y, w, psi after the step
        if prev is not None:
            for j in range(3):
                for k in range(1, K):
                    X.append(mlp.features(prev[j][k], k, K, t))
                    y.append(ranks[j][k] / chi)
        prev = logs
    st.close()
    return np.array(X, dtype=np.float32), np.array(y, dtype=np.float32)


def test_trained_network_against_constant_rank(mpsw):
    n, chi, eps, steps = 6, 64, 1e-7, 60
    X, y = _log_training_data(mpsw, n, chi, eps, steps)
    _say("training rows", len(y), "mean label", float(y.mean()))
    w0 = mlp.init(seed=1).astype(np.float32)
    w = mpsw.mlp_train(X, y, w0, epochs=400, lr=2e-3, alpha=4.0)
    L0, _ = mpsw.mlp_grad(X, y, w0, 4.0)
    L1, _ = mpsw.mlp_grad(X, y, w, 4.0)
    _say(f"training loss {L0:.3e} -> {L1:.3e}")
    assert L1 < L0
    res = {}
    for name, model in [("trained", w), ("constant", constant_model(float(np.mean(y))))]:
        ln, _ = _run(mpsw, n, chi, eps, steps, mpsw.MPSW_RANK_LEARNED, model)
        ln.step(steps)
        st = ln.stats(0)
        res[name] = (st["sketches"], st["fallbacks"])
        _say(f"{name}: sketches {st['sketches']} fallbacks {st['fallbacks']}")
        ln.close()
    # the trained network's sketches are rejected no more often than a
    # constant rank's
    ft = res["trained"][1] / max(res["trained"][0], 1)
    fc = res["constant"][1] / max(res["constant"][0], 1)
    assert ft <= fc + 0.05, (res, ft, fc)
