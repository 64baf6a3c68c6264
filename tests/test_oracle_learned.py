"""Pins of the oracle's learned-rank rounding (oracle.rrf.LearnedRounding):
on a tensor of known exact rank a sketch wide enough is accepted and the
result is the exact rounding; a sketch too narrow is rejected, the exact SVD
runs (the result is the exact rounding bit for bit) and the bond then waits
1, 2, 4, ... steps before it is sketched again."""
import numpy as np

from oracle import mlp
from oracle import mps as M
from oracle import rrf


def constant_net(frac):
    w = np.zeros(mlp.NPARAM)
    w[-1] = frac
    return w


def low_rank_sum(K, r, seed):
    """Three copies of one random bond-r MPS (coefficients 1, 0.5, -0.25):
    formal bond 3 r, exact rank at most r."""
    rng = np.random.default_rng(seed)
    bonds = [1] + [min(r, 2 ** k, 2 ** (K - k)) for k in range(1, K)] + [1]
    A = [rng.standard_normal((bonds[k], 2, bonds[k + 1])) for k in range(K)]
    return M.direct_sum([A, A, A], [1.0, 0.5, -0.25]), bonds


def test_wide_sketch_is_exact_on_low_rank_tensor():
    K, r, chi, eps = 12, 16, 64, 1e-10
    T, bonds = low_rank_sum(K, r, seed=1)
    exact = M.round_mps(T, eps, chi)
    lr = rrf.LearnedRounding(constant_net(0.25), seed=5, K=K)   # r_hat = 16, width 24
    first, _ = lr.round(T, eps, chi, step=0, rnd=0)               # no log yet: exact
    assert lr.sketches == 0
    second, tail = lr.round(T, eps, chi, step=1, rnd=0)
    assert lr.sketches > 0 and lr.fallbacks == 0
    assert M.bonds_of(second) == M.bonds_of(exact) == bonds
    ref = M.to_dense(exact)
    assert np.linalg.norm(M.to_dense(second) - ref) < 1e-12 * np.linalg.norm(ref)
    assert tail < 1e-24 * np.sum(ref ** 2)


def test_narrow_sketch_is_rejected_and_waits():
    K, r, chi, eps = 12, 16, 64, 1e-10
    T, _ = low_rank_sum(K, r, seed=2)
    exact = M.to_dense(M.round_mps(T, eps, chi))
    lr = rrf.LearnedRounding(constant_net(2.0 / 64), seed=5, K=K)   # r_hat = 2, width 10 < rank
    sketched_at = []
    for step in range(12):
        before = lr.sketches
        out, _ = lr.round(T, eps, chi, step=step, rnd=1)
        assert np.array_equal(M.to_dense(out), exact)     # every sketch rejected: exact SVDs
        if lr.sketches > before:
            sketched_at.append(step)
    assert lr.fallbacks == lr.sketches > 0
    # first sketch at step 1 (step 0 has no log), then waits of 1, 2, 4, ... steps
    assert sketched_at == [1, 3, 6, 11]


def test_accepted_sketch_misses_only_values_below_the_cutoff():
    rng = np.random.default_rng(3)
    m, n, eps = 96, 64, 1e-6
    s = np.concatenate([np.geomspace(1.0, 1e-4, 12), 1e-8 * np.ones(40)])
    U, _ = np.linalg.qr(rng.standard_normal((m, s.size)))
    V, _ = np.linalg.qr(rng.standard_normal((n, s.size)))
    Mx = (U * s) @ V.T
    lr = rrf.LearnedRounding(constant_net(12.0 / 64), seed=7, K=4)
    lr.sig[(0, 2)] = s[:32]
    Vt, US, S, r, tail = lr.svd(Mx, eps, 64, rnd=0, k=2, step=3)
    assert lr.sketches == 1 and lr.fallbacks == 0
    assert r == 12
    assert np.linalg.norm(US @ Vt - Mx) ** 2 <= tail * (1 + 1e-6)
    assert tail < 40 * (1e-8) ** 2 * 1.01


def test_previous_rank_baseline_sketches_at_the_last_kept_rank():
    """The baseline without a network: the first rounding has no rank to go
    by (exact SVDs), the second sketches every bond at the rank it kept, and
    on a tensor of exact rank r those sketches (width r + 8) are all accepted
    and give the exact rounding."""
    K, r, chi, eps = 12, 16, 64, 1e-10
    T, bonds = low_rank_sum(K, r, seed=4)
    exact = M.round_mps(T, eps, chi)
    lr = rrf.LearnedRounding(None, seed=5, K=K, prev_rank=True)
    lr.round(T, eps, chi, step=0, rnd=2)
    assert lr.sketches == 0
    assert all(lr.rank[(2, k)] == bonds[k] for k in range(1, K))
    second, tail = lr.round(T, eps, chi, step=1, rnd=2)
    assert lr.sketches > 0 and lr.fallbacks == 0
    assert M.bonds_of(second) == M.bonds_of(exact)
    ref = M.to_dense(exact)
    assert np.linalg.norm(M.to_dense(second) - ref) < 1e-12 * np.linalg.norm(ref)
