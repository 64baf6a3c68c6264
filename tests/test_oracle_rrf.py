"""Pins of the randomized range finder oracle: the generator's published
outputs, exact recovery of low-rank matrices, the acceptance rule on
constructed spectra."""
import numpy as np

from oracle import rrf


def test_splitmix64_published_outputs():
    # SplitMix64 seeded with 0: the state advances by the golden gamma before
    # each output; these are its first three outputs
    x, out = 0, []
    for _ in range(3):
        out.append(rrf.splitmix64(x))
        x = (x + 0x9E3779B97F4A7C15) & rrf.MASK
    assert out == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_sketch_normals_are_standard_normal():
    g = rrf.omega(seed=12345, step=7, rnd=1, site=3, m=200, l=100).ravel()
    assert abs(g.mean()) < 0.02 and abs(g.std() - 1.0) < 0.02
    # distinct keys give distinct entries, equal keys equal entries
    assert rrf.sketch_normal(1, 2, 0, 5, 3, 4) == rrf.sketch_normal(1, 2, 0, 5, 3, 4)
    assert rrf.sketch_normal(1, 2, 0, 5, 3, 4) != rrf.sketch_normal(1, 2, 0, 5, 4, 3)
    assert rrf.sketch_normal(1, 2, 0, 5, 3, 4) != rrf.sketch_normal(1, 2, 1, 5, 3, 4)


def _matrix(m, n, s, seed):
    rng = np.random.default_rng(seed)
    U, _ = np.linalg.qr(rng.standard_normal((m, len(s))))
    V, _ = np.linalg.qr(rng.standard_normal((n, len(s))))
    return (U * s) @ V.T


def test_exact_recovery_of_low_rank_matrix():
    s = np.array([5.0, 3.0, 1.0, 0.5, 0.25])
    M = _matrix(60, 40, s, seed=3)
    Om = rrf.omega(seed=9, step=0, rnd=0, site=2, m=60, l=8)
    Q, B, S, W = rrf.range_finder(M, Om)
    assert np.allclose(S[:5], s, rtol=1e-12)
    assert np.all(S[5:] < 1e-12)
    assert np.allclose(Q.T @ Q, np.eye(8), atol=1e-13)
    assert np.allclose(B @ Q.T, M, atol=1e-12)
    ok, r = rrf.accept(M, Q, B, S, eps=1e-6, chi=10)
    assert ok and r == 5


def test_acceptance_rule():
    # rank above the sketch: every sketched value is above the cutoff -> reject
    s = 2.0 ** -np.arange(30)
    M = _matrix(64, 64, s, seed=4)
    Om = rrf.omega(seed=9, step=1, rnd=2, site=5, m=64, l=10)
    Q, B, S, W = rrf.range_finder(M, Om)
    ok, r = rrf.accept(M, Q, B, S, eps=1e-8, chi=40)
    assert not ok and r == 10
    # fast decay beyond the cutoff inside the sketch -> accept, same rank as exact
    s = np.concatenate([np.ones(6), 1e-9 * np.ones(20)])
    M = _matrix(64, 64, s, seed=5)
    Q, B, S, W = rrf.range_finder(M, Om)
    ok, r = rrf.accept(M, Q, B, S, eps=1e-6, chi=40)
    assert ok and r == 6
    # capped: in-sketch tail large against what the sketch misses -> accept
    s = np.concatenate([np.ones(8), 0.5 * np.ones(2), 1e-8 * np.ones(10)])
    M = _matrix(64, 64, s, seed=6)
    Q, B, S, W = rrf.range_finder(M, Om)
    ok, r = rrf.accept(M, Q, B, S, eps=1e-6, chi=8)
    assert ok and r == 8
    # capped with a flat spectrum beyond the sketch -> reject
    s = np.concatenate([np.ones(8), 0.5 * np.ones(30)])
    M = _matrix(64, 64, s, seed=7)
    Q, B, S, W = rrf.range_finder(M, Om)
    ok, r = rrf.accept(M, Q, B, S, eps=1e-6, chi=8)
    assert not ok


def test_residual_is_formed_directly():
    """At a small cutoff a sketch that misses singular values above it must be
    rejected; ||M||^2 - ||B||^2 would lose them in its rounding noise."""
    eps = 1e-10
    s = np.concatenate([np.ones(4), 1e-9 * np.ones(8)])   # 8 values 10x above the cutoff
    M = _matrix(64, 48, s, seed=8)
    Om = rrf.omega(seed=3, step=0, rnd=0, site=1, m=64, l=4)   # width 4 sees only the leading values
    Q, B, S, W = rrf.range_finder(M, Om)
    missed = 8 * 1e-18
    diff2 = float(np.sum(M * M) - np.sum(B * B))
    assert abs(diff2 - missed) > 10 * missed   # the difference of squares is rounding noise here
    E = M - B @ Q.T
    assert np.isclose(np.sum(E * E), missed, rtol=1e-6)
    ok, r = rrf.accept(M, Q, B, S, eps=eps, chi=40)
    assert not ok
