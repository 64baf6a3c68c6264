"""Pins of the MPS oracle: algebra against dense arithmetic, rounding against
known singular values / the dense TT-SVD / its invariances (Sec. 4.1-4.3)."""
import numpy as np
import pytest

from oracle import mps as M
from oracle import fdtd as F
import synth


def _rand_mps(K, r, seed):
    bonds = [1] + [min(r, 2 ** k, 2 ** (K - k)) for k in range(1, K)] + [1]
    return synth.random_mps_cores(K, bonds, seed)


@pytest.mark.parametrize("K", [1, 2, 5, 8])
def test_tt_svd_exact_reconstruction(K):
    rng = np.random.default_rng(K)
    t = rng.standard_normal(2 ** K)
    cores = M.tt_svd(t, K, 0.0, 1 << 20)
    np.testing.assert_allclose(M.to_dense(cores), t, atol=1e-12)
    b = M.bonds_of(cores)
    assert all(b[k] <= min(2 ** k, 2 ** (K - k)) for k in range(K + 1))


def test_rounding_matches_known_singular_values():
    """Eckart-Young pin: a tensor whose unfoldings all have singular values
    exactly (1, 1e-3) (two basis states that differ in the first bit, each with
    its own orthonormal last-site vector) is kept whole or cut to the best
    rank-1 approximation depending on eps."""
    rng = np.random.default_rng(5)
    K = 8
    m = 2 ** (K - 1)
    U = np.zeros((m, 2))
    U[3, 0] = 1.0
    U[m // 2 + 6, 1] = 1.0
    V, _ = np.linalg.qr(rng.standard_normal((2, 2)))
    s = np.array([1.0, 1e-3])
    T = (U * s) @ V.T
    for eps, r_expect in [(1e-4, 2), (1e-2, 1)]:
        log = []
        cores = M.tt_svd(T.reshape(-1), K, eps, 1 << 20, log)
        k_last, s_last, r_last = log[0]
        assert k_last == K - 1 and r_last == r_expect
        np.testing.assert_allclose(s_last, s, rtol=1e-12)
        assert [r for _, _, r in log] == [r_expect] * (K - 1)
        approx = M.to_dense(cores).reshape(m, 2)
        best = (U[:, :r_expect] * s[:r_expect]) @ V[:, :r_expect].T
        np.testing.assert_allclose(approx, best, atol=1e-12)


@pytest.mark.parametrize("K,r,eps,chi", [(6, 8, 1e-1, 8), (8, 16, 3e-2, 6), (10, 12, 1e-2, 9)])
def test_round_mps_equals_dense_tt_svd(K, r, eps, chi):
    """QR sweep + SVD sweep on cores == R->L TT-SVD of the dense tensor."""
    A = _rand_mps(K, r, seed=K)
    B = _rand_mps(K, r, seed=K + 100)
    T = M.direct_sum([A, B], [1.0, 0.5])          # bond 2r, rank-deficient-ish
    rounded = M.round_mps(T, eps, chi)
    ref = M.tt_svd(M.to_dense(T), K, eps, chi)
    d = M.to_dense(ref)
    assert np.linalg.norm(M.to_dense(rounded) - d) <= 1e-11 * np.linalg.norm(d)
    assert M.bonds_of(rounded) == M.bonds_of(ref)


def test_rounding_error_bound_and_idempotence():
    K, eps, chi = 10, 5e-2, 7
    T = _rand_mps(K, 20, seed=1)
    log = []
    R = M.round_mps(T, eps, chi, log)
    dT = M.to_dense(T)
    err = np.linalg.norm(M.to_dense(R) - dT)
    # TT-SVD bound: squared error <= sum of the discarded squared singular values
    bound = np.sqrt(sum(np.sum(s[r:] ** 2) for _, s, r in log))
    assert err <= bound * (1 + 1e-10)
    # With a cap only (eps = 0) a rounded tensor already has bonds <= chi, so
    # rounding it again changes nothing.  (With eps > 0 the sequential R->L
    # truncation is not idempotent: cutting bond k-1 changes the spectrum seen
    # at bond k.)
    Rc = M.round_mps(T, 0.0, chi)
    Rc2 = M.round_mps(Rc, 0.0, chi)
    np.testing.assert_allclose(M.to_dense(Rc2), M.to_dense(Rc), atol=1e-12 * np.linalg.norm(dT))


def test_rounding_scale_equivariant_and_gauge_free():
    K, eps, chi = 8, 1e-2, 6
    T = _rand_mps(K, 12, seed=2)
    R = M.to_dense(M.round_mps(T, eps, chi))
    R3 = M.to_dense(M.round_mps(M.scale(T, -3.0), eps, chi))
    np.testing.assert_allclose(R3, -3.0 * R, atol=1e-12 * np.linalg.norm(R) * 3)
    rng = np.random.default_rng(9)
    G = [c.copy() for c in T]
    for k in range(K - 1):
        r = G[k].shape[2]
        X = rng.standard_normal((r, r)) + 3 * np.eye(r)
        G[k] = np.tensordot(G[k], X, axes=(2, 0))
        G[k + 1] = np.tensordot(np.linalg.inv(X), G[k + 1], axes=(1, 0))
    RG = M.to_dense(M.round_mps(G, eps, chi))
    np.testing.assert_allclose(RG, R, atol=1e-10 * np.linalg.norm(R))


def test_direct_sum_and_hadamard():
    K = 7
    A, B, C = (_rand_mps(K, 5, s) for s in (1, 2, 3))
    S = M.direct_sum([A, B, C], [2.0, -1.0, 0.25])
    np.testing.assert_allclose(M.to_dense(S), 2 * M.to_dense(A) - M.to_dense(B)
                               + 0.25 * M.to_dense(C), atol=1e-12)
    H = M.hadamard(A, B)
    np.testing.assert_allclose(M.to_dense(H), M.to_dense(A) * M.to_dense(B), atol=1e-12)
    assert M.bonds_of(H) == [a * b for a, b in zip(M.bonds_of(A), M.bonds_of(B))]


@pytest.mark.parametrize("n", [1, 2, 3, 4])
@pytest.mark.parametrize("boundary", ["periodic", "open"])
def test_shift_and_laplacian_on_mps(n, boundary):
    K = 2 * n
    N = 1 << n
    A = _rand_mps(K, 6, seed=n)
    u = M.to_dense(A).reshape(N, N)
    for ax in (0, 1):
        for d in (+1, -1):
            got = M.to_dense(M.apply_mpo(M.shift_mpo_2d(n, ax, d, boundary), A)).reshape(N, N)
            ref = F.shift_plus(u, ax, boundary) if d > 0 else F.shift_minus(u, ax, boundary)
            np.testing.assert_allclose(got, ref, atol=1e-13)
    L = M.to_dense(M.laplacian_mps(A, n, boundary)).reshape(N, N)
    np.testing.assert_allclose(L, F.laplacian(u, boundary), atol=1e-12)


@pytest.mark.parametrize("n", [2, 4])
def test_laplacian_mps_vs_brute_matrix(n):
    N = 1 << n
    A = _rand_mps(2 * n, 4, seed=7)
    Lb = F.brute_laplacian_matrix(n, "periodic")
    np.testing.assert_allclose(M.to_dense(M.laplacian_mps(A, n)), Lb @ M.to_dense(A), atol=1e-12)


def test_special_states():
    n = 4
    N = 1 << n
    e = M.to_dense(M.point_state(n, 5, 11)).reshape(N, N)
    assert e[5, 11] == 1.0 and np.count_nonzero(e) == 1
    c2 = np.full(N * N, 4.0e6)
    assert M.bonds_of(M.tt_svd(c2, 2 * n, 1e-12, 1 << 20)) == [1] * (2 * n + 1)
    Z = M.round_mps(M.zero_mps(2 * n), 1e-8, 4)
    assert M.bonds_of(Z) == [1] * (2 * n + 1) and not np.any(M.to_dense(Z))


def test_choose_rank_rule():
    s = np.array([1.0, 0.5, 1e-7, 9.99e-8, 0.0])
    assert M.choose_rank(s, 1e-7, 10) == 3           # sigma >= eps*sigma_1 kept
    assert M.choose_rank(s, 1e-7, 2) == 2            # chi cap
    assert M.choose_rank(s, 2.0, 10) == 1            # at least one
    assert M.choose_rank(np.zeros(3), 1e-7, 10) == 1
    assert M.choose_rank(s, 0.0, 10) == 5            # eps = 0 keeps everything


def test_svd_falls_back_when_divide_and_conquer_fails(monkeypatch):
    """When LAPACK's divide-and-conquer SVD does not converge, the oracle's
    helper takes the QR-iteration driver: the same singular values (to
    rounding), orthonormal factors and the same matrix back."""
    rng = np.random.default_rng(7)
    A = rng.standard_normal((40, 24)) @ np.diag(np.logspace(0, -9, 24)) @ rng.standard_normal((24, 24))
    ref = np.linalg.svd(A, compute_uv=False)

    def fail(*a, **k):
        raise np.linalg.LinAlgError("SVD did not converge")

    monkeypatch.setattr(M.np.linalg, "svd", fail)
    U, s, Vt = M.svd(A)
    monkeypatch.undo()
    assert np.allclose(s, ref, rtol=0, atol=1e-14 * ref[0])
    assert np.allclose(U.T @ U, np.eye(24), atol=1e-13) and np.allclose(Vt @ Vt.T, np.eye(24), atol=1e-13)
    assert np.linalg.norm(U * s @ Vt - A) < 1e-13 * np.linalg.norm(A)
