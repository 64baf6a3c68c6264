"""Pins of the LCU simulation of the wavefield update (Sec. 3.2, eq. 7; the
Laplacian as a sum of shift unitaries, eq. 6; the shifts from the incrementer
circuits of Sec. 3.1).  The transition operator is checked against the dense
FDTD update of eq. 2 (itself pinned to index loops), the block encoding
against A / |alpha|_1 and unitarity, and the postselected circuit step against
eq. 2 over several steps on grids up to 32 x 32."""
import numpy as np
import pytest

from oracle import fdtd as F
from oracle import lcu


def _c2(n, seed):
    N = 1 << n
    return 0.5 + np.random.default_rng(seed).random((N, N))


@pytest.mark.parametrize("n", [1, 2, 3])
def test_terms_are_unitary_and_sum_to_A(n):
    c2, lam = _c2(n, n), 0.3
    alphas, units, beta = lcu.lcu_terms(c2, lam)
    assert len(alphas) == 11 and np.all(alphas >= 0.0)
    assert np.isclose(np.sum(alphas), 2.0 + 8.0 * beta)
    A = lcu.transition_dense(c2, lam)
    rng = np.random.default_rng(10 + n)
    for _ in range(3):
        v = rng.standard_normal(c2.size) + 1j * rng.standard_normal(c2.size)
        acc = np.zeros_like(v)
        for a, U in zip(alphas, units):
            Uv = U(v)
            assert np.isclose(np.linalg.norm(Uv), np.linalg.norm(v))
            acc += a * Uv
        np.testing.assert_allclose(acc, A @ v, atol=1e-12)


@pytest.mark.parametrize("n", [2, 3])
def test_transition_operator_is_the_fdtd_update(n):
    """A psi - psi_prev equals eq. 2 on the periodic grid (no source)."""
    c2, lam = _c2(n, 20 + n), 0.4
    rng = np.random.default_rng(n)
    N = 1 << n
    u, up = rng.standard_normal((N, N)), rng.standard_normal((N, N))
    A = lcu.transition_dense(c2, lam)
    ref = F.fdtd_step(u, up, c2, lam, 0.0, (0, 0), "periodic")
    np.testing.assert_allclose((A @ u.ravel() - up.ravel()).reshape(N, N), ref, atol=1e-12)


def test_block_encoding_top_left_block_and_unitarity():
    n, lam = 2, 0.35
    c2 = _c2(n, 3)
    alphas, units, _ = lcu.lcu_terms(c2, lam)
    nidx = lcu.index_size(len(alphas))
    P = lcu.prepare_matrix(alphas, nidx)
    np.testing.assert_allclose(P.T @ P, np.eye(nidx), atol=1e-14)
    np.testing.assert_allclose(P[:, 0] ** 2, np.r_[alphas, np.zeros(nidx - len(alphas))] / np.sum(alphas), atol=1e-15)
    M = c2.size
    W = np.zeros((nidx * M, nidx * M), dtype=complex)
    for col in range(nidx * M):
        e = np.zeros((nidx, M), dtype=complex)
        e[col // M, col % M] = 1.0
        W[:, col] = lcu.block_encode_apply(e, alphas, units, P).ravel()
    np.testing.assert_allclose(W.conj().T @ W, np.eye(nidx * M), atol=1e-12)
    np.testing.assert_allclose(W[:M, :M], lcu.transition_dense(c2, lam) / np.sum(alphas), atol=1e-13)


@pytest.mark.parametrize("n", [2, 3, 5])
def test_postselected_circuit_step_is_eq2(n):
    """Iterated LCU steps follow eq. 2; the circuit is norm-preserving and the
    postselection probability is |psi^{k+1}|^2 / (|alpha|_1 |psi^k| + |psi^{k-1}|)^2."""
    N = 1 << n
    c2, lam = _c2(n, 40 + n), 0.3
    rng = np.random.default_rng(50 + n)
    up, u = rng.standard_normal((N, N)), rng.standard_normal((N, N))
    a, b = up, u
    alphas, _, _ = lcu.lcu_terms(c2, lam)
    for k in range(4):
        nxt, p, total = lcu.lcu_step(u, up, c2, lam)
        a, b = b, F.fdtd_step(b, a, c2, lam, 0.0, (0, 0), "periodic")
        assert np.linalg.norm(nxt - b) <= 1e-12 * np.linalg.norm(b), k
        assert abs(total - 1.0) < 1e-12
        w = np.sum(alphas) * np.linalg.norm(u) + np.linalg.norm(up)
        assert np.isclose(p, np.linalg.norm(b) ** 2 / w ** 2, rtol=1e-10)
        up, u = u, nxt


def test_step_from_rest():
    """psi^{-1} = 0: the second select branch carries no weight."""
    n, lam = 3, 0.3
    N = 1 << n
    c2 = _c2(n, 7)
    u = np.random.default_rng(8).standard_normal((N, N))
    nxt, p, total = lcu.lcu_step(u, np.zeros((N, N)), c2, lam)
    ref = F.fdtd_step(u, np.zeros((N, N)), c2, lam, 0.0, (0, 0), "periodic")
    assert np.linalg.norm(nxt - ref) <= 1e-12 * np.linalg.norm(ref)
    assert abs(total - 1.0) < 1e-12
