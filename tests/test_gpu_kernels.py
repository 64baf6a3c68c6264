"""Unit tests of the factorisation kernels (QR, one-sided Jacobi SVD) on
single matrices, against LAPACK through NumPy."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mpsw():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    from paper_2609_01904_amd import mpsw as m
    m.load()
    return m


def _graded(m, n, seed, decay=12.0):
    rng = np.random.default_rng(seed)
    U, _ = np.linalg.qr(rng.standard_normal((m, min(m, n))))
    V, _ = np.linalg.qr(rng.standard_normal((n, min(m, n))))
    s = np.logspace(0, -decay, min(m, n))
    return (U * s) @ V.T


@pytest.mark.parametrize("m,n", [(32, 8), (128, 32), (64, 40), (300, 100), (512, 200), (8, 8), (16, 40),
                                 (2048, 100), (4096, 48),    # 8- and 4-wide panels (LDS)
                                 (1024, 1024), (2048, 512), (2048, 2048), (4096, 1024)])   # the n = 10, 11 TT-SVDs
def test_qr(mpsw, m, n):
    print("qr", m, n, flush=True)
    A = np.random.default_rng(m + n).standard_normal((m, n))
    Q, R = mpsw.debug_factor(0, A)
    q = Q.shape[1]
    assert q == (n if m > n else m)
    np.testing.assert_allclose(Q @ R, A, atol=1e-12 * np.abs(A).max() * np.sqrt(m))
    np.testing.assert_allclose(Q.T @ Q, np.eye(q), atol=1e-13 * m)
    if m > n:
        assert np.allclose(np.tril(R, -1), 0.0)


@pytest.mark.parametrize("m,n", [(8, 8), (16, 32), (64, 64), (32, 64), (64, 40), (100, 256), (256, 256), (300, 128),
                                 (512, 400), (400, 600),    # factors of 257-512 columns
                                 (2048, 504), (1024, 504)])  # bond matrices of the n = 11 TT-SVD
def test_svd(mpsw, m, n):
    print("svd", m, n, flush=True)
    A = _graded(m, n, seed=m * 7 + n)
    Vt, US = mpsw.debug_factor(1, A)
    r = min(m, n)
    s = np.linalg.norm(US, axis=0)
    ref = np.linalg.svd(A, compute_uv=False)
    np.testing.assert_allclose(s, ref, atol=1e-13 * ref[0] * np.sqrt(max(m, n)), rtol=0)
    np.testing.assert_allclose(Vt @ Vt.T, np.eye(r), atol=1e-12)
    np.testing.assert_allclose(US @ Vt, A, atol=1e-13 * np.sqrt(max(m, n)))
    assert np.all(np.diff(s) <= 1e-15)


@pytest.mark.parametrize("scaled", [False, True])
def test_qr_of_a_numerically_low_rank_field(mpsw, scaled):
    """The 4096 x 1024 unfolding of the n = 11 layered-model c^2: its trailing
    columns fall to about 1e-159 of the matrix (squares in the subnormal
    range) once its numerical rank is spent; the reflectors must stay
    orthogonal there."""
    import synth
    A = synth.get_config("C5")["c2"].reshape(4096, 1024)
    if scaled:
        A = A / np.linalg.norm(A)
    Q, R = mpsw.debug_factor(0, A)
    err = np.linalg.norm(Q @ R - A) / np.linalg.norm(A)
    orth = np.linalg.norm(Q.T @ Q - np.eye(Q.shape[1]))
    print(f"low-rank field QR (scaled {scaled}): |QR - A|/|A| {err:.1e}, |Q^T Q - I| {orth:.1e}", flush=True)
    assert err < 1e-13 and orth < 1e-11


def test_svd_of_a_strongly_graded_bond_matrix(mpsw):
    """A bond matrix of the n = 11 c^2 TT-SVD taken in LAPACK's gauge (site 12,
    1024 x 190, singular values from 2.3e10 down to 3.5e-8, 18 orders): the
    values above the noise level 1e-14 ||M||_F are resolved, their vectors
    are orthonormal and reconstruct M; the values below it are not kept (the
    Jacobi sweep cannot resolve their directions)."""
    import synth
    cfg = synth.get_config("C5")
    n, eps = cfg["n"], cfg["eps_c"]
    K = 2 * n
    T = cfg["c2"].reshape(-1)
    rt, X, Qs = 1, T.reshape(1, -1), []
    for k in range(K - 1):   # left-to-right QR sweep of the dense tensor
        m = 2 * rt
        A = X.reshape(m, X.size // m)
        if m <= A.shape[1]:
            Qs.append(None)
            X, rt = A, m
            continue
        Q, R = np.linalg.qr(A)
        Qs.append(Q)
        X, rt = R, R.shape[0]
    B = X.reshape(rt, -1)
    for k in range(K - 1, 12, -1):   # right-to-left truncated SVD sweep down to site 12
        U, s, Vt = np.linalg.svd(B, full_matrices=False)
        keep = max(1, int(np.sum(s >= eps * s[0])))
        prev = U[:, :keep] * s[:keep]
        if Qs[k - 1] is not None:
            prev = Qs[k - 1] @ prev
        B = prev.reshape(prev.shape[0] // 2, 2 * keep)
    M = B
    ref = np.linalg.svd(M, compute_uv=False)
    Vt, US = mpsw.debug_factor(1, M)
    r = Vt.shape[0]
    noise = 1e-14 * np.linalg.norm(M)
    sg = np.linalg.norm(US, axis=0)
    print(f"graded {M.shape}: sigma {ref[0]:.2e} .. {ref[-1]:.2e}, kept {r} of {len(ref)} "
          f"(above the noise level: {int(np.sum(ref > noise))})", flush=True)
    # values within a factor 2 of the noise level may fall on either side of it
    assert int(np.sum(ref > 2 * noise)) <= r <= int(np.sum(ref > noise / 2)), r
    np.testing.assert_allclose(sg, ref[:r], atol=1e-13 * ref[0] * np.sqrt(M.shape[0]), rtol=0)
    np.testing.assert_allclose(Vt @ Vt.T, np.eye(r), atol=1e-10)
    assert np.linalg.norm(US @ Vt - M) <= 1e-13 * np.sqrt(M.shape[0]) * np.linalg.norm(M)
