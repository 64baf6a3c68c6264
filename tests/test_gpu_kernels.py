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
