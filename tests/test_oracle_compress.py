"""Pins of the oracle's alternative compressions (oracle.compress): the
Laplacian and c^2 operators as single MPOs against the pinned core-level
constructions and the dense stencil, zip-up and the variational fit exact when
nothing needs truncating, the variational fit never worse than the rounding it
starts from, and the right-orthonormal form."""
import numpy as np
import pytest

from oracle import compress as C
from oracle import fdtd as F
from oracle import mps as M


def random_mps(K, r, seed):
    rng = np.random.default_rng(seed)
    bonds = [1] + [min(r, 2 ** k, 2 ** (K - k)) for k in range(1, K)] + [1]
    return [rng.standard_normal((bonds[k], 2, bonds[k + 1])) for k in range(K)]


def dense(cores):
    return M.to_dense(cores).reshape(-1)


@pytest.mark.parametrize("boundary", ["periodic", "open"])
def test_laplacian_mpo_equals_the_stencil(boundary):
    n = 3
    psi = random_mps(2 * n, 4, seed=1)
    u = M.from_sites(M.to_dense(psi), n)
    y = M.apply_mpo(C.laplacian_mpo(n, boundary), psi)
    assert np.allclose(dense(y), dense(M.laplacian_mps(psi, n, boundary)), atol=1e-12)
    assert np.allclose(M.from_sites(M.to_dense(y), n), F.laplacian(u, boundary), atol=1e-12)


def test_diagonal_mpo_is_the_hadamard_product():
    c2, y = random_mps(6, 3, seed=2), random_mps(6, 4, seed=3)
    out = M.apply_mpo(C.diagonal_mpo(c2), y)
    assert np.allclose(dense(out), dense(c2) * dense(y), atol=1e-12)


def test_right_orthonormal_form():
    psi = random_mps(8, 5, seed=4)
    G = C.right_orthonormal(psi)
    assert np.allclose(dense(G), dense(psi), atol=1e-12 * np.linalg.norm(dense(psi)))
    for g in G[1:]:
        r0, d, r1 = g.shape
        A = g.reshape(r0, d * r1)
        assert np.allclose(A @ A.T, np.eye(r0), atol=1e-12)


@pytest.mark.parametrize("method", ["zipup", "variational"])
def test_exact_when_nothing_is_cut(method):
    n = 3
    psi = random_mps(2 * n, 4, seed=5)
    W = C.laplacian_mpo(n)
    ref = dense(M.apply_mpo(W, psi))
    out = C.zip_up(W, psi, 0.0, 1 << 20) if method == "zipup" else C.variational(W, psi, 0.0, 1 << 20)
    assert np.linalg.norm(dense(out) - ref) < 1e-12 * np.linalg.norm(ref)


def test_zip_up_exact_on_a_plane_wave():
    """A plane wave is a quantics MPS of rank 2 and so is its Laplacian: zip-up
    with a cap of 2 loses nothing."""
    n = 5
    N = 1 << n
    x = np.arange(N)
    u = np.cos(2 * np.pi * (3 * x[:, None] + 5 * x[None, :]) / N)
    psi = M.tt_svd(M.to_sites(u), 2 * n, 1e-12, 8)
    out = C.zip_up(C.laplacian_mpo(n), psi, 1e-12, 2)
    assert max(M.bonds_of(out)) <= 2
    assert np.allclose(M.from_sites(M.to_dense(out), n), F.laplacian(u), atol=1e-10)


def test_variational_fit_never_worse_than_its_start():
    """From the rounding of the exact product, or from the zip-up result (its
    default start), the fit keeps the bonds (the zip-up's up to dimensions
    beyond a bond's possible rank) and does not move away from the exact
    product."""
    n = 4
    psi = random_mps(2 * n, 8, seed=6)
    W = C.laplacian_mpo(n)
    exact = dense(M.apply_mpo(W, psi))
    for chi in (3, 6, 10):
        r = M.round_mps(M.apply_mpo(W, psi), 0.0, chi)
        v = C.variational(W, psi, 0.0, chi, sweeps=3, start=r)
        er, ev = np.linalg.norm(dense(r) - exact), np.linalg.norm(dense(v) - exact)
        assert M.bonds_of(v) == M.bonds_of(r)
        assert ev <= er * (1 + 1e-10), (chi, ev, er)
        z = C.zip_up(W, psi, 0.0, chi)
        vz = C.variational(W, psi, 0.0, chi, sweeps=3)
        ez, evz = np.linalg.norm(dense(z) - exact), np.linalg.norm(dense(vz) - exact)
        # the fit's gauge steps drop bond dimensions the zip-up kept beyond the
        # rank a bond can have (it truncates before the last sites are seen)
        assert all(a <= b for a, b in zip(M.bonds_of(vz), M.bonds_of(z)))
        assert evz <= ez * (1 + 1e-10), (chi, evz, ez)
        print(chi, "rounding %.3e  zip-up %.3e  fit from zip-up %.3e" % (er, ez, evz))
