"""Pins of the interleaved site order x_{n-1} z_{n-1} ... x_0 z_0 in the oracle:
the site permutation against bit-by-bit index arithmetic, the shift MPOs
against the dense shifts of eq. 2 on every basis field, the Laplacian against
the five-point stencil, the untruncated step against eq. 2 (Table 1) and the
truncated MPS step against the dense-detour step."""
import numpy as np
import pytest

from oracle import mps as M
from oracle import fdtd as F
from oracle import stepper as S
import synth


def _morton(x, z, n):
    """Flat site-order index of (x, z) in the interleaved order, bit by bit."""
    idx = 0
    for m in range(n - 1, -1, -1):
        idx = (idx << 1) | ((x >> m) & 1)
        idx = (idx << 1) | ((z >> m) & 1)
    return idx


@pytest.mark.parametrize("n", [1, 2, 3, 4])
def test_site_permutation(n):
    N = 1 << n
    u = np.random.default_rng(n).standard_normal((N, N))
    t = M.to_sites(u, "interleaved")
    for x in range(N):
        for z in range(N):
            assert t[_morton(x, z, n)] == u[x, z]
    np.testing.assert_array_equal(M.to_sites(u, "sequential"), u.reshape(-1))
    for o in M.ORDERINGS:
        np.testing.assert_array_equal(M.from_sites(M.to_sites(u, o), n, o), u)


@pytest.mark.parametrize("n", [2, 3])
def test_point_state_interleaved(n):
    N = 1 << n
    for ix in range(N):
        for iz in range(N):
            e = M.from_sites(M.to_dense(M.point_state(n, ix, iz, "interleaved")), n, "interleaved")
            assert e[ix, iz] == 1.0 and np.count_nonzero(e) == 1


@pytest.mark.parametrize("n", [1, 2, 3])
@pytest.mark.parametrize("boundary", ["periodic", "open"])
def test_shift_mpo_interleaved_on_basis_fields(n, boundary):
    """Every column of the interleaved shift MPO is the dense shift of a basis field."""
    N = 1 << n
    for ax in (0, 1):
        for d in (+1, -1):
            W = M.mpo_to_dense(M.shift_mpo_2d(n, ax, d, boundary, "interleaved"))
            for x in range(N):
                for z in range(N):
                    e = np.zeros((N, N))
                    e[x, z] = 1.0
                    ref = F.shift_plus(e, ax, boundary) if d > 0 else F.shift_minus(e, ax, boundary)
                    got = M.from_sites(W @ M.to_sites(e, "interleaved"), n, "interleaved")
                    np.testing.assert_array_equal(got, ref)


@pytest.mark.parametrize("n", [1, 2, 3, 4])
@pytest.mark.parametrize("boundary", ["periodic", "open"])
def test_laplacian_interleaved_is_five_point_stencil(n, boundary):
    K = 2 * n
    bonds = [1] + [min(5, 2 ** k, 2 ** (K - k)) for k in range(1, K)] + [1]
    A = synth.random_mps_cores(K, bonds, seed=3 + n)
    u = M.from_sites(M.to_dense(A), n, "interleaved")
    L = M.from_sites(M.to_dense(M.laplacian_mps(A, n, boundary, "interleaved")), n, "interleaved")
    np.testing.assert_allclose(L, F.laplacian(u, boundary), atol=1e-12)


@pytest.mark.parametrize("n", [2, 3, 4])
@pytest.mark.parametrize("boundary", ["periodic", "open"])
def test_untruncated_interleaved_step_equals_fdtd(n, boundary):
    """Table 1 in the interleaved order: no truncation reproduces eq. 2."""
    N = 1 << n
    rng = np.random.default_rng(10 + n)
    c2 = 0.5 + rng.random((N, N))
    lam = 0.4
    wav = rng.standard_normal(10)
    src = (N // 2, 1)
    st = S.MPSStepper(n, lam, 0.0, 1 << 20, S.c2_mps(c2, n, 0.0, "interleaved"), boundary,
                      src=src, wavelet=wav, ordering="interleaved")
    up, u = synth.random_fields(n, seed=n, smooth=False)
    st.set_fields(up, u)
    a, b = up, u
    for k in range(10):
        st.step()
        a, b = b, F.fdtd_step(b, a, c2, lam, wav[k], src, boundary)
        assert np.linalg.norm(st.dense() - b) <= 1e-12 * np.linalg.norm(b)
        assert np.linalg.norm(st.dense(1) - a) <= 1e-12 * np.linalg.norm(a)


@pytest.mark.parametrize("n,eps,chi", [(4, 1e-3, 6), (5, 1e-6, 12)])
def test_interleaved_mps_stepper_equals_dense_stepper(n, eps, chi):
    N = 1 << n
    c2 = synth.layered_fault_velocity(n, dh=40.0) * (1e-3 / 40.0) ** 2 / 1e-6
    lam = 1e-3
    c2m = S.c2_mps(c2, n, 1e-6, "interleaved")
    c2d = M.from_sites(M.to_dense(c2m), n, "interleaved")
    wav = synth.ricker(25, 1e-3, 25.0) * 1e3
    st = S.MPSStepper(n, lam, eps, chi, c2m, src=(N // 2, 1), wavelet=wav, ordering="interleaved")
    ds = S.DenseStepper(n, lam, eps, chi, c2d, src=(N // 2, 1), wavelet=wav, ordering="interleaved")
    up, u = synth.random_fields(n, seed=2)
    st.set_fields(up, u)
    ds.set_fields(up, u)
    for _ in range(25):
        st.step()
        ds.step()
    d = ds.dense()
    assert np.linalg.norm(st.dense() - d) <= 1e-10 * np.linalg.norm(d)
    assert M.bonds_of(st.psi) == ds.ranks[-1][2]


def test_orders_agree_when_nothing_is_cut():
    """With a cutoff far below every kept singular value and no cap, both site
    orders advance the same field (truncation only drops noise-level terms)."""
    n = 4
    N = 1 << n
    c2 = synth.layered_fault_velocity(n, dh=40.0) * (1e-3 / 40.0) ** 2 / 1e-6
    lam = 1e-3
    wav = synth.ricker(15, 1e-3, 25.0) * 1e3
    out = []
    for o in M.ORDERINGS:
        c2d = M.from_sites(M.to_dense(S.c2_mps(c2, n, 0.0, o)), n, o)
        st = S.MPSStepper(n, lam, 1e-14, 1 << 20, S.c2_mps(c2d, n, 0.0, o), src=(N // 2, 1),
                          wavelet=wav, ordering=o)
        for _ in range(15):
            st.step()
        out.append(st.dense())
    assert np.linalg.norm(out[0] - out[1]) <= 1e-11 * np.linalg.norm(out[0])
