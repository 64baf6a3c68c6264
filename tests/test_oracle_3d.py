"""Pins of the three-dimensional oracle (K = 3n sites, registers x, y, z): the
seven-point stencil against index loops, the shift MPOs against the dense
shifts on every basis field, the Laplacian MPS against the stencil, eq. 2 in
3D without truncation (Table 1's equivalence), a 3D plane wave against its
closed-form dispersion relation, and the core-level stepper against the
dense-detour stepper with truncation.  Both site orders."""
import numpy as np
import pytest

from oracle import mps as M
from oracle import fdtd as F
from oracle import stepper as S
import synth

ORD = ("sequential", "interleaved")


def _brute_laplacian3(u, boundary):
    N = u.shape[0]
    out = np.zeros_like(u)
    for x in range(N):
        for y in range(N):
            for z in range(N):
                acc = -6.0 * u[x, y, z]
                for dx, dy, dz in ((1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)):
                    xx, yy, zz = x + dx, y + dy, z + dz
                    if boundary == "periodic":
                        xx, yy, zz = xx % N, yy % N, zz % N
                    elif not (0 <= xx < N and 0 <= yy < N and 0 <= zz < N):
                        continue
                    acc += u[xx, yy, zz]
                out[x, y, z] = acc
    return out


@pytest.mark.parametrize("boundary", ["periodic", "open"])
def test_seven_point_stencil_against_index_loops(boundary):
    u = np.random.default_rng(1).standard_normal((4, 4, 4))
    np.testing.assert_allclose(F.laplacian(u, boundary), _brute_laplacian3(u, boundary), atol=1e-13)


@pytest.mark.parametrize("n", [1, 2])
@pytest.mark.parametrize("boundary", ["periodic", "open"])
@pytest.mark.parametrize("ordering", ORD)
def test_shift_mpo_3d_on_basis_fields(n, boundary, ordering):
    N = 1 << n
    for ax in range(3):
        for d in (+1, -1):
            W = M.mpo_to_dense(M.shift_mpo_nd(n, ax, d, boundary, ordering, 3))
            for idx in np.ndindex(N, N, N):
                e = np.zeros((N, N, N))
                e[idx] = 1.0
                ref = F.shift_plus(e, ax, boundary) if d > 0 else F.shift_minus(e, ax, boundary)
                got = M.from_sites(W @ M.to_sites(e, ordering), n, ordering, 3)
                np.testing.assert_array_equal(got, ref)


@pytest.mark.parametrize("n", [1, 2, 3])
@pytest.mark.parametrize("boundary", ["periodic", "open"])
@pytest.mark.parametrize("ordering", ORD)
def test_laplacian_mps_3d_is_seven_point_stencil(n, boundary, ordering):
    K = 3 * n
    bonds = [1] + [min(4, 2 ** k, 2 ** (K - k)) for k in range(1, K)] + [1]
    A = synth.random_mps_cores(K, bonds, seed=n)
    u = M.from_sites(M.to_dense(A), n, ordering, 3)
    L = M.from_sites(M.to_dense(M.laplacian_mps(A, n, boundary, ordering, 3)), n, ordering, 3)
    np.testing.assert_allclose(L, _brute_laplacian3(u, boundary), atol=1e-12)


def test_point_state_3d():
    n = 2
    for o in ORD:
        for idx in [(0, 0, 0), (3, 1, 2), (2, 3, 0)]:
            e = M.from_sites(M.to_dense(M.point_state_nd(n, idx, o)), n, o, 3)
            assert e[idx] == 1.0 and np.count_nonzero(e) == 1


@pytest.mark.parametrize("n", [2, 3])
@pytest.mark.parametrize("boundary", ["periodic", "open"])
@pytest.mark.parametrize("ordering", ORD)
def test_untruncated_3d_step_equals_fdtd(n, boundary, ordering):
    N = 1 << n
    rng = np.random.default_rng(30 + n)
    c2 = 0.5 + rng.random((N, N, N))
    lam = 0.3
    wav = rng.standard_normal(6)
    src = (N // 2, 1, N - 1)
    st = S.MPSStepper(n, lam, 0.0, 1 << 20, S.c2_mps(c2, n, 0.0, ordering), boundary,
                      src=src, wavelet=wav, ordering=ordering, ndim=3)
    up, u = rng.standard_normal((N, N, N)), rng.standard_normal((N, N, N))
    st.set_fields(up, u)
    a, b = up, u
    for k in range(6):
        st.step()
        a, b = b, F.fdtd_step(b, a, c2, lam, wav[k], src, boundary)
        assert np.linalg.norm(st.dense() - b) <= 1e-12 * np.linalg.norm(b)


@pytest.mark.parametrize("ordering", ORD)
def test_plane_wave_3d_closed_form(ordering):
    """cos(2 pi (mx x + my y + mz z) / N - k omega dt) solves the 3D scheme
    exactly when sin^2(omega dt / 2) = C^2 (sum over axes of sin^2(pi m / N));
    it has quantics rank 2 in any site order."""
    n, ms, courant = 4, (3, 5, 1), 0.4
    N = 1 << n
    s2 = sum(np.sin(np.pi * m / N) ** 2 for m in ms)
    wdt = 2.0 * np.arcsin(courant * np.sqrt(s2))
    grid = np.meshgrid(*[np.arange(N)] * 3, indexing="ij")
    theta = 2.0 * np.pi * sum(m * g for m, g in zip(ms, grid)) / N + 0.3
    st = S.MPSStepper(n, courant, 1e-12, 8, S.c2_mps(np.ones((N, N, N)), n, 1e-12, ordering),
                      ordering=ordering, ndim=3)
    st.set_fields(np.cos(theta + wdt), np.cos(theta))
    steps = 12
    for _ in range(steps):
        st.step()
    assert np.max(np.abs(st.dense() - np.cos(theta - steps * wdt))) < 1e-11
    assert max(M.bonds_of(st.psi)) == 2


@pytest.mark.parametrize("ordering", ORD)
def test_3d_mps_stepper_equals_dense_stepper(ordering):
    n, eps, chi = 3, 1e-4, 10
    N = 1 << n
    rng = np.random.default_rng(7)
    c2 = 0.6 + 0.2 * rng.random((N, N, N))
    lam = 0.3
    c2m = S.c2_mps(c2, n, 1e-6, ordering)
    c2d = M.from_sites(M.to_dense(c2m), n, ordering, 3)
    wav = synth.ricker(15, 0.02, 4.0)
    src = (N // 2, N // 2, 1)
    st = S.MPSStepper(n, lam, eps, chi, c2m, src=src, wavelet=wav, ordering=ordering, ndim=3)
    ds = S.DenseStepper(n, lam, eps, chi, c2d, src=src, wavelet=wav, ordering=ordering)
    for _ in range(15):
        st.step()
        ds.step()
    d = ds.dense()
    assert np.linalg.norm(st.dense() - d) <= 1e-10 * np.linalg.norm(d)
    assert M.bonds_of(st.psi) == ds.ranks[-1][2]
