"""Pins of the dense FDTD oracle (Sec. 2, eq. 2; Sec. 3.2, eq. 7)."""
import numpy as np
import pytest

from oracle import fdtd as F
import synth


@pytest.mark.parametrize("n", [1, 2, 3, 4])
@pytest.mark.parametrize("boundary", ["periodic", "open"])
def test_laplacian_vs_index_loops(n, boundary):
    rng = np.random.default_rng(n)
    N = 1 << n
    u = rng.standard_normal((N, N))
    L = F.brute_laplacian_matrix(n, boundary)
    np.testing.assert_allclose(F.laplacian(u, boundary).reshape(-1), L @ u.reshape(-1),
                               rtol=0, atol=1e-12)


@pytest.mark.parametrize("n", [2, 3])
@pytest.mark.parametrize("boundary", ["periodic", "open"])
def test_step_equals_transition_operator(n, boundary):
    """Eq. 2 == eq. 7: u^{k+1} = A u^k - u^{k-1}, A = 2I + lambda^2 C^2 L."""
    rng = np.random.default_rng(10 + n)
    N = 1 << n
    c2 = 1.0 + rng.random((N, N))
    u, up = rng.standard_normal((N, N)), rng.standard_normal((N, N))
    lam = 0.3
    A = F.brute_transition_matrix(n, c2, lam, boundary)
    ref = A @ u.reshape(-1) - up.reshape(-1)
    np.testing.assert_allclose(F.fdtd_step(u, up, c2, lam, boundary=boundary).reshape(-1),
                               ref, rtol=0, atol=1e-12)


@pytest.mark.parametrize("n,mx,mz", [(6, 1, 0), (6, 3, 5), (8, 7, 2), (10, 13, 29)])
def test_plane_wave_dispersion(n, mx, mz):
    """Discrete dispersion relation: cos(theta - k w dt) is exact for eq. 2."""
    courant = 0.5
    N = 1 << n
    c2 = np.full((N, N), 1.0)
    lam = courant
    up, u = synth.plane_wave_fields(n, mx, mz, courant)
    wdt = synth.fields.plane_wave_omega_dt(n, mx, mz, courant)
    steps = 200
    _, u_end, _ = F.fdtd_run(up, u, c2, lam, steps)
    x = np.arange(N)[:, None]
    z = np.arange(N)[None, :]
    exact = np.cos(2 * np.pi * (mx * x + mz * z) / N - steps * wdt)
    assert np.max(np.abs(u_end - exact)) < 1e-10


@pytest.mark.parametrize("n,mx,mz", [(4, 1, 1), (6, 3, 5), (8, 7, 2), (10, 13, 29)])
def test_sine_mode_dispersion_open_boundary(n, mx, mz):
    """With zero-fill shifts (eq. 11 as printed), standing sine modes are exact
    eigenvectors of the 5-point Laplacian, so cos(phi - k w dt) v is exact."""
    courant = 0.5
    N = 1 << n
    c2 = np.full((N, N), 1.0)
    up, u = synth.sine_mode_fields(n, mx, mz, courant, phase=0.3)
    wdt = synth.fields.sine_mode_omega_dt(n, mx, mz, courant)
    steps = 200
    _, u_end, _ = F.fdtd_run(up, u, c2, courant, steps, boundary="open")
    _, v = synth.sine_mode_fields(n, mx, mz, courant, phase=0.0)
    exact = np.cos(0.3 - steps * wdt) * v
    assert np.max(np.abs(u_end - exact)) < 1e-10
    # and it is not a solution of the periodic scheme (the boundary matters)
    _, u_per, _ = F.fdtd_run(up, u, c2, courant, steps, boundary="periodic")
    assert np.max(np.abs(u_per - exact)) > 1e-3


@pytest.mark.parametrize("boundary", ["periodic", "open"])
def test_energy_conserved(boundary):
    n = 5
    N = 1 << n
    c2 = synth.layered_fault_velocity(n) / 4500.0 ** 2
    lam = 0.6
    up, u = synth.random_fields(n, seed=3)
    e0 = F.energy(u, up, c2, lam, boundary)
    es = []
    for _ in range(400):
        up, u = u, F.fdtd_step(u, up, c2, lam, boundary=boundary)
        es.append(F.energy(u, up, c2, lam, boundary))
    assert max(abs(e - e0) for e in es) <= 1e-12 * abs(e0) * 50


def test_lambda_zero_is_linear_in_time():
    n = 3
    rng = np.random.default_rng(0)
    up, u = rng.standard_normal((2, 8, 8))
    c2 = 1 + rng.random((8, 8))
    a, b = up, u
    for k in range(1, 6):
        a, b = b, F.fdtd_step(b, a, c2, 0.0)
        np.testing.assert_allclose(b, u + k * (u - up), atol=1e-12)


def test_point_source_enters_next_step():
    n = 3
    c2 = np.ones((8, 8))
    z = np.zeros((8, 8))
    u1 = F.fdtd_step(z, z, c2, 0.4, s=2.5, src=(3, 6))
    assert u1[3, 6] == 2.5 and np.count_nonzero(u1) == 1
