"""Pins of the MPS time step (eq. 17): Table 1's equivalence with eq. 2 when no
truncation happens, agreement of the two oracle steppers with truncation, the
plane-wave closed form and the discrete energy invariant."""
import numpy as np
import pytest

from oracle import mps as M
from oracle import fdtd as F
from oracle import stepper as S
import synth


@pytest.mark.parametrize("n", [2, 3, 4])
@pytest.mark.parametrize("boundary", ["periodic", "open"])
def test_untruncated_step_equals_fdtd(n, boundary):
    """Table 1: eq. 17 without truncation reproduces eq. 2 (rel. L2 <= 1e-12)."""
    N = 1 << n
    rng = np.random.default_rng(n)
    c2 = 0.5 + rng.random((N, N))
    lam = 0.4
    wav = rng.standard_normal(12)
    src = (N // 2, 1)
    c2m = S.c2_mps(c2, n, 0.0)
    st = S.MPSStepper(n, lam, 0.0, 1 << 20, c2m, boundary, src=src, wavelet=wav)
    up, u = synth.random_fields(n, seed=n, smooth=False)
    st.set_fields(up, u)
    a, b = up, u
    for k in range(12):
        st.step()
        a, b = b, F.fdtd_step(b, a, c2, lam, wav[k], src, boundary)
        assert np.linalg.norm(st.dense() - b) <= 1e-12 * np.linalg.norm(b)


@pytest.mark.parametrize("n,eps,chi", [(4, 1e-3, 6), (5, 1e-4, 10), (5, 1e-8, 64)])
def test_mps_stepper_equals_dense_stepper(n, eps, chi):
    """The cores-based step and the dense TT-SVD step give the same rounded states."""
    N = 1 << n
    c2 = synth.layered_fault_velocity(n, dh=40.0) * (1e-3 / 40.0) ** 2 / 1e-6
    lam = 1e-3
    c2m = S.c2_mps(c2, n, 1e-6)
    c2d = M.to_dense(c2m).reshape(N, N)
    wav = synth.ricker(30, 1e-3, 25.0)
    st = S.MPSStepper(n, lam, eps, chi, c2m, src=(N // 2, 1), wavelet=wav * 1e3)
    ds = S.DenseStepper(n, lam, eps, chi, c2d, src=(N // 2, 1), wavelet=wav * 1e3)
    up, u = synth.random_fields(n, seed=1)
    st.set_fields(up, u)
    ds.set_fields(up, u)
    for _ in range(30):
        st.step()
        ds.step()
    d = ds.dense()
    assert np.linalg.norm(st.dense() - d) <= 1e-10 * np.linalg.norm(d)
    assert M.bonds_of(st.psi) == ds.ranks[-1][2]


@pytest.mark.parametrize("n,mx,mz", [(6, 2, 3), (8, 5, 1)])
def test_plane_wave_stays_rank_two(n, mx, mz):
    courant = 0.5
    N = 1 << n
    lam = courant
    c2 = np.ones((N, N))
    up, u = synth.plane_wave_fields(n, mx, mz, courant, phase=0.3)
    wdt = synth.fields.plane_wave_omega_dt(n, mx, mz, courant)
    ds = S.DenseStepper(n, lam, 1e-10, 16, c2)
    ds.set_fields(up, u)
    steps = 40
    for _ in range(steps):
        ds.step()
    x = np.arange(N)[:, None]
    z = np.arange(N)[None, :]
    exact = np.cos(2 * np.pi * (mx * x + mz * z) / N + 0.3 - steps * wdt)
    assert np.max(np.abs(ds.dense() - exact)) < 1e-10
    assert max(ds.ranks[-1][2]) == 2


@pytest.mark.parametrize("n,mx,mz", [(6, 2, 3), (8, 5, 1)])
def test_open_boundary_sine_mode_stays_rank_two(n, mx, mz):
    """Zero-fill shifts: a standing sine mode has quantics rank 2 (sin(a x + b)
    over the bits of x) and stays one, following its closed form."""
    courant = 0.5
    N = 1 << n
    c2 = np.ones((N, N))
    up, u = synth.sine_mode_fields(n, mx, mz, courant, phase=0.3)
    wdt = synth.fields.sine_mode_omega_dt(n, mx, mz, courant)
    ds = S.DenseStepper(n, courant, 1e-10, 16, c2, boundary="open")
    ms = S.MPSStepper(n, courant, 1e-10, 16, S.c2_mps(c2, n, 1e-12), boundary="open")
    _, v = synth.sine_mode_fields(n, mx, mz, courant)
    steps = 30
    for stepper in (ds, ms):
        stepper.set_fields(up, u)
        for _ in range(steps):
            stepper.step()
        assert np.max(np.abs(stepper.dense() - np.cos(0.3 - steps * wdt) * v)) < 1e-10
    assert max(ds.ranks[-1][2]) == 2
    assert max(c.shape[2] for c in ms.psi) == 2


def test_energy_conserved_untruncated_mps():
    n = 3
    N = 1 << n
    rng = np.random.default_rng(4)
    c2 = 0.5 + rng.random((N, N))
    lam = 0.5
    st = S.MPSStepper(n, lam, 0.0, 1 << 20, S.c2_mps(c2, n, 0.0))
    up, u = synth.random_fields(n, seed=2, smooth=False)
    st.set_fields(up, u)
    c2d = M.to_dense(st.c2).reshape(N, N)
    e0 = F.energy(st.dense(0), st.dense(1), c2d, lam)
    for _ in range(40):
        st.step()
        e = F.energy(st.dense(0), st.dense(1), c2d, lam)
        assert abs(e - e0) <= 1e-11 * abs(e0)


def test_zero_state_and_first_source_step():
    n = 3
    N = 1 << n
    c2 = np.ones((N, N))
    st = S.MPSStepper(n, 0.3, 1e-10, 8, S.c2_mps(c2, n, 1e-8), src=(2, 5),
                      wavelet=np.array([0.75, 0.0]))
    st.step()
    e = st.dense()
    assert e[2, 5] == pytest.approx(0.75, abs=1e-14) and np.count_nonzero(np.abs(e) > 1e-14) == 1
    assert M.bonds_of(st.psi) == [1] * (2 * n + 1)


def test_lambda_zero_linear_in_time():
    n = 3
    N = 1 << n
    st = S.MPSStepper(n, 0.0, 1e-12, 64, S.c2_mps(np.ones((N, N)), n, 1e-8))
    up, u = synth.random_fields(n, seed=5)
    st.set_fields(up, u)
    u0, um = st.dense(0).copy(), st.dense(1).copy()
    for k in range(1, 5):
        st.step()
        np.testing.assert_allclose(st.dense(), u0 + k * (u0 - um), atol=1e-10)
