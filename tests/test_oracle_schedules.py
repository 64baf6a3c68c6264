"""Pins of the alternative rounding schedules of the oracle stepper (Sec. 4.3:
a compression after operator applications; "three" roundings per step as in
eq. 17, "seven" with a rounding after each shift-operator application, "one"
with only the update sum rounded).  Without truncation every schedule is eq. 2
exactly; with a small bond cap a plane wave (quantics rank 2, so every
intermediate of every schedule is exactly representable) still follows its
closed-form dispersion relation."""
import numpy as np
import pytest

from oracle import fdtd as F
from oracle import mps as M
from oracle import stepper as S
import synth


@pytest.mark.parametrize("schedule", S.SCHEDULES)
@pytest.mark.parametrize("boundary", ["periodic", "open"])
def test_untruncated_schedules_equal_eq2(schedule, boundary):
    n, lam = 3, 0.4
    N = 1 << n
    rng = np.random.default_rng(3)
    c2 = 0.5 + rng.random((N, N))
    wav = rng.standard_normal(5)
    src = (N // 2, 1)
    st = S.MPSStepper(n, lam, 0.0, 1 << 20, S.c2_mps(c2, n, 0.0), boundary, src=src, wavelet=wav,
                      schedule=schedule)
    up, u = synth.random_fields(n, seed=4, smooth=False)
    st.set_fields(up, u)
    a, b = up, u
    for k in range(5):
        st.step()
        a, b = b, F.fdtd_step(b, a, c2, lam, wav[k], src, boundary)
        assert np.linalg.norm(st.dense() - b) <= 1e-12 * np.linalg.norm(b), k


@pytest.mark.parametrize("schedule", S.SCHEDULES)
def test_plane_wave_under_a_small_cap(schedule):
    n, mx, mz, courant = 5, 3, 7, 0.5
    N = 1 << n
    st = S.MPSStepper(n, courant, 1e-12, 4, S.c2_mps(np.ones((N, N)), n, 1e-12), schedule=schedule)
    up, u = synth.plane_wave_fields(n, mx, mz, courant, phase=0.3)
    st.set_fields(up, u)
    wdt = synth.fields.plane_wave_omega_dt(n, mx, mz, courant)
    steps = 12
    for _ in range(steps):
        st.step()
    x = np.arange(N)[:, None]
    z = np.arange(N)[None, :]
    exact = np.cos(2 * np.pi * (mx * x + mz * z) / N + 0.3 - steps * wdt)
    assert np.max(np.abs(st.dense() - exact)) < 1e-11
    assert max(M.bonds_of(st.psi)) == 2


def test_seven_rounds_each_shift():
    """The literal schedule logs 2 ndim shift roundings (tag 3) per step besides
    the three of eq. 17; the others log none."""
    n = 3
    N = 1 << n
    c2 = S.c2_mps(np.ones((N, N)), n, 1e-12)
    counts = {}
    for sch in S.SCHEDULES:
        st = S.MPSStepper(n, 0.3, 1e-8, 16, c2, schedule=sch)
        up, u = synth.random_fields(n, seed=1)
        st.set_fields(up, u)
        st.step()
        counts[sch] = sorted({(w, site) for (_, w, site, _, _) in st.log if w == 3})
    K = 2 * n
    assert len(counts["seven"]) == K - 1   # one log entry per bond of one tag
    assert counts["three"] == [] and counts["one"] == []
    with pytest.raises(ValueError):
        S.MPSStepper(n, 0.3, 1e-8, 16, c2, schedule="five")
