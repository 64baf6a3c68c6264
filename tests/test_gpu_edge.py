"""Degenerate and extreme cases of the HIP path against the FP64 oracle,
through the C ABI: the smallest grid (n = 1, two sites), a rank-one cap, a
field that is zero (sigma_1 = 0 at every bond), truncation by the cap alone
(eps = 0), a coarse cutoff, and the largest grid the library takes (n = 11)
with a closed-form solution.  Tolerances as in the other parity tests."""
import sys

import numpy as np
import pytest

from oracle import fdtd as F
from oracle import stepper as S
import synth
from helpers import oracle_velocity

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def mpsw():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    from paper_2609_01904_amd import mpsw as m
    m.load()
    return m


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


@pytest.mark.parametrize("boundary", [0, 1])
@pytest.mark.parametrize("ordering", [0, 1])
def test_two_site_grid_equals_fdtd(mpsw, boundary, ordering):
    """n = 1: one bit per register; the shift MPOs are single cores."""
    _say("n=1", boundary, ordering)
    n, lam = 1, 0.3
    rng = np.random.default_rng(5)
    c2 = 0.5 + rng.random((2, 2))
    wav = rng.standard_normal(8)
    st = mpsw.State(mpsw.make_config(n, 2, 0.0, lam, boundary=boundary, ordering=ordering))
    c2r = oracle_velocity(st, c2, 0.0, ordering)
    up, u = rng.standard_normal((2, 2)), rng.standard_normal((2, 2))
    st.set_fields(0, up, u)
    st.set_source(0, 1, 0, wav)
    a, b = up, u
    for k in range(8):
        st.step(1)
        a, b = b, F.fdtd_step(b, a, c2r, lam, wav[k], (1, 0), "periodic" if boundary == 0 else "open")
        assert rel(st.to_dense(0, 0), b) < 1e-12, k
    st.close()


def _against_dense_stepper(mpsw, n, chi, eps, steps, seed):
    N = 1 << n
    c2 = synth.layered_fault_velocity(n, dh=40.0) * 1e-8
    lam = 0.5
    wav = synth.ricker(steps, 0.004, 20.0)
    st = mpsw.State(mpsw.make_config(n, chi, eps, lam))
    c2r = oracle_velocity(st, c2, 1e-8)
    up, u = synth.random_fields(n, seed=seed)
    st.set_fields(0, up, u)
    src = (N // 3, 2)
    st.set_source(0, src[0], src[1], wav)
    ds = S.DenseStepper(n, lam, eps, chi, c2r, src=src, wavelet=wav)
    ds.set_fields(up, u)
    for k in range(steps):
        ds.step()
    st.step(steps)
    g = st.to_dense(0, 0)
    err = rel(g, ds.dense())
    _say(f"n={n} chi={chi} eps={eps}: rel-L2 {err:.2e}; bonds {st.bonds(0, 0)}")
    assert st.bonds(0, 0) == ds.ranks[-1][2]
    return err


def test_rank_one_cap(mpsw):
    assert _against_dense_stepper(mpsw, 5, 1, 0.0, 20, seed=11) < 1e-10


def test_cap_alone_truncates(mpsw):
    assert _against_dense_stepper(mpsw, 5, 6, 0.0, 25, seed=12) < 1e-10


def test_coarse_cutoff(mpsw):
    assert _against_dense_stepper(mpsw, 5, 32, 0.3, 25, seed=13) < 1e-10


def test_zero_field_stays_zero(mpsw):
    """No source and zero fields: every bond matrix is zero (sigma_1 = 0), the
    rule keeps one zero singular value and the field stays exactly zero."""
    n = 4
    st = mpsw.State(mpsw.make_config(n, 8, 1e-6, 0.5))
    st.set_velocity_dense(synth.layered_fault_velocity(n, dh=40.0) * 1e-8, 1e-8)
    st.step(5)
    g = st.to_dense(0, 0)
    assert np.all(g == 0.0)
    assert st.bonds(0, 0) == [1] * (2 * n + 1)
    st.close()


def test_largest_grid_plane_wave(mpsw):
    """n = 11 (2048 x 2048), the largest grid: a plane wave stays rank 2 and
    follows the closed-form dispersion relation."""
    n, mx, mz, courant = 11, 301, 77, 0.5
    N = 1 << n
    st = mpsw.State(mpsw.make_config(n, 8, 1e-10, courant))
    st.set_velocity_dense(np.ones((N, N)), 1e-12)
    up, u = synth.plane_wave_fields(n, mx, mz, courant, phase=0.4)
    st.set_fields(0, up, u)
    wdt = synth.fields.plane_wave_omega_dt(n, mx, mz, courant)
    steps = 10
    st.step(steps)
    x = np.arange(N)[:, None]
    z = np.arange(N)[None, :]
    exact = np.cos(2 * np.pi * (mx * x + mz * z) / N + 0.4 - steps * wdt)
    g = st.to_dense(0, 0)
    _say("plane wave n=11", np.max(np.abs(g - exact)), max(st.bonds(0, 0)))
    assert np.max(np.abs(g - exact)) < 1e-10
    assert max(st.bonds(0, 0)) == 2
    st.close()
