"""Parity of the HIP path in the interleaved site order (x_{n-1} z_{n-1} ...
x_0 z_0) with the FP64 oracle in the same order, through the C ABI: the
velocity operator and the dense field layout, eq. 2 when nothing is cut
(Table 1), each of the three roundings, a truncated trajectory, a plane wave
at the measured grid size and one step of the measured workload.  Tolerances
as in the sequential-order parity tests (1e-10 relative L2 truncated, 1e-12
untruncated)."""
import sys

import numpy as np
import pytest

from oracle import fdtd as F
from oracle import mps as M
from oracle import stepper as S
import synth
from helpers import oracle_c2, oracle_velocity

pytestmark = pytest.mark.gpu
IL = "interleaved"


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


def make_state(mpsw, n, chi, eps, lam, boundary=0):
    return mpsw.State(mpsw.make_config(n, chi, eps, lam, boundary=boundary, ordering=mpsw.MPSW_INTERLEAVED))


def test_velocity_and_fields_interleaved(mpsw):
    for n in (4, 6, 8, 10):
        _say("interleaved velocity", n)
        c2 = synth.layered_fault_velocity(n)
        st = make_state(mpsw, n, 16, 1e-8, 1e-4)
        st.set_velocity_dense(c2, 1e-6)
        ref = S.c2_mps(c2, n, 1e-6, IL)
        assert st.bonds(0, 2) == M.bonds_of(ref)
        assert rel(st.to_dense(0, 2), M.from_sites(M.to_dense(ref), n, IL)) < 1e-12
        st.close()
    n = 5
    st = make_state(mpsw, n, 1 << n, 0.0, 0.1)
    c2 = synth.layered_fault_velocity(n) * 1e-8
    ref = S.c2_mps(c2, n, 1e-10, IL)
    st.set_velocity_mpo(M.bonds_of(ref), ref)
    assert rel(st.to_dense(0, 2), M.from_sites(M.to_dense(ref), n, IL)) < 1e-13
    up, u = synth.random_fields(n, seed=3, smooth=False)
    st.set_fields(0, up, u)
    assert rel(st.to_dense(0, 0), u) < 1e-13
    assert rel(st.to_dense(0, 1), up) < 1e-13
    st.close()


@pytest.mark.parametrize("n", [3, 4])
@pytest.mark.parametrize("boundary", [0, 1])
def test_untruncated_interleaved_step_equals_fdtd(mpsw, n, boundary):
    _say("interleaved untruncated", n, boundary)
    N = 1 << n
    rng = np.random.default_rng(20 + n)
    c2 = 0.5 + rng.random((N, N))
    lam = 0.4
    wav = rng.standard_normal(10)
    src = (N // 2 + 1, 1)
    st = make_state(mpsw, n, 1 << n, 0.0, lam, boundary)
    c2r = oracle_velocity(st, c2, 0.0, IL)
    up, u = synth.random_fields(n, seed=n, smooth=False)
    st.set_fields(0, up, u)
    st.set_source(0, src[0], src[1], wav)
    a, b = up, u
    bname = "periodic" if boundary == 0 else "open"
    for k in range(10):
        st.step(1)
        a, b = b, F.fdtd_step(b, a, c2r, lam, wav[k], src, bname)
        assert rel(st.to_dense(0, 0), b) < 1e-12, k
    st.close()


def test_each_rounding_matches_oracle_interleaved(mpsw):
    n, chi, eps = 5, 12, 1e-6
    c2 = synth.layered_fault_velocity(n, dh=40.0) * 1e-8
    lam = 0.5
    c2m = S.c2_mps(c2, n, 1e-8, IL)
    st = make_state(mpsw, n, chi, eps, lam)
    st.set_velocity_mpo(M.bonds_of(c2m), c2m)
    up, u = synth.random_fields(n, seed=7)
    st.set_fields(0, up, u)
    psi = M.tt_svd(M.to_sites(u, IL), 2 * n, eps, chi)
    psip = M.tt_svd(M.to_sites(up, IL), 2 * n, eps, chi)
    st.step(1)
    y = M.round_mps(M.laplacian_mps(psi, n, "periodic", IL), eps, chi)
    w = M.round_mps(M.hadamard(c2m, y), eps, chi)
    nxt = M.round_mps(M.direct_sum([psi, psip, w], [2.0, -1.0, lam * lam]), eps, chi)
    for which, ref in ((3, y), (4, w), (0, nxt)):
        assert st.bonds(0, which) == M.bonds_of(ref), which
        assert rel(st.to_dense(0, which), M.from_sites(M.to_dense(ref), n, IL)) < 1e-11, which
    st.close()


def test_c2_prefix_matches_oracle_interleaved(mpsw):
    steps = 40
    cfg = synth.get_config("C2", steps=steps)
    n = cfg["n"]
    st = make_state(mpsw, n, cfg["chi"], cfg["eps"], cfg["lam"])
    c2r = oracle_velocity(st, cfg["c2"], cfg["eps_c"], IL)
    st.set_source(0, cfg["ix"], cfg["iz"], cfg["wavelet_samples"])
    ds = S.DenseStepper(n, cfg["lam"], cfg["eps"], cfg["chi"], c2r, src=(cfg["ix"], cfg["iz"]),
                        wavelet=cfg["wavelet_samples"], ordering=IL)
    for _ in range(steps):
        ds.step()
    st.step(steps)
    g = st.to_dense(0, 0)
    _say("C2 prefix, interleaved", rel(g, ds.dense()), st.bonds(0, 0))
    assert rel(g, ds.dense()) < 1e-10
    assert st.bonds(0, 0) == ds.ranks[-1][2]
    st.close()


def test_plane_wave_production_size_interleaved(mpsw):
    """n = 10: a plane wave is a product of per-bit phases in any site order, so
    it stays rank 2 and follows the closed-form dispersion relation."""
    n, mx, mz, courant = 10, 17, 5, 0.5
    N = 1 << n
    st = make_state(mpsw, n, 8, 1e-10, courant)
    st.set_velocity_dense(np.ones((N, N)), 1e-12)
    up, u = synth.plane_wave_fields(n, mx, mz, courant, phase=0.2)
    st.set_fields(0, up, u)
    wdt = synth.fields.plane_wave_omega_dt(n, mx, mz, courant)
    steps = 20
    st.step(steps)
    x = np.arange(N)[:, None]
    z = np.arange(N)[None, :]
    exact = np.cos(2 * np.pi * (mx * x + mz * z) / N + 0.2 - steps * wdt)
    g = st.to_dense(0, 0)
    _say("plane wave n=10, interleaved", np.max(np.abs(g - exact)), max(st.bonds(0, 0)))
    assert np.max(np.abs(g - exact)) < 1e-10
    assert max(st.bonds(0, 0)) == 2
    st.close()


def test_c3_step_matches_oracle_interleaved(mpsw):
    """The measured workload (n = 10, chi = 128, eps = 1e-6) in the interleaved
    order, 4 shots from developed wavefields: after a warm-up step, two sampled
    shots' next step against the oracle step from the same fields."""
    import torch
    import bench
    cfg0 = synth.get_config("C3")
    bonds, cores, c2r = oracle_c2(cfg0["c2"], cfg0["eps_c"], IL)
    st, cfg, fields = bench.make_state(mpsw, synth, "C3", 4, "fp64", ordering=IL, velocity=(bonds, cores))
    st.step(1)
    torch.cuda.synchronize()
    n = cfg["n"]
    sample = [0, 3]
    before = {s: (st.to_dense(s, 1), st.to_dense(s, 0), st.stats(s)["step"]) for s in sample}
    st.step(1)
    torch.cuda.synchronize()
    for s in sample:
        up, u, k = before[s]
        ds = S.DenseStepper(n, cfg["lam"], cfg["eps"], cfg["chi"], c2r, src=fields[s][2],
                            wavelet=cfg["wavelet_samples"], ordering=IL)
        ds.u_prev, ds.u, ds.k = up, u, k
        ds.step()
        g = st.to_dense(s, 0)
        err = rel(g, ds.dense())
        _say(f"C3 interleaved shot {s} (step {k + 1}): rel-L2 vs oracle {err:.2e}; bonds {st.bonds(s, 0)}")
        assert err < 1e-10, (s, err)
        assert st.bonds(s, 0) == ds.ranks[-1][2], s
    st.close()
