"""The sensitivity floor of the precision workload (layered model, n = 6,
eps = 1e-6, 80 steps): the distance perturbations of rounding size make.

The floor is linear in the perturbation once it is above roundoff and the
same for any cutoff eps (it is how the scheme carries per-step errors, not
truncation decisions), and at FP32's unit roundoff it already exceeds 1e-6: a
1e-6 relative-L2 target for FP32 contractions is below what 80 steps of this
workload allow any FP32 arithmetic.
"""
import numpy as np
import pytest

from oracle import mps as M
from oracle import stepper as S
import synth
import sensitivity


@pytest.fixture(scope="module")
def workload():
    n, eps, chi, steps = 6, 1e-6, 64, 80
    N = 1 << n
    cfg = synth.get_config("C2", n=n, steps=steps)
    c2 = M.to_dense(S.c2_mps(cfg["c2"], n, cfg["eps_c"])).reshape(N, N)
    return dict(n=n, lam=cfg["lam"], eps=eps, chi=chi, c2=c2, src=(N // 2, 1),
                wav=synth.ricker(steps, cfg["dt"], 40.0), steps=steps)


def test_floor_is_linear_and_above_the_fp32_target(workload):
    f = {d: sensitivity.floor(delta=d, **workload) for d in (1e-7, 1e-5)}
    assert 30 < f[1e-5] / f[1e-7] < 300, f
    f32 = sensitivity.floor(delta=2.0 ** -24, **workload)
    assert f32 > 1e-6, f32


def test_zero_perturbation_has_zero_floor(workload):
    a = sensitivity.run(**workload)
    b = sensitivity.run(**workload, delta=0.0, seed=5)
    assert np.array_equal(a, b)


def test_floor_does_not_depend_on_the_cutoff(workload):
    d = 2.0 ** -20
    f6 = sensitivity.floor(delta=d, **workload)
    f12 = sensitivity.floor(delta=d, **dict(workload, eps=1e-12))
    assert abs(f12 / f6 - 1.0) < 0.1, (f6, f12)
