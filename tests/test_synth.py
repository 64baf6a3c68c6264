"""Checks of the seeded input generators (not part of the method)."""
import numpy as np

import synth


def test_ricker_shape():
    f0, dt = 15.0, 1e-4
    w = synth.ricker(4000, dt, f0)
    t0 = 1.5 / f0
    k0 = int(round(t0 / dt))
    assert abs(w[k0] - 1.0) < 1e-12 and np.argmax(w) == k0
    # zero crossings at t0 +- 1/(pi f0 sqrt 2)
    tz = t0 + 1.0 / (np.pi * f0 * np.sqrt(2.0))
    kz = int(tz / dt)
    assert w[kz] > 0 > w[kz + 1]


def test_layered_model_properties():
    n = 8
    v = synth.layered_fault_velocity(n, return_velocity=True)
    assert v.shape == (256, 256)
    assert abs(v[:, 0].mean() - 1500.0) < 1e-9          # water at the surface
    assert v.min() >= 1500.0 - 1e-9 and v.max() <= 4500.0 + 1e-9
    assert v[:, -1].mean() > 4000.0                     # deepest layer is fast
    v2 = synth.layered_fault_velocity(n, return_velocity=True)
    np.testing.assert_array_equal(v, v2)                # seeded
    c2 = synth.layered_fault_velocity(n)
    np.testing.assert_allclose(c2, v * v)


def test_configs_resolve():
    for name in ("C1", "C2", "C3"):
        cfg = synth.get_config(name)
        N = 1 << cfg["n"]
        assert cfg["c2"].shape == (N, N)
        # CFL: lambda^2 max(c^2) * 2 <= 1
        assert cfg["lam"] ** 2 * cfg["c2"].max() * 2 <= 1.0
