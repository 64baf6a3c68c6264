"""Named workloads (pure data plus seeded generators; no solver arithmetic).

Parameters follow the paper's run (Sec. 5: dh = dx = dz = 10 m, dt = 1 ms,
chi_max = 128, SVD cutoff 1e-7, 300 steps, source at the grid centre) and the
workload list this library is measured on:

* C0  paper replica: n=8, layered-fault model, impulse at (128, 128), 300 steps,
      eps = 1e-7, chi = 128.
* C1  n=6, constant c = 2000 m/s, c dt/dh = 0.5, Ricker 15 Hz (t0 = 0.1 s) at the
      centre, 200 steps, eps = 1e-10, chi = 32.
* C2  n=8, layered-fault model, c^2 MPO cutoff 1e-6, Ricker 15 Hz at 10 m depth,
      1000 steps, chi = 64, eps = 1e-7 (the paper's cutoff).
* C3  n=10, same model family, 2000 steps, chi = 128, eps = 1e-6.
* C4  64 shots, n in {8, 9, 10}, chi in {32, 64, 128}, Ricker f0 ~ U[8, 25] Hz at
      random x, depth 10 m, 1000 steps, eps = 1e-6.
* C5  n=11, chi = 256, eps = 1e-6, 3000 steps.
* C3D three-dimensional form: 128^3 cube (n=7, K = 21 sites), layered-fault
      model with undulations along y, Ricker 15 Hz at the top centre, chi = 64,
      eps = 1e-6, dt = 1 ms (c dt/dh <= 0.45 < 1/sqrt(3)).
"""
import numpy as np

from .velocity import layered_fault_velocity, layered_fault_velocity_3d, constant_velocity
from .wavelet import ricker, impulse

DH = 10.0
DT = 1e-3

CONFIGS = {
    "C0": dict(n=8, dh=DH, dt=DT, model="layered_fault", seed=0, src=("center",),
               wavelet="impulse", steps=300, eps=1e-7, chi=128, eps_c=1e-6),
    "C1": dict(n=6, dh=DH, dt=2.5e-3, model="constant", c=2000.0, src=("center",),
               wavelet="ricker", f0=15.0, steps=200, eps=1e-10, chi=32, eps_c=1e-6),
    "C2": dict(n=8, dh=DH, dt=DT, model="layered_fault", seed=0, src=("depth", 1),
               wavelet="ricker", f0=15.0, steps=1000, eps=1e-7, chi=64, eps_c=1e-6),
    "C3": dict(n=10, dh=DH, dt=DT, model="layered_fault", seed=0, src=("depth", 1),
               wavelet="ricker", f0=15.0, steps=2000, eps=1e-6, chi=128, eps_c=1e-6),
    "C5": dict(n=11, dh=DH, dt=DT, model="layered_fault", seed=0, src=("depth", 1),
               wavelet="ricker", f0=15.0, steps=3000, eps=1e-6, chi=256, eps_c=1e-6),
    "C3D": dict(n=7, ndim=3, dh=DH, dt=DT, model="layered_fault_3d", seed=0, src=("depth", 1),
                wavelet="ricker", f0=15.0, steps=1000, eps=1e-6, chi=64, eps_c=1e-6),
}


def get_config(name, **overrides):
    """Resolved workload: dict with c2 (dense), wavelet, source index, lambda."""
    cfg = dict(CONFIGS[name])
    cfg.update(overrides)
    n = cfg["n"]
    N = 1 << n
    if cfg["model"] == "constant":
        c2 = constant_velocity(n, cfg["c"])
    elif cfg["model"] == "layered_fault_3d":
        c2 = layered_fault_velocity_3d(n, cfg["dh"], cfg.get("seed", 0))
    else:
        c2 = layered_fault_velocity(n, cfg["dh"], cfg.get("seed", 0))
    kind = cfg["src"]
    if kind[0] == "center":
        ix, iz = N // 2, N // 2
    elif kind[0] == "depth":
        ix, iz = N // 2, int(kind[1])
    else:
        ix, iz = int(kind[1]), int(kind[2])
    nt = cfg["steps"]
    if cfg["wavelet"] == "ricker":
        w = ricker(nt, cfg["dt"], cfg["f0"])
    else:
        w = impulse(nt)
    cfg.setdefault("ndim", 2)
    if cfg["ndim"] == 3:
        cfg["iy"] = N // 2
    cfg.update(c2=c2, ix=ix, iz=iz, wavelet_samples=w, lam=cfg["dt"] / cfg["dh"])
    return cfg


def batch_shots(nshots=64, seed=1, steps=1000):
    """Shot list of the batched workload: n ~ U{8,9,10}, chi ~ U{32,64,128},
    f0 ~ U[8, 25] Hz, source x ~ U{0..N-1} at depth index 1."""
    rng = np.random.default_rng(seed)
    shots = []
    for _ in range(nshots):
        n = int(rng.choice([8, 9, 10]))
        chi = int(rng.choice([32, 64, 128]))
        f0 = float(rng.uniform(8.0, 25.0))
        ix = int(rng.integers(0, 1 << n))
        shots.append(dict(n=n, chi=chi, f0=f0, ix=ix, iz=1, steps=steps, eps=1e-6,
                          dt=DT, dh=DH, wavelet_samples=ricker(steps, DT, f0)))
    return shots
