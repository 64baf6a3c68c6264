"""Source time functions (input generators only).

The paper uses an impulsive source of strength 1 (Sec. 5); the workloads here
also use Ricker wavelets r(t) = (1 - 2 pi^2 f0^2 (t-t0)^2) exp(-pi^2 f0^2 (t-t0)^2)
sampled at t_k = k*dt, k = 0..nt-1, with delay t0 = 1.5/f0 by default.  Sample k
is added at grid point (ix, iz) of u^{k+1} by the step that advances u^k.
"""
import numpy as np


def ricker(nt, dt, f0, t0=None):
    if t0 is None:
        t0 = 1.5 / f0
    t = np.arange(nt) * dt - t0
    a = (np.pi * f0 * t) ** 2
    return (1.0 - 2.0 * a) * np.exp(-a)


def impulse(nt):
    w = np.zeros(nt)
    if nt > 0:
        w[0] = 1.0
    return w
