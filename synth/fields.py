"""Initial fields and random tensor-train cores (input generators only).

Fields are float64 arrays u[x, z] of shape (2^n, 2^n).  The flat index of grid
point (x, z) is x*2^n + z, i.e. the quantics sites are the bits of x (most
significant first) followed by the bits of z (Sec. 3, eq. 3).
"""
import numpy as np


def plane_wave_omega_dt(n, mx, mz, courant):
    """omega*dt of the discrete plane wave with integer wave numbers (mx, mz).

    For the second-order leapfrog / 5-point scheme on a periodic 2^n grid with
    constant c and Courant number c*dt/dh, a discrete plane wave
    cos(kx*x*dh + kz*z*dh - k*omega*dt) is an exact solution iff
    sin^2(omega dt / 2) = courant^2 (sin^2(kx dh/2) + sin^2(kz dh/2)),
    kx*dh = 2 pi mx / 2^n (and likewise for z).
    """
    N = 1 << n
    sx = np.sin(np.pi * mx / N) ** 2
    sz = np.sin(np.pi * mz / N) ** 2
    arg = courant * np.sqrt(sx + sz)
    if arg > 1.0:
        raise ValueError("plane wave is unstable at this Courant number")
    return 2.0 * np.arcsin(arg)


def plane_wave_fields(n, mx, mz, courant, phase=0.0):
    """(u^{-1}, u^0) such that u^k = cos(theta - k omega dt) for all k >= -1."""
    N = 1 << n
    wdt = plane_wave_omega_dt(n, mx, mz, courant)
    x = np.arange(N)[:, None]
    z = np.arange(N)[None, :]
    theta = 2.0 * np.pi * (mx * x + mz * z) / N + phase
    return np.cos(theta + wdt), np.cos(theta)


def sine_mode_omega_dt(n, mx, mz, courant):
    """omega*dt of a standing sine mode on the 2^n grid with zero-fill (open)
    shifts: sin(pi mx (x+1)/(N+1)) sin(pi mz (z+1)/(N+1)) is an eigenvector of
    the 5-point Laplacian with that boundary, eigenvalue
    -4 (sin^2(pi mx / (2(N+1))) + sin^2(pi mz / (2(N+1)))), so
    sin^2(omega dt / 2) = courant^2 (sin^2(pi mx / (2(N+1))) + sin^2(pi mz / (2(N+1))))."""
    N = 1 << n
    s = courant ** 2 * (np.sin(np.pi * mx / (2 * (N + 1))) ** 2 + np.sin(np.pi * mz / (2 * (N + 1))) ** 2)
    return 2.0 * np.arcsin(np.sqrt(s))


def sine_mode_fields(n, mx, mz, courant, phase=0.0):
    """(u^{-1}, u^0) such that u^k = cos(phase - k omega dt) v for all k >= -1,
    v the standing sine mode (mx, mz) of the open boundary."""
    N = 1 << n
    wdt = sine_mode_omega_dt(n, mx, mz, courant)
    x = np.arange(N)[:, None]
    z = np.arange(N)[None, :]
    v = np.sin(np.pi * mx * (x + 1) / (N + 1)) * np.sin(np.pi * mz * (z + 1) / (N + 1))
    return np.cos(phase + wdt) * v, np.cos(phase) * v


def random_fields(n, seed=0, smooth=True):
    """Two seeded smooth random fields (u^{-1}, u^0)."""
    rng = np.random.default_rng(seed)
    N = 1 << n
    out = []
    for _ in range(2):
        f = rng.standard_normal((N, N))
        if smooth:
            k = np.fft.fftfreq(N)
            filt = np.exp(-(k[:, None] ** 2 + k[None, :] ** 2) * 200.0)
            f = np.real(np.fft.ifft2(np.fft.fft2(f) * filt))
        out.append(f)
    return out[0], out[1]


def random_mps_cores(K, bonds, seed=0):
    """Seeded random cores, core k of shape (bonds[k], 2, bonds[k+1]).

    bonds has K+1 entries with bonds[0] = bonds[K] = 1.
    """
    assert len(bonds) == K + 1 and bonds[0] == 1 and bonds[K] == 1
    rng = np.random.default_rng(seed)
    return [rng.standard_normal((bonds[k], 2, bonds[k + 1])) / np.sqrt(2 * bonds[k])
            for k in range(K)]


def wavefront_fields_3d(n, seed=0, nfronts=48, dh=10.0, dt=1e-3, f0=15.0, vmin=1500.0, vmax=4500.0):
    """(u^{-1}, u^0) on a cube: the same recipe as wavefront_fields with
    spherical fronts (centres uniform over the cube, amplitude a_j / (R_j / dh)
    for spherical spreading)."""
    rng = np.random.default_rng(seed)
    N = 1 << n
    X = N * dh
    cen = rng.uniform(0.0, X, (nfronts, 3))
    R = rng.uniform(0.05 * X, 0.8 * X, nfronts)
    c = rng.uniform(vmin, vmax, nfronts)
    amp = rng.uniform(0.5, 1.0, nfronts) * rng.choice([-1.0, 1.0], nfronts)
    g = np.arange(N) * dh
    x, y, z = g[:, None, None], g[None, :, None], g[None, None, :]
    out = []
    for t in (-dt, 0.0):
        u = np.zeros((N, N, N))
        for j in range(nfronts):
            dist = np.sqrt((x - cen[j, 0]) ** 2 + (y - cen[j, 1]) ** 2 + (z - cen[j, 2]) ** 2)
            tau = (dist - R[j] - c[j] * t) / c[j]
            a = (np.pi * f0 * tau) ** 2
            u += amp[j] / (R[j] / dh) * (1.0 - 2.0 * a) * np.exp(-a)
        out.append(u)
    return out[0], out[1]


def wavefront_fields(n, seed=0, nfronts=48, dh=10.0, dt=1e-3, f0=15.0, vmin=1500.0, vmax=4500.0):
    """(u^{-1}, u^0) of a developed wavefield: a seeded superposition of
    expanding circular Ricker wavefronts.

    Front j has centre p_j (uniform over the grid), radius R_j, speed c_j and
    amplitude a_j / sqrt(R_j / dh) (cylindrical spreading); its profile is the
    Ricker shape of the travel-time offset tau = (|p - p_j| - R_j - c_j t) / c_j.
    u^0 is the field at t = 0 and u^{-1} at t = -dt.  Used as a saturated
    starting state (all bonds at the chi cap) for timing steady-state steps.
    """
    rng = np.random.default_rng(seed)
    N = 1 << n
    X = N * dh
    cx = rng.uniform(0.0, X, nfronts)
    cz = rng.uniform(0.0, X, nfronts)
    R = rng.uniform(0.05 * X, 0.8 * X, nfronts)
    c = rng.uniform(vmin, vmax, nfronts)
    amp = rng.uniform(0.5, 1.0, nfronts) * rng.choice([-1.0, 1.0], nfronts)
    x = (np.arange(N) * dh)[:, None]
    z = (np.arange(N) * dh)[None, :]
    out = []
    for t in (-dt, 0.0):
        u = np.zeros((N, N))
        for j in range(nfronts):
            dist = np.sqrt((x - cx[j]) ** 2 + (z - cz[j]) ** 2)
            tau = (dist - R[j] - c[j] * t) / c[j]
            a = (np.pi * f0 * tau) ** 2
            u += amp[j] / np.sqrt(R[j] / dh) * (1.0 - 2.0 * a) * np.exp(-a)
        out.append(u)
    return out[0], out[1]
