"""Seeded velocity models (input generators only).

The paper runs on a 256x256 subset of the Marmousi model (Sec. 5).  That data
set is not available here, so a seeded "Marmousi-like" layered model with a
dipping fault stands in for it.  Recipe (all lengths in metres, grid spacing
dh, square domain X = Z = N*dh, arrays indexed v[x, z] with x horizontal and z
depth, both 0-based, x_i = i*dh):

* water: v = 1500 m/s for z < 0.08 Z (flat water bottom);
* 12 layers below the water, velocities linear from 1700 to 4500 m/s; the top
  of layer l (l = 1..12) is z_l(x) = z0_l + A_l sin(2 pi x / L_l + phi_l) with
  z0_l = 0.08 Z + (l-1) * 0.92 Z / 12, A_l ~ U[10, 60] m, L_l ~ U[500, 2000] m,
  phi_l ~ U[0, 2 pi) drawn in that order from numpy default_rng(seed), A_1 = 0;
* one fault dipping at 60 degrees through (X/2, Z/2): on the hanging wall
  (x > x_f(z) = X/2 + (z - Z/2)/tan 60deg) the interfaces l >= 2 are 50 m deeper;
* Gaussian smoothing with sigma = 2 cells (mode "nearest") of v.

The model is returned as c^2 (m^2/s^2), the quantity the update uses.
"""
import numpy as np
from scipy.ndimage import gaussian_filter

N_LAYERS = 12
V_WATER = 1500.0
V_TOP, V_BOTTOM = 1700.0, 4500.0
WATER_FRACTION = 0.08
FAULT_THROW = 50.0
FAULT_DIP_DEG = 60.0
SMOOTH_SIGMA_CELLS = 2.0


def layered_fault_velocity(n, dh=10.0, seed=0, return_velocity=False):
    """c^2[x, z] (float64, shape (2^n, 2^n)) of the seeded layered-fault model."""
    N = 1 << n
    X = Z = N * dh
    rng = np.random.default_rng(seed)
    A = rng.uniform(10.0, 60.0, N_LAYERS)
    L = rng.uniform(500.0, 2000.0, N_LAYERS)
    phi = rng.uniform(0.0, 2.0 * np.pi, N_LAYERS)
    A[0] = 0.0
    v_layers = np.linspace(V_TOP, V_BOTTOM, N_LAYERS)
    z_water = WATER_FRACTION * Z
    z0 = z_water + np.arange(N_LAYERS) * (1.0 - WATER_FRACTION) * Z / N_LAYERS

    x = np.arange(N) * dh
    z = np.arange(N) * dh
    xx, zz = np.meshgrid(x, z, indexing="ij")          # [x, z]
    x_fault = X / 2 + (zz - Z / 2) / np.tan(np.deg2rad(FAULT_DIP_DEG))
    hanging = xx > x_fault

    v = np.full((N, N), V_WATER)
    for l in range(N_LAYERS):
        top = z0[l] + A[l] * np.sin(2.0 * np.pi * xx / L[l] + phi[l])
        if l >= 1:
            top = top + np.where(hanging, FAULT_THROW, 0.0)
        v = np.where(zz >= top, v_layers[l], v)
    v = gaussian_filter(v, sigma=SMOOTH_SIGMA_CELLS, mode="nearest")
    if return_velocity:
        return v
    return v * v


def layered_fault_velocity_3d(n, dh=10.0, seed=0):
    """c^2[x, y, z] (float64, shape (2^n,)*3): the layered-fault recipe on a
    cube.  After the draws of the two-dimensional model, each interface gets a
    second undulation along y, B_l sin(2 pi y / M_l + psi_l) with B_l ~ U[10, 40]
    m, M_l ~ U[500, 2000] m, psi_l ~ U[0, 2 pi) (B_1 = 0); the fault plane
    strikes along y; smoothing is the same Gaussian (sigma = 2 cells) in 3D."""
    N = 1 << n
    X = Z = N * dh
    rng = np.random.default_rng(seed)
    A = rng.uniform(10.0, 60.0, N_LAYERS)
    L = rng.uniform(500.0, 2000.0, N_LAYERS)
    phi = rng.uniform(0.0, 2.0 * np.pi, N_LAYERS)
    B = rng.uniform(10.0, 40.0, N_LAYERS)
    Ly = rng.uniform(500.0, 2000.0, N_LAYERS)
    psi = rng.uniform(0.0, 2.0 * np.pi, N_LAYERS)
    A[0] = 0.0
    B[0] = 0.0
    v_layers = np.linspace(V_TOP, V_BOTTOM, N_LAYERS)
    z_water = WATER_FRACTION * Z
    z0 = z_water + np.arange(N_LAYERS) * (1.0 - WATER_FRACTION) * Z / N_LAYERS
    c = np.arange(N) * dh
    xx, yy, zz = np.meshgrid(c, c, c, indexing="ij")     # [x, y, z]
    x_fault = X / 2 + (zz - Z / 2) / np.tan(np.deg2rad(FAULT_DIP_DEG))
    hanging = xx > x_fault
    v = np.full((N, N, N), V_WATER)
    for l in range(N_LAYERS):
        top = z0[l] + A[l] * np.sin(2.0 * np.pi * xx / L[l] + phi[l]) + B[l] * np.sin(2.0 * np.pi * yy / Ly[l] + psi[l])
        if l >= 1:
            top = top + np.where(hanging, FAULT_THROW, 0.0)
        v = np.where(zz >= top, v_layers[l], v)
    v = gaussian_filter(v, sigma=SMOOTH_SIGMA_CELLS, mode="nearest")
    return v * v


def constant_velocity(n, c=2000.0):
    """c^2 of a constant model (shape (2^n, 2^n))."""
    N = 1 << n
    return np.full((N, N), float(c) * float(c))
