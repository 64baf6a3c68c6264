"""Dense FDTD reference (Sec. 2, eq. 2) and its invariants.  TEST INFRASTRUCTURE.

u^{k+1}_{i,j} = 2 u^k_{i,j} - u^{k-1}_{i,j}
               + lambda^2 c^2_{i,j} (u^k_{i+1,j} + u^k_{i-1,j} + u^k_{i,j+1} + u^k_{i,j-1} - 4 u^k_{i,j})

with lambda = dt/dh.  Arrays are u[x, z] (x = i horizontal, z = j depth).  The
same update in three dimensions, u[x, y, z] with the seven-point sum
(- 6 u), is the 3D form the paper anticipates for its MPS solver; every
function here takes fields of either rank.  The boundary is not stated in the
paper; two readings are offered:

* "periodic": indices wrap mod 2^n (the cyclic shifts of Sec. 3.1 / Sec. 4.2);
* "open":     values outside the grid are zero (the terminal shift core of
              eq. 11 as printed, which drops the carry out of the top bit).

A point source adds s_k at (ix, iz) of u^{k+1}.
"""
import numpy as np


def _along(axis, ndim, sl):
    idx = [slice(None)] * ndim
    idx[axis] = sl
    return tuple(idx)


def shift_plus(u, axis, boundary):
    """(S^+ u)[x] = u[x-1]: the amplitude of |x> moves to |x+1> (eq. 5)."""
    if boundary == "periodic":
        return np.roll(u, 1, axis=axis)
    out = np.zeros_like(u)
    out[_along(axis, u.ndim, slice(1, None))] = u[_along(axis, u.ndim, slice(None, -1))]
    return out


def shift_minus(u, axis, boundary):
    """(S^- u)[x] = u[x+1]: the adjoint of S^+."""
    if boundary == "periodic":
        return np.roll(u, -1, axis=axis)
    out = np.zeros_like(u)
    out[_along(axis, u.ndim, slice(None, -1))] = u[_along(axis, u.ndim, slice(1, None))]
    return out


def laplacian(u, boundary="periodic"):
    """Five-point sum of eq. 2 (second row), in grid units (no 1/dh^2); the
    seven-point sum for a three-dimensional field."""
    out = shift_plus(u, 0, boundary) + shift_minus(u, 0, boundary)
    for ax in range(1, u.ndim):
        out = out + shift_plus(u, ax, boundary) + shift_minus(u, ax, boundary)
    return out - 2.0 * u.ndim * u


def fdtd_step(u, u_prev, c2, lam, s=0.0, src=None, boundary="periodic"):
    """One leapfrog step of eq. 2; returns u^{k+1}."""
    u_next = 2.0 * u - u_prev + (lam * lam) * c2 * laplacian(u, boundary)
    if src is not None and s != 0.0:
        u_next[tuple(src)] += s
    return u_next


def fdtd_run(u_prev, u, c2, lam, nsteps, wavelet=None, src=None, boundary="periodic",
             record=()):
    """Run nsteps; returns (u^{k-1}, u^k, {step: u^step for step in record})."""
    rec = {}
    for k in range(nsteps):
        s = 0.0 if wavelet is None else float(wavelet[k])
        u_prev, u = u, fdtd_step(u, u_prev, c2, lam, s, src, boundary)
        if (k + 1) in record:
            rec[k + 1] = u.copy()
    return u_prev, u, rec


def energy(u_next, u, c2, lam, boundary="periodic"):
    """Discrete energy E^{k+1/2} = <u^{k+1}-u^k, (u^{k+1}-u^k)/c^2> - lambda^2 <u^{k+1}, L u^k>.

    Conserved by eq. 2 without source for any symmetric L (both boundaries):
    taking the inner product of eq. 2 divided by c^2 with u^{k+1} - u^{k-1}
    telescopes to E^{k+1/2} = E^{k-1/2}.
    """
    d = u_next - u
    return float(np.sum(d * d / c2) - lam * lam * np.sum(u_next * laplacian(u, boundary)))


# ---------------------------------------------------------------------------
# Brute force: explicit 4^n x 4^n operators (n <= 4), built by index loops.
# ---------------------------------------------------------------------------

def brute_laplacian_matrix(n, boundary="periodic"):
    """The 5-point operator as a dense (4^n, 4^n) matrix, flat index x*2^n + z."""
    N = 1 << n
    L = np.zeros((N * N, N * N))
    for x in range(N):
        for z in range(N):
            row = x * N + z
            L[row, row] -= 4.0
            for dx, dz in ((1, 0), (-1, 0), (0, 1), (0, -1)):
                xx, zz = x + dx, z + dz
                if boundary == "periodic":
                    xx %= N
                    zz %= N
                elif not (0 <= xx < N and 0 <= zz < N):
                    continue
                L[row, xx * N + zz] += 1.0
    return L


def brute_transition_matrix(n, c2, lam, boundary="periodic"):
    """A = 2 I + lambda^2 C^2 L of eq. 7 as a dense matrix."""
    N = 1 << n
    L = brute_laplacian_matrix(n, boundary)
    C2 = np.diag(np.asarray(c2, dtype=np.float64).reshape(N * N))
    return 2.0 * np.eye(N * N) + lam * lam * C2 @ L
