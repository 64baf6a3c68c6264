"""Alternative compressions of an MPO-times-MPS product in FP64.  TEST INFRASTRUCTURE.

Sec. 4.3 asks for a compression after each operator application and does not
fix how.  The stepper's default forms the exact product (bonds multiply) and
rounds it (left-to-right QR sweep, right-to-left truncated SVD sweep:
``mps.round_mps``).  The two usual alternatives are written here:

* zip-up: the input is brought to right-orthonormal form, then the product is
  formed and truncated one site at a time from the left, so the product's full
  bonds never exist beyond one site;
* variational fitting: the bonds are fixed and each core in turn is replaced by the
  least-squares optimum against the exact product, with the others
  orthonormal, sweeping left and right (one-site alternating least squares);
  the bonds are the zip-up result's, which is also the starting point.

Both use the rounding's truncation rule (``mps.choose_rank``).  Cores are
(r_{k-1}, 2, r_k); MPO cores (w_left, w_right, s_out, s_in).
"""
import numpy as np

from . import mps as M


def right_orthonormal(cores):
    """The same MPS with cores 1..K-1 right-orthonormal (RQ sweep from the
    right, no truncation)."""
    G = [c.copy() for c in cores]
    for k in range(len(G) - 1, 0, -1):
        r0, d, r1 = G[k].shape
        Q, R = np.linalg.qr(G[k].reshape(r0, d * r1).T)   # G^T = Q R, so G = R^T Q^T
        G[k] = Q.T.reshape(Q.shape[1], d, r1)
        G[k - 1] = np.tensordot(G[k - 1], R.T, axes=(2, 0))
    return G


def mpo_sum(mpos, coeffs):
    """sum_t coeffs[t] W_t as one MPO (block-diagonal bonds, first core
    concatenated along its right bond, last along its left)."""
    K = len(mpos[0])
    out = []
    for k in range(K):
        blocks = [W[k] for W in mpos]
        if K == 1:
            out.append(sum(c * b for c, b in zip(coeffs, blocks)))
            continue
        wl = 1 if k == 0 else sum(b.shape[0] for b in blocks)
        wr = 1 if k == K - 1 else sum(b.shape[1] for b in blocks)
        C = np.zeros((wl, wr, 2, 2))
        i = j = 0
        for c, b in zip(coeffs, blocks):
            bl, br = b.shape[0], b.shape[1]
            scale = c if k == 0 else 1.0
            if k == 0:
                C[0:1, j:j + br] = scale * b
            elif k == K - 1:
                C[i:i + bl, 0:1] = b
            else:
                C[i:i + bl, j:j + br] = b
            i += bl
            j += br
        out.append(C)
    return out


def laplacian_mpo(n, boundary="periodic", ordering="sequential", ndim=2):
    """L = sum over axes of (S^+ + S^-) - 2 ndim I (eqs. 6, 14-16) as one MPO."""
    terms, coeffs = [], []
    for ax in range(ndim):
        for d in (+1, -1):
            terms.append(M.shift_mpo_nd(n, ax, d, boundary, ordering, ndim))
            coeffs.append(1.0)
    terms.append(M.identity_mpo(ndim * n))
    coeffs.append(-2.0 * ndim)
    return mpo_sum(terms, coeffs)


def diagonal_mpo(cores):
    """The diagonal MPO whose diagonal is the MPS `cores` (the c^2 operator):
    W[a, b, s', s] = C[a, s, b] if s' = s, else 0."""
    out = []
    for c in cores:
        r0, d, r1 = c.shape
        W = np.zeros((r0, r1, d, d))
        for s in range(d):
            W[:, :, s, s] = c[:, s, :]
        out.append(W)
    return out


def zip_up(W, cores, eps, chi_max, log=None):
    """Zip-up application of the MPO W to the MPS `cores`, truncating with the
    rounding's rule at every bond as the product is formed from the left.  The
    carry keeps the operator and state bonds apart (carry[r, w, i]), so no
    product core of the full bond w r is formed."""
    G = right_orthonormal(cores)
    K = len(G)
    out = []
    carry = np.ones((1, 1, 1))   # (new left bond, operator bond, state bond)
    for k in range(K):
        T = np.einsum("rwi,wxts,isj->rtxj", carry, W[k], G[k], optimize=True)   # (r, 2, wr, ir)
        r, d, wr, ir = T.shape
        if k == K - 1:
            out.append(T.reshape(r, d, wr * ir))
            break
        U, s, Vt = M.svd(T.reshape(r * d, wr * ir))
        keep = M.choose_rank(s, eps, chi_max)
        if log is not None:
            log.append((k + 1, s.copy(), keep))
        out.append(U[:, :keep].reshape(r, d, keep))
        carry = (s[:keep, None] * Vt[:keep]).reshape(keep, wr, ir)
    return out


def _grow_left(L, a, w, g):
    """Left environment one site further: L[a, w, i] -> L'[b, x, j]."""
    return np.einsum("awi,atb,wxts,isj->bxj", L, a, w, g, optimize=True)


def _grow_right(R, a, w, g):
    """Right environment one site further left: R[b, x, j] -> R'[a, w, i]."""
    return np.einsum("bxj,atb,wxts,isj->awi", R, a, w, g, optimize=True)


def variational(W, cores, eps, chi_max, sweeps=2, start=None):
    """Variational fit of W psi at fixed bonds: `start` (default: the zip-up
    result) as the first guess, then `sweeps` pairs of one-site least-squares
    sweeps (right to left, then left to right).  Each local update is the exact
    minimiser of ||phi - W psi|| over one core with the others orthonormal, so
    the distance never grows.  The environments keep the three layers (fit,
    operator, state) apart, so the exact product is never formed."""
    phi = [c.copy() for c in (start if start is not None else zip_up(W, cores, eps, chi_max))]
    K = len(phi)
    for k in range(K - 1):   # left-orthonormal cores 0..K-2, the centre at K-1
        r0, d, r1 = phi[k].shape
        Q, R = np.linalg.qr(phi[k].reshape(r0 * d, r1))
        phi[k] = Q.reshape(r0, d, Q.shape[1])
        phi[k + 1] = np.tensordot(R, phi[k + 1], axes=(1, 0))
    one = np.ones((1, 1, 1))
    left = [one]
    for k in range(K - 1):
        left.append(_grow_left(left[-1], phi[k], W[k], cores[k]))
    right = [None] * (K + 1)
    right[K] = one

    def update(k):
        return np.einsum("awi,wxts,isj,bxj->atb", left[k], W[k], cores[k], right[k + 1], optimize=True)

    for _ in range(sweeps):
        for k in range(K - 1, -1, -1):            # right to left
            phi[k] = update(k)
            if k > 0:                              # the centre moves left
                r0, d, r1 = phi[k].shape
                Q, Rm = np.linalg.qr(phi[k].reshape(r0, d * r1).T)
                phi[k] = Q.T.reshape(Q.shape[1], d, r1)
                phi[k - 1] = np.tensordot(phi[k - 1], Rm.T, axes=(2, 0))
                right[k] = _grow_right(right[k + 1], phi[k], W[k], cores[k])
        left = [one]
        for k in range(K):                         # left to right
            phi[k] = update(k)
            if k < K - 1:                          # the centre moves right
                r0, d, r1 = phi[k].shape
                Q, Rm = np.linalg.qr(phi[k].reshape(r0 * d, r1))
                phi[k] = Q.reshape(r0, d, Q.shape[1])
                phi[k + 1] = np.tensordot(Rm, phi[k + 1], axes=(1, 0))
                left.append(_grow_left(left[k], phi[k], W[k], cores[k]))
    return phi
