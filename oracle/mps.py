"""Quantics MPS arithmetic in FP64.  TEST INFRASTRUCTURE.

Representation (Sec. 4.1, eq. 8): a field on a 2^n x 2^n grid is a tensor with
K = 2n binary indices; sites 1..n are the bits x_{n-1} .. x_0 of the horizontal
index (most significant first) and sites n+1..2n the bits z_{n-1} .. z_0
(eq. 3).  This is exactly the C-order reshape of u[x, z] to [2]*K.  Core k is a
real array G_k of shape (r_{k-1}, 2, r_k) with r_0 = r_K = 1 (the fields are
real, so the complex cores of eq. 8 are not needed).

A second site order, "interleaved", pairs the bits of equal significance:
sites x_{n-1}, z_{n-1}, x_{n-2}, z_{n-2}, ..., x_0, z_0.  It represents the same
fields (the paper fixes the register order of eq. 3; the interleaved order is
the usual alternative for quantics grids and changes only the ranks needed).

Three-dimensional fields u[x, y, z] use K = 3n sites in the same way (three
registers, sequential or interleaved); the functions taking ``ndim`` default
to the paper's two dimensions.

An MPO core has shape (w_left, w_right, 2, 2) indexed [a_l, a_r, s_out, s_in].
"""
import numpy as np

# Local operators (matrices [s_out, s_in]).
I2 = np.eye(2)
SIGMA_PLUS = np.array([[0.0, 0.0], [1.0, 0.0]])   # |1><0|
SIGMA_MINUS = np.array([[0.0, 1.0], [0.0, 0.0]])  # |0><1|


# ---------------------------------------------------------------------------
# dense <-> cores
# ---------------------------------------------------------------------------

ORDERINGS = ("sequential", "interleaved")


def site_bits(n, ordering="sequential", ndim=2):
    """(register, bit) of each of the K = ndim n sites; registers 0.. are the
    axes (x, z in two dimensions; x, y, z in three) and bit is the significance
    (n-1 = most significant)."""
    if ordering == "sequential":
        return [(r, n - 1 - m) for r in range(ndim) for m in range(n)]
    if ordering == "interleaved":
        return [(r, n - 1 - m) for m in range(n) for r in range(ndim)]
    raise ValueError(ordering)


def to_sites(u, ordering="sequential"):
    """Flat tensor over the sites (C order over [2]*K) of the field u[x, z]
    (or u[x, y, z])."""
    u = np.asarray(u)
    n = int(u.shape[0]).bit_length() - 1
    t = u.reshape([2] * (u.ndim * n))     # axes x_{n-1}..x_0, then the next register
    axes = [r * n + (n - 1 - b) for r, b in site_bits(n, ordering, u.ndim)]
    return np.transpose(t, axes).reshape(-1)


def from_sites(v, n, ordering="sequential", ndim=2):
    """Inverse of to_sites: the field (2^n per axis) of a site-order tensor."""
    axes = [r * n + (n - 1 - b) for r, b in site_bits(n, ordering, ndim)]
    t = np.asarray(v).reshape([2] * (ndim * n))
    return np.transpose(t, np.argsort(axes)).reshape((1 << n,) * ndim)


def to_dense(cores):
    """Contract the chain; returns the flat vector of length 2^K."""
    v = np.ones((1, 1))
    for G in cores:
        r0, d, r1 = G.shape
        v = (v @ G.reshape(r0, d * r1)).reshape(-1, r1)
    return v.reshape(-1)


def bonds_of(cores):
    return [cores[0].shape[0]] + [G.shape[2] for G in cores]


def choose_rank(s, eps, chi_max):
    """Truncation rule of Sec. 4.3: discard sigma_i < eps * sigma_max, cap at chi_max.

    At least one singular value is kept; an all-zero matrix keeps rank 1 (its
    kept factor is zero, so the tensor stays zero).
    """
    if s.size == 0:
        return 1
    if s[0] <= 0.0:
        return 1
    r = int(np.count_nonzero(s >= eps * s[0]))
    return max(1, min(r, chi_max))


# Sensitivity windows of a cut.  Two backward-stable FP64 factorisations of
# the same matrix, or of two matrices that differ by rounding, agree on every
# sigma_i to about delta = 1e-14 sigma_1.  A cut is flagged when a change of
# that size could alter what is kept by more than about 1e-11 of the tensor:
TAU_GAP = 1e-3     # cap cut: kept and first discarded value closer than this, relative to the kept one
TAU_CUT = 1e-13    # a value this close to the cutoff eps * sigma_1, relative to sigma_1


def cut_flags(s, r, eps):
    """Why the truncation of the descending spectrum s at rank r is not decided
    with a margin against rounding (Sec. 4.3's rule is discontinuous in sigma):
    a set of

    'gap'  the cap cuts (more than r values pass the cutoff) and
           sigma_r - sigma_{r+1} < TAU_GAP sigma_r: the kept subspace turns by
           about delta / gap under a perturbation delta, which changes the kept
           part by about sigma_r delta / gap;
    'cut'  some |sigma_i - eps sigma_1| < TAU_CUT sigma_1: that value can fall
           on either side of the cutoff, a jump of about eps sigma_1.

    Exactly equal values that the cutoff keeps or drops together are no
    ambiguity; only a cut between them is.  Empty when the cut is decided with
    a margin.
    """
    s = np.asarray(s, dtype=np.float64)
    out = set()
    if s.size == 0 or s[0] <= 0.0:
        return out
    capped = r < s.size and (s[r] >= eps * s[0])
    if capped and s[r - 1] - s[r] < TAU_GAP * s[r - 1]:
        out.add("gap")
    if eps > 0.0 and np.any(np.abs(s - eps * s[0]) < TAU_CUT * s[0]):
        out.add("cut")
    return out


def svd(M):
    """Thin SVD (U, s, Vt) of M.  LAPACK's divide-and-conquer driver (numpy's)
    fails to converge on rare matrices; the QR-iteration driver then computes
    the same decomposition."""
    try:
        return np.linalg.svd(M, full_matrices=False)
    except np.linalg.LinAlgError:
        import scipy.linalg
        return scipy.linalg.svd(M, full_matrices=False, lapack_driver="gesvd")


def tt_svd(t, K, eps, chi_max, log=None):
    """Right-to-left truncated TT-SVD of a dense tensor with 2^K entries.

    Moving from the last site to the first, the current tensor is unfolded as
    (2^{k-1}, 2 r_k), its SVD is truncated with ``choose_rank`` and the kept
    right singular vectors become core k; U_r Sigma_r carries on to the left.
    This is the sequential-SVD construction of Sec. 4.1 and, applied to an
    arbitrary tensor, the definition of the rounding used below.
    """
    X = np.asarray(t, dtype=np.float64).reshape(-1, 1)
    cores = [None] * K
    rho = 1
    for k in range(K - 1, 0, -1):
        M = X.reshape(-1, 2 * rho)
        U, s, Vt = svd(M)
        r = choose_rank(s, eps, chi_max)
        if log is not None:
            log.append((k, s.copy(), r))
        cores[k] = Vt[:r].reshape(r, 2, rho)
        X = U[:, :r] * s[:r]
        rho = r
    cores[0] = X.reshape(1, 2, rho)
    return cores


def round_mps(cores, eps, chi_max, log=None):
    """Compression of Sec. 4.3: left-to-right QR sweep, then right-to-left SVD sweep.

    The QR sweep makes cores 1..K-1 left-orthonormal (Householder QR of the
    (2 r_{k-1}, r_k) unfolding, R pushed into the next core).  The SVD sweep then
    factors each (r_{k-1}, 2 r_k) unfolding, keeps the right singular vectors
    selected by ``choose_rank`` as core k and pushes U_r Sigma_r into core k-1.
    """
    G = [c.copy() for c in cores]
    K = len(G)
    for k in range(K - 1):
        r0, d, r1 = G[k].shape
        Q, R = np.linalg.qr(G[k].reshape(r0 * d, r1))
        G[k] = Q.reshape(r0, d, Q.shape[1])
        G[k + 1] = np.tensordot(R, G[k + 1], axes=(1, 0))
    for k in range(K - 1, 0, -1):
        r0, d, r1 = G[k].shape
        U, s, Vt = svd(G[k].reshape(r0, d * r1))
        r = choose_rank(s, eps, chi_max)
        if log is not None:
            log.append((k, s.copy(), r))
        G[k] = Vt[:r].reshape(r, d, r1)
        G[k - 1] = np.tensordot(G[k - 1], U[:, :r] * s[:r], axes=(2, 0))
    return G


# ---------------------------------------------------------------------------
# MPS algebra
# ---------------------------------------------------------------------------

def zero_mps(K):
    return [np.zeros((1, 2, 1)) for _ in range(K)]


def product_state(bits):
    """Basis state |b_1 ... b_K> as a bond-1 MPS."""
    cores = []
    for b in bits:
        G = np.zeros((1, 2, 1))
        G[0, b, 0] = 1.0
        cores.append(G)
    return cores


def point_state(n, ix, iz, ordering="sequential"):
    """e_(ix, iz): sites are the bits of ix (MSB first) then of iz (eq. 3), or
    the two interleaved."""
    return point_state_nd(n, (ix, iz), ordering)


def point_state_nd(n, coords, ordering="sequential"):
    """The basis field at grid point coords (one index per axis)."""
    return product_state([(coords[r] >> b) & 1 for r, b in site_bits(n, ordering, len(coords))])


def scale(cores, alpha):
    out = [c.copy() for c in cores]
    out[0] = out[0] * alpha
    return out


def direct_sum(terms, coeffs):
    """sum_t coeffs[t] * terms[t] as one MPS (block-diagonal cores)."""
    K = len(terms[0])
    if K == 1:
        return [sum(a * t[0] for a, t in zip(coeffs, terms))]
    out = []
    for k in range(K):
        blocks = [t[k] for t in terms]
        if k == 0:
            G = np.concatenate([a * b for a, b in zip(coeffs, blocks)], axis=2)
        elif k == K - 1:
            G = np.concatenate(blocks, axis=0)
        else:
            r0 = sum(b.shape[0] for b in blocks)
            r1 = sum(b.shape[2] for b in blocks)
            G = np.zeros((r0, 2, r1))
            i = j = 0
            for b in blocks:
                G[i:i + b.shape[0], :, j:j + b.shape[2]] = b
                i += b.shape[0]
                j += b.shape[2]
        out.append(G)
    return out


def hadamard(A, B):
    """Elementwise product: cores C_k[(a,i), s, (b,j)] = A_k[a,s,b] B_k[i,s,j].

    Applying a diagonal MPO whose diagonal is the MPS A (Sec. 4.3, the c^2
    operator of eq. 4) is exactly this product.
    """
    out = []
    for a, b in zip(A, B):
        ra0, d, ra1 = a.shape
        rb0, _, rb1 = b.shape
        G = np.einsum("asb,isj->aisbj", a, b).reshape(ra0 * rb0, d, ra1 * rb1)
        out.append(G)
    return out


def apply_mpo(W, cores):
    """(W psi)_k[(a,i), s', (b,j)] = sum_s W_k[a,b,s',s] G_k[i,s,j]."""
    out = []
    for w, g in zip(W, cores):
        wl, wr, _, _ = w.shape
        r0, _, r1 = g.shape
        G = np.einsum("abts,isj->aitbj", w, g).reshape(wl * r0, 2, wr * r1)
        out.append(G)
    return out


# ---------------------------------------------------------------------------
# Shift MPOs (Sec. 4.2)
# ---------------------------------------------------------------------------

def shift_mpo_1d(n, direction=+1, boundary="periodic"):
    """Cores of S^+ (direction +1) or S^- (-1) on an n-bit register, in site order.

    The carry bit flows from the least significant bit to the most significant
    one.  Bulk core of eq. 9 (row = incoming carry, column = outgoing carry):
    [[I, 0], [sigma+, sigma-]]; eq. 13 swaps sigma+ and sigma- for S^-.  The LSB
    core is the second row of the bulk (eq. 10: carry 1 injected).  The MSB core
    is the first column of the bulk (eq. 11) for the "open" reading; for the
    cyclic shift (x+1 mod 2^n) the carry out of the top bit is summed instead,
    i.e. the MSB core is the sum of both columns.

    Sites are ordered MSB first, so in site order the left bond of a core is its
    outgoing carry and the right bond its incoming carry.
    """
    A, B = (SIGMA_PLUS, SIGMA_MINUS) if direction > 0 else (SIGMA_MINUS, SIGMA_PLUS)
    bulk = np.zeros((2, 2, 2, 2))          # [carry_in, carry_out, s_out, s_in]
    bulk[0, 0] = I2
    bulk[1, 0] = A
    bulk[1, 1] = B
    lsb = bulk[1]                          # [carry_out, s_out, s_in]
    if boundary == "periodic":
        msb = bulk[:, 0] + bulk[:, 1]      # [carry_in, s_out, s_in]
    else:
        msb = bulk[:, 0]
    if n == 1:
        op = lsb[0] + lsb[1] if boundary == "periodic" else lsb[0]
        return [op.reshape(1, 1, 2, 2)]
    cores = [msb.reshape(1, 2, 2, 2)]                       # [out=1, in, s', s]
    for _ in range(n - 2):
        cores.append(np.transpose(bulk, (1, 0, 2, 3)).copy())  # [out, in, s', s]
    cores.append(lsb.reshape(2, 1, 2, 2))                  # [out, in=1, s', s]
    return cores


def identity_mpo(n):
    return [I2.reshape(1, 1, 2, 2).copy() for _ in range(n)]


def passthrough_mpo_core(r):
    """Identity on a site of the other register while a carry of bond r passes."""
    return np.einsum("ab,ts->abts", np.eye(r), I2)


def shift_mpo_2d(n, axis, direction, boundary="periodic", ordering="sequential"):
    """S_x^{+-} = S^{+-} (x) I (eq. 14) and S_z^{+-} = I (x) S^{+-} (eq. 15)."""
    return shift_mpo_nd(n, axis, direction, boundary, ordering, 2)


def shift_mpo_nd(n, axis, direction, boundary="periodic", ordering="sequential", ndim=2):
    """The shift along one axis as an MPO over all K = ndim n sites: the
    register's shift cores, identities elsewhere.

    In the interleaved order the register's cores alternate with identity cores
    of the other registers; a site that lies between two cores of the shifted
    register passes the carry bond through unchanged.
    """
    s = shift_mpo_1d(n, direction, boundary)
    if ordering == "sequential":
        return identity_mpo(n * axis) + s + identity_mpo(n * (ndim - 1 - axis))
    out = []
    for m in range(n):
        for r in range(ndim):
            if r == axis:
                out.append(s[m])
            elif r > axis:      # a site after core m: the carry into core m
                out.append(passthrough_mpo_core(s[m].shape[1]))
            else:               # a site before core m: the carry out of core m
                out.append(passthrough_mpo_core(s[m].shape[0]))
    return out


def mpo_to_dense(W):
    """Dense matrix [out, in] of an MPO (small K only)."""
    M = np.ones((1, 1, 1))                  # [a, out, in]
    for w in W:
        wl, wr, _, _ = w.shape
        M = np.einsum("aoi,abts->botis", M, w)
        b, o, t, i, s = M.shape
        M = M.reshape(b, o * t, i * s)
    return M[0]


def laplacian_mps(cores, n, boundary="periodic", ordering="sequential", ndim=2):
    """L psi with L = S_x+ + S_x- + S_z+ + S_z- - 4 I (eqs. 6 and 16) as one MPS.

    Each shift MPO is applied separately and the five terms are added as a
    direct sum (bond 2chi+2chi+chi+chi+chi inside a register).  With ndim = 3
    the six shifts and -6 I give the seven-point operator.
    """
    terms = [apply_mpo(shift_mpo_nd(n, ax, d, boundary, ordering, ndim), cores)
             for ax in range(ndim) for d in (+1, -1)]
    terms.append(cores)
    return direct_sum(terms, [1.0] * (2 * ndim) + [-2.0 * ndim])
