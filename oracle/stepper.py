"""The MPS time step of eq. 17, plainly.  TEST INFRASTRUCTURE.

psi^{k+1} = 2 psi^k - psi^{k-1} + lambda^2 C^2 (S_x+ + S_x- + S_z+ + S_z- - 4 I) psi^k

with a compression after each operator application (Sec. 4.3).  Both steppers
take the site order (sequential registers of eq. 3, or interleaved bits) as a
parameter; fields given to and returned by them are always u[x, z], or
u[x, y, z] for the three-dimensional form (MPSStepper's ndim = 3; the dense
stepper takes the rank of its c^2 array).  Reading used
throughout (three roundings per step, "S1"):

    y        = round(L psi^k)
    w        = round(C^2 . y)
    psi^{k+1} = round(2 psi^k - psi^{k-1} + lambda^2 w + s_k e_src)

Each round() is the QR sweep + truncated SVD sweep with the same (eps, chi_max).
The c^2 diagonal MPO is the TT-SVD of the dense c^2 with the same per-bond rule
and cutoff eps_c (no bond cap).  Two implementations are given:

* MPSStepper   operates on cores (shift MPOs, direct sums, Hadamard products,
               QR/SVD sweeps) exactly as the paper describes;
* DenseStepper keeps dense fields and replaces every round(T) by the
               right-to-left truncated TT-SVD of dense(T).  After the QR sweep
               the left part of the chain is orthonormal, so each SVD of the
               sweep sees the singular values of the current tensor's
               unfolding: the two give the same tensor in exact arithmetic.
"""
import numpy as np

from . import mps as M
from . import fdtd as F


def c2_mps(c2_dense, n, eps_c, ordering="sequential"):
    """The c^2 diagonal operator as an MPS (its diagonal), TT-SVD with cutoff eps_c."""
    c2_dense = np.asarray(c2_dense, dtype=np.float64)
    return M.tt_svd(M.to_sites(c2_dense, ordering), c2_dense.ndim * n, eps_c, chi_max=1 << 30)


# Rounding schedules of one step: "three" rounds the
# Laplacian result, the c^2 product and the update sum (eq. 17); "seven"
# rounds after each of the 2 ndim shift-operator applications and after their
# sum as well (the literal reading of a compression after every operator
# application); "one" rounds only the update sum, so the Laplacian and the c^2
# product are exact (bonds multiply: usable on small grids only); "zipup" and
# "variational" compress the Laplacian and the c^2 products by zip-up or by a
# variational fit (oracle.compress) instead of rounding the exact products,
# and round the update sum.
SCHEDULES = ("three", "seven", "one", "zipup", "variational")


def qr_sweep_rows(rin):
    """Row counts of the bond matrices a left-to-right QR sweep leaves for
    input bonds rin[0..K]: rt_0 = 1, rt_{k+1} = min(2 rt_k, rin_{k+1})."""
    rt = [1]
    for k in range(1, len(rin)):
        rt.append(min(2 * rt[-1], int(rin[k])))
    return rt


def library_rows(which, n, bonds, c2_bonds, ndim=2):
    """Row counts of the bond matrices of the library's rounding `which` (0: L psi,
    1: c^2 y, 2: the sum; sequential site order) from the bonds of its input
    terms: it applies L as one fused operator (bonds 3 inside the x register,
    2 at the register boundary, 4 inside the z register) instead of the direct
    sum of the five terms, and forms the c^2 product in its middle
    unfolding (the left half in the identity basis, bond 2^k; the right half
    densely, bond at most 2^(K-k)).  The tensors are the same; only the sizes
    the learned-rank plan sees differ."""
    K = ndim * n
    if which == 0:
        w = [1] + [3] * (n - 1) + [2] + [4] * (n - 1) + [1]
        rin = [w[k] * bonds[0][k] for k in range(K + 1)]
    elif which == 1:
        rin = [2 ** k if k < K // 2 else 2 ** (K - k) for k in range(K + 1)]
    else:
        rin = [sum(b[k] for b in bonds) if 0 < k < K else 1 for k in range(K + 1)]
    return qr_sweep_rows(rin)


class MPSStepper:
    def __init__(self, n, lam, eps, chi_max, c2_cores, boundary="periodic",
                 src=None, wavelet=None, ordering="sequential", ndim=2, schedule="three", learned=None,
                 learned_rows=None):
        """learned: an oracle.rrf.LearnedRounding to replace bond SVDs by sketches
        (the learned-rank rounding); None rounds exactly.  learned_rows =
        "library" plans the sketches with the bond-matrix sizes of the
        library's representation (library_rows; two dimensions, sequential
        order), None with those of the cores built here."""
        if schedule not in SCHEDULES:
            raise ValueError(f"schedule must be one of {SCHEDULES}")
        self.schedule = schedule
        self.n, self.K, self.ndim = n, ndim * n, ndim
        self.lam, self.eps, self.chi = lam, eps, chi_max
        self.c2 = c2_cores
        self.boundary = boundary
        self.ordering = ordering
        self.src = src
        self.wavelet = wavelet
        self.k = 0
        self.psi = M.zero_mps(self.K)
        self.psi_prev = M.zero_mps(self.K)
        self.log = []            # (step, rounding, site, sigma, rank)
        self.flags = []          # (step, rounding, site, flags) of every flagged cut (mps.cut_flags)
        self.learned = learned
        self.learned_rows = learned_rows
        self._terms = []         # bonds of the terms of the rounding in progress
        self.tails = {}          # (step, rounding) -> discarded energy of that rounding

    def set_fields(self, u_prev, u):
        """Initial fields given densely; stored as their rounded MPS."""
        self.psi_prev = M.tt_svd(M.to_sites(u_prev, self.ordering), self.K, self.eps, self.chi)
        self.psi = M.tt_svd(M.to_sites(u, self.ordering), self.K, self.eps, self.chi)

    def _round(self, cores, which):
        log = []
        if self.learned is not None and which in (0, 1, 2):
            rows = library_rows(which, self.n, self._terms, M.bonds_of(self.c2), self.ndim) \
                if self.learned_rows == "library" else None
            out, tail = self.learned.round(cores, self.eps, self.chi, self.k, which, log, rows)
            self.tails[(self.k, which)] = tail
        else:
            out = M.round_mps(cores, self.eps, self.chi, log)
        for site, s, r in log:
            self.log.append((self.k, which, site, s, r))
            f = M.cut_flags(s, r, self.eps)
            if f:
                self.flags.append((self.k, which, site, f))
        return out

    def _compress(self, W, cores, which):
        """W cores compressed by the schedule's method (zip-up or variational)."""
        from . import compress as C
        if self.schedule == "zipup":
            log = []
            out = C.zip_up(W, cores, self.eps, self.chi, log)
            for site, s, r in log:
                self.log.append((self.k, which, site, s, r))
            return out
        return C.variational(W, cores, self.eps, self.chi)

    def tail2(self, step, which):
        """Discarded sum of sigma^2 over the bonds of one rounding of one step."""
        return float(sum(np.sum(s[r:] ** 2) for k, w, _, s, r in self.log if k == step and w == which))

    def step(self):
        s_k = 0.0
        if self.wavelet is not None and self.k < len(self.wavelet):
            s_k = float(self.wavelet[self.k])
        if self.schedule == "one":
            # no rounding before the last: the Laplacian and the c^2 product
            # enter the sum at their full bonds
            w = M.hadamard(self.c2, M.laplacian_mps(self.psi, self.n, self.boundary, self.ordering,
                                                    self.ndim))
        elif self.schedule in ("zipup", "variational"):
            from . import compress as C
            lap = C.laplacian_mpo(self.n, self.boundary, self.ordering, self.ndim)
            y = self._compress(lap, self.psi, 0)
            w = self._compress(C.diagonal_mpo(self.c2), y, 1)
        else:
            if self.schedule == "seven":
                # a rounding after each shift-operator application, then one
                # after their sum with -2 ndim psi
                shifted = [self._round(M.apply_mpo(M.shift_mpo_nd(self.n, ax, d, self.boundary,
                                                                  self.ordering, self.ndim), self.psi), 3)
                           for ax in range(self.ndim) for d in (+1, -1)]
                y = self._round(M.direct_sum(shifted + [self.psi],
                                             [1.0] * (2 * self.ndim) + [-2.0 * self.ndim]), 0)
            else:
                self._terms = [M.bonds_of(self.psi)]
                y = self._round(M.laplacian_mps(self.psi, self.n, self.boundary, self.ordering, self.ndim), 0)
            self._terms = [M.bonds_of(y)]
            w = self._round(M.hadamard(self.c2, y), 1)
        terms = [self.psi, self.psi_prev, w]
        coeffs = [2.0, -1.0, self.lam * self.lam]
        if self.src is not None:
            terms.append(M.point_state_nd(self.n, tuple(self.src), self.ordering))
            coeffs.append(s_k)
        self._terms = [M.bonds_of(t) for t in terms]
        nxt = self._round(M.direct_sum(terms, coeffs), 2)
        self.psi_prev, self.psi = self.psi, nxt
        self.k += 1

    def dense(self, which=0):
        return M.from_sites(M.to_dense(self.psi if which == 0 else self.psi_prev), self.n,
                            self.ordering, self.ndim)


class DenseStepper:
    """Same rounded trajectory as MPSStepper, through dense TT-SVDs."""

    def __init__(self, n, lam, eps, chi_max, c2_dense, boundary="periodic",
                 src=None, wavelet=None, ordering="sequential", keep_log=True):
        c2_dense = np.asarray(c2_dense, dtype=np.float64)
        self.ndim = c2_dense.ndim
        self.n, self.K = n, self.ndim * n
        self.N = 1 << n
        self.lam, self.eps, self.chi = lam, eps, chi_max
        self.c2 = np.asarray(c2_dense, dtype=np.float64)
        self.boundary = boundary
        self.ordering = ordering
        self.src = src
        self.wavelet = wavelet
        self.k = 0
        self.u = np.zeros((self.N,) * self.ndim)
        self.u_prev = np.zeros((self.N,) * self.ndim)
        self.keep_log = keep_log
        self.log = []            # (step, rounding, site, sigma, rank) when keep_log
        self.ranks = []          # per step: (bonds of y, bonds of w, bonds of psi)
        self.tail2 = []          # per step: discarded sum of sigma^2 of each rounding
        self.flags = []          # (step, rounding, site, flags) of every flagged cut (mps.cut_flags)

    def _round(self, t, which):
        log = []
        cores = M.tt_svd(M.to_sites(t, self.ordering), self.K, self.eps, self.chi, log)
        tail = 0.0
        for site, s, r in log:
            if self.keep_log:
                self.log.append((self.k, which, site, s, r))
            tail += float(np.sum(s[r:] ** 2))
            f = M.cut_flags(s, r, self.eps)
            if f:
                self.flags.append((self.k, which, site, f))
        self._tail[which] = tail
        return M.from_sites(M.to_dense(cores), self.n, self.ordering, self.ndim), M.bonds_of(cores)

    def first_flag(self):
        """Step index of the first flagged cut (None if none so far)."""
        return self.flags[0][0] if self.flags else None

    def set_fields(self, u_prev, u):
        self._tail = {}
        self.u_prev, _ = self._round(np.asarray(u_prev, dtype=np.float64), -1)
        self.u, _ = self._round(np.asarray(u, dtype=np.float64), -1)

    def step(self):
        s_k = 0.0
        if self.wavelet is not None and self.k < len(self.wavelet):
            s_k = float(self.wavelet[self.k])
        self._tail = {}
        y, by = self._round(F.laplacian(self.u, self.boundary), 0)
        w, bw = self._round(self.c2 * y, 1)
        t = 2.0 * self.u - self.u_prev + (self.lam * self.lam) * w
        if self.src is not None:
            t[tuple(self.src)] += s_k
        nxt, bp = self._round(t, 2)
        self.ranks.append((by, bw, bp))
        self.tail2.append((self._tail[0], self._tail[1], self._tail[2]))
        self.u_prev, self.u = self.u, nxt
        self.k += 1

    def dense(self, which=0):
        return self.u if which == 0 else self.u_prev
