"""Randomized range finder of a bond matrix, plainly.  TEST INFRASTRUCTURE.

Halko, Martinsson and Tropp (SIAM Review 2011), Algorithm 4.4 with one power
iteration, applied to the row space of M (m x n):

    Y = M^T Omega,  Q_Y = orth(Y),  Z = M Q_Y,  Q_Z = orth(Z),
    Y = M^T Q_Z,    Q = orth(Y),    B = M Q,    B = U S W^T,

so M ~ U S (Q W)^T.  The truncation rule of Sec. 4.3 is applied to S.

Acceptance of the sketch (the exact SVD is taken otherwise), with r the rank
the rule keeps from S, res2 = ||M - B Q^T||_F^2 the energy the sketch misses
(formed directly: the difference ||M||^2 - ||B||^2 carries rounding noise of
about 1e-16 ||M||^2, as large as (eps S_1)^2 at eps near 1e-8) and
T = sum of S_i^2 for i > r:

    r below the cap:  r < l and res2 <= (eps S_1)^2 (a Frobenius-norm bound on
                      the residual, at least as strict as its spectral norm);
    r at the cap:     res2 <= 0.21 T   (kept error T + res2 <= 1.21 T, and the
                      optimal error is at least T since S_i <= sigma_i).

Gaussian test matrix: entry (i, j) of the sketch of bond k in rounding j' at
step t is a Box-Muller normal from two uniforms, each the top 53 bits of
SplitMix64 (Steele, Lea and Flood, OOPSLA 2014) of seed XOR (2 key) and
seed XOR (2 key + 1), key = ((((t 3 + j') 64 + k) 4096 + i) 1024 + j); the
first uniform is shifted to (0, 1].
"""
import numpy as np

from .mps import choose_rank, svd

MASK = (1 << 64) - 1


def splitmix64(x):
    """One output of SplitMix64 from state x (python ints, 64-bit wraparound)."""
    z = (x + 0x9E3779B97F4A7C15) & MASK
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK
    return z ^ (z >> 31)


def sketch_normal(seed, step, rnd, site, i, j):
    key = ((((step * 3 + rnd) * 64 + site) * 4096 + i) * 1024 + j) & MASK
    u1 = ((splitmix64(seed ^ ((2 * key) & MASK)) >> 11) + 1) * 2.0 ** -53
    u2 = (splitmix64(seed ^ ((2 * key + 1) & MASK)) >> 11) * 2.0 ** -53
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)


def omega(seed, step, rnd, site, m, l):
    return np.array([[sketch_normal(seed, step, rnd, site, i, j) for j in range(l)] for i in range(m)])


def orth(X):
    q, _ = np.linalg.qr(X)
    return q


def range_finder(M, Om):
    """(Q, B, S, W): row-space basis Q (n x l), B = M Q, B = U S W^T."""
    Q = orth(M.T @ Om)
    Qz = orth(M @ Q)
    Q = orth(M.T @ Qz)
    B = M @ Q
    _, S, Wt = svd(B)
    return Q, B, S, Wt.T


def accept(M, Q, B, S, eps, chi):
    """(accepted, r) by the rule above."""
    l = B.shape[1]
    r = choose_rank(S, eps, chi)
    E = M - B @ Q.T
    res2 = float(np.sum(E * E))
    tail = float(np.sum(S[r:] ** 2))
    if r >= chi:
        return res2 <= 0.21 * tail, r
    return (r < l and res2 <= (eps * S[0]) ** 2), r


# ---------------------------------------------------------------------------
# The learned-rank rounding, plainly: the compression of Sec. 4.3 (QR sweep,
# then SVD sweep with the truncation rule) in which the SVD of a bond matrix
# may be replaced by the sketch above.  Per bond of the SVD sweep:
#
#   r_hat = the network's rank from the bond's leading singular values of the
#           previous step (mlp.features / mlp.forward, read as ceil(out chi));
#   sketch when the bond has a singular-value log, r_hat < chi, l = r_hat + 8
#   satisfies l <= 512, 4 l <= 3 min(m, n), l <= m and l <= n, and the bond
#   is not waiting after a rejected sketch;
#   accept as in `accept`, else take the exact SVD; after a rejection the bond
#   waits 1, 2, 4, ..., 64 steps (doubling per further rejection) before its
#   next sketch, and an accepted sketch resets the wait.
#
# m above is the row count of the bond matrix, which depends on how the
# rounding's input is represented, not only on the tensor: `round` takes the
# row counts to plan with (the rows a given implementation's QR sweep leaves)
# and otherwise uses those of the cores it is given.
# ---------------------------------------------------------------------------
OVERSAMPLE = 8
MAX_WIDTH = 512


class LearnedRounding:
    """State of the learned-rank rounding of one shot across steps: the
    singular-value log each bond's features come from, and the waits."""

    def __init__(self, w, seed, K, rank_of_out=None, prev_rank=False):
        from . import mlp
        self.mlp = mlp
        self.w = None if w is None else np.asarray(w, dtype=np.float64)
        self.seed = int(seed)
        self.K = K
        # baseline without a network: sketch at the rank the bond kept in the
        # same rounding at the previous step
        self.prev_rank = bool(prev_rank)
        self.rank = {}           # (rounding, bond) -> rank kept at the last step
        # rank from the network output (default: ceil(out chi) clamped to [1, chi])
        self.rank_of_out = rank_of_out or (lambda o, chi: int(np.clip(np.ceil(o * chi), 1, chi)))
        self.sig = {}            # (rounding, bond) -> leading 32 singular values of the last step
        self.skip = {}           # (rounding, bond) -> first step a sketch may run again
        self.back = {}           # (rounding, bond) -> current wait
        self.sketches = 0
        self.fallbacks = 0

    def planned_width(self, rnd, k, m, n, chi, step):
        """Sketch width l, or 0 when the exact SVD is taken."""
        lg = self.sig.get((rnd, k))
        if lg is None or lg[0] <= 0.0 or (self.w is None and not self.prev_rank):
            return 0
        if self.prev_rank:
            rhat = self.rank.get((rnd, k), 0)
            if rhat < 1:
                return 0
        else:
            x = self.mlp.features(lg, k, self.K, step)
            out, _ = self.mlp.forward(self.w, x[None, :])
            rhat = self.rank_of_out(float(out[0]), chi)
        l = rhat + OVERSAMPLE
        if step < self.skip.get((rnd, k), 0):
            return 0
        if rhat < chi and l <= MAX_WIDTH and 4 * l <= 3 * min(m, n) and m >= l and n >= l:
            return l
        return 0

    def svd(self, M, eps, chi, rnd, k, step, rows=None):
        """(core rows V_r^T, U_r Sigma_r, sigma logged, kept rank, discarded energy)."""
        m, n = M.shape
        l = self.planned_width(rnd, k, m if rows is None else rows, n, chi, step)
        if l:
            self.sketches += 1
            Q, B, S, W = range_finder(M, omega(self.seed, step, rnd, k, m, l))
            ok, r = accept(M, Q, B, S, eps, chi)
            if ok:
                E = M - B @ Q.T
                self.back[(rnd, k)] = 0
                self.sig[(rnd, k)] = S[:32].copy()
                self.rank[(rnd, k)] = r
                return (W[:, :r].T @ Q.T), B @ W[:, :r], S, r, float(np.sum(S[r:] ** 2) + np.sum(E * E))
            self.fallbacks += 1
            b = min(64, max(1, 2 * self.back.get((rnd, k), 0)))
            self.back[(rnd, k)] = b
            self.skip[(rnd, k)] = step + 1 + b
        U, s, Vt = svd(M)
        r = choose_rank(s, eps, chi)
        self.sig[(rnd, k)] = s[:32].copy()
        self.rank[(rnd, k)] = r
        return Vt[:r], U[:, :r] * s[:r], s, r, float(np.sum(s[r:] ** 2))

    def round(self, cores, eps, chi, step, rnd, log=None, rows=None):
        """QR sweep, then the SVD sweep with sketched or exact bond SVDs
        (rows[k]: the row count of bond matrix k to plan with)."""
        G = [c.copy() for c in cores]
        K = len(G)
        for k in range(K - 1):
            r0, d, r1 = G[k].shape
            Q, R = np.linalg.qr(G[k].reshape(r0 * d, r1))
            G[k] = Q.reshape(r0, d, Q.shape[1])
            G[k + 1] = np.tensordot(R, G[k + 1], axes=(1, 0))
        tail = 0.0
        for k in range(K - 1, 0, -1):
            r0, d, r1 = G[k].shape
            Vt, US, s, r, t = self.svd(G[k].reshape(r0, d * r1), eps, chi, rnd, k, step,
                                       None if rows is None else rows[k])
            tail += t
            if log is not None:
                log.append((k, s.copy(), r))
            G[k] = Vt.reshape(r, d, r1)
            G[k - 1] = np.tensordot(G[k - 1], US, axes=(2, 0))
        return G, tail
