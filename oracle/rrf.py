"""Randomized range finder of a bond matrix, plainly.  TEST INFRASTRUCTURE.

Halko, Martinsson and Tropp (SIAM Review 2011), Algorithm 4.4 with one power
iteration, applied to the row space of M (m x n):

    Y = M^T Omega,  Q_Y = orth(Y),  Z = M Q_Y,  Q_Z = orth(Z),
    Y = M^T Q_Z,    Q = orth(Y),    B = M Q,    B = U S W^T,

so M ~ U S (Q W)^T.  The truncation rule of Sec. 4.3 is applied to S.

Acceptance of the sketch (the exact SVD is taken otherwise), with r the rank
the rule keeps from S, res2 = ||M||_F^2 - ||B||_F^2 the energy the sketch
misses and T = sum of S_i^2 for i > r:

    r below the cap:  r < l and res2 <= (eps S_1)^2;
    r at the cap:     res2 <= 0.21 T   (kept error T + res2 <= 1.21 T, and the
                      optimal error is at least T since S_i <= sigma_i).

Gaussian test matrix: entry (i, j) of the sketch of bond k in rounding j' at
step t is a Box-Muller normal from two uniforms, each the top 53 bits of
SplitMix64 (Steele, Lea and Flood, OOPSLA 2014) of seed XOR (2 key) and
seed XOR (2 key + 1), key = ((((t 3 + j') 64 + k) 4096 + i) 1024 + j); the
first uniform is shifted to (0, 1].
"""
import numpy as np

from .mps import choose_rank

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
    _, S, Wt = np.linalg.svd(B, full_matrices=False)
    return Q, B, S, Wt.T


def accept(M, B, S, eps, chi):
    """(accepted, r) by the rule above."""
    l = B.shape[1]
    r = choose_rank(S, eps, chi)
    res2 = max(float(np.sum(M * M) - np.sum(B * B)), 0.0)
    tail = float(np.sum(S[r:] ** 2))
    if r >= chi:
        return res2 <= 0.21 * tail, r
    return (r < l and res2 <= (eps * S[0]) ** 2), r
