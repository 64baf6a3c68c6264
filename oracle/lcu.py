"""Statevector simulation of the wavefield update of Sec. 3.2 as a linear
combination of unitaries (LCU).  TEST INFRASTRUCTURE: only tests import it.

The update is eq. 7, psi^{k+1} = A psi^k - psi^{k-1}, with the transition
operator A = 2 I + lambda^2 C^2 L and the Laplacian L written as the sum of the
four shift unitaries minus 4 I (eq. 6).  The shifts are the permutations that
the incrementer and decrementer circuits of Sec. 3.1 realise gate by gate
(oracle/circuit.py), placed on the x or z register in the register order of
eq. 3 (flat index x * 2^n + z).

The paper gives the LCU only in outline, so the constructions below are the
standard ones:

* C^2 is diagonal and positive, not unitary.  With beta = lambda^2 max(c^2),
  lambda^2 C^2 = (beta / 2) (V + V^dagger) for the diagonal unitary
  V = diag(exp(i theta)), cos(theta) = lambda^2 c^2 / beta.  Expanding A gives
  eleven unitaries with non-negative weights: 2 I; (beta / 2) s S for
  s in {V, V^dagger} and each of the four shifts S; 2 beta (-s) for the two
  diagonal unitaries (the -4 I of eq. 6 folded into them).
* PREPARE maps the index register's |0> to sum_j sqrt(alpha_j / |alpha|_1) |j>
  (a real orthogonal matrix with that first column); SELECT applies U_j to the
  system register when the index register holds j.  Then
  <0| PREPARE^dagger SELECT PREPARE |0> = A / |alpha|_1 (block encoding).
* The outline's subtraction of the older time level is taken as a two-term
  LCU over state-preparation unitaries: a select qubit c weighted
  (|alpha|_1 |psi^k|, |psi^{k-1}|) chooses between the block encoding of A
  applied to the prepared psi^k and the prepared psi^{k-1}, with a phase
  inversion on the c = 1 branch for the minus sign.  Postselecting c = 0 and
  the index register at 0 leaves (A psi^k - psi^{k-1}) / (|alpha|_1 |psi^k| +
  |psi^{k-1}|) in the system register.  (A controlled SWAP between two
  registers that hold psi^k and psi^{k-1} would leave the second register
  entangled with the branch, so the state-preparation form is used.)

States are arrays over (index register, system register); operators act
without forming the full matrices, so grids up to n = 5 (1024 system
amplitudes, 16 LCU terms) stay cheap.
"""
import numpy as np

from . import circuit


def shift_unitaries(n):
    """The four shift unitaries of eq. 6 on the 2n-qubit register, as index
    maps: (S u)[f(i)] = u[i], built from the incrementer/decrementer circuits."""
    N = 1 << n
    x = np.arange(N)
    inc = np.array([circuit.increment(v, n) for v in x])
    dec = np.array([circuit.decrement(v, n) for v in x])
    X, Z = np.meshgrid(x, x, indexing="ij")
    maps = []
    for f in (inc, dec):                      # x register
        maps.append((f[X] * N + Z).ravel())
    for f in (inc, dec):                      # z register
        maps.append((X * N + f[Z]).ravel())
    return maps


def apply_map(m, u):
    out = np.empty_like(u)
    out[m] = u
    return out


def lcu_terms(c2, lam):
    """Weights alpha_j >= 0 and unitaries U_j (callables on system vectors)
    with sum_j alpha_j U_j = A = 2 I + lambda^2 C^2 L; also beta."""
    c2 = np.asarray(c2, dtype=float)
    n = int(np.log2(c2.shape[0]))
    d = (lam * lam) * c2.ravel()
    beta = float(d.max())
    theta = np.arccos(np.clip(d / beta, -1.0, 1.0))
    v = np.exp(1j * theta)
    shifts = shift_unitaries(n)
    alphas, units = [2.0], [lambda u: u]
    for s in (v, np.conj(v)):
        for m in shifts:
            alphas.append(beta / 2.0)
            units.append(lambda u, s=s, m=m: s * apply_map(m, u))
        alphas.append(2.0 * beta)
        units.append(lambda u, s=s: -s * u)
    return np.array(alphas), units, beta


def transition_dense(c2, lam):
    """A = 2 I + lambda^2 C^2 L as a dense matrix, from the shift unitaries."""
    c2 = np.asarray(c2, dtype=float)
    n = int(np.log2(c2.shape[0]))
    M = c2.size
    L = -4.0 * np.eye(M)
    for m in shift_unitaries(n):
        P = np.zeros((M, M))
        P[m, np.arange(M)] = 1.0
        L += P
    return 2.0 * np.eye(M) + (lam * lam) * np.diag(c2.ravel()) @ L


def prepare_matrix(alphas, size):
    """Real orthogonal size x size matrix whose first column is
    sqrt(alpha / |alpha|_1) (zero-padded): a Householder reflection of e_0."""
    a = np.zeros(size)
    a[:len(alphas)] = np.sqrt(np.asarray(alphas) / np.sum(alphas))
    e0 = np.zeros(size)
    e0[0] = 1.0
    w = e0 - a
    nw = np.linalg.norm(w)
    if nw < 1e-15:
        return np.eye(size)
    w /= nw
    return np.eye(size) - 2.0 * np.outer(w, w)


def index_size(nterms):
    return 1 << int(np.ceil(np.log2(nterms)))


def block_encode_apply(state, alphas, units, P):
    """PREPARE^dagger SELECT PREPARE on a state of shape (index, system)."""
    s = P @ state
    t = np.zeros_like(s)
    for j, U in enumerate(units):
        t[j] = U(s[j])
    t[len(units):] = s[len(units):]           # padding terms: identity
    return P.conj().T @ t


def householder_prep(v):
    """Real orthogonal matrix whose first column is v / |v| (state preparation)."""
    v = np.asarray(v, dtype=float)
    if np.linalg.norm(v) == 0.0:               # a zero state: any preparation
        return np.eye(v.size)
    a = v / np.linalg.norm(v)
    e0 = np.zeros(v.size)
    e0[0] = 1.0
    w = e0 - a
    nw = np.linalg.norm(w)
    if nw < 1e-15:
        return np.eye(v.size)
    w /= nw
    return np.eye(v.size) - 2.0 * np.outer(w, w)


def lcu_step(u, u_prev, c2, lam):
    """One update of eq. 7 by the circuit of the module docstring.

    Returns (psi^{k+1} as a grid, the postselection probability, the total
    probability of all outcomes).  The circuit acts on (select qubit c,
    index register, system register), starting from |0, 0, 0>."""
    shape = np.shape(u)
    u = np.asarray(u, dtype=float).ravel()
    u_prev = np.asarray(u_prev, dtype=float).ravel()
    alphas, units, _ = lcu_terms(c2, lam)
    nidx = index_size(len(alphas))
    P = prepare_matrix(alphas, nidx)
    nu, npv = np.linalg.norm(u), np.linalg.norm(u_prev)
    w0, w1 = np.sum(alphas) * nu, npv
    Q = householder_prep([np.sqrt(w0), np.sqrt(w1)])
    Pk, Pk1 = householder_prep(u), householder_prep(u_prev)
    M = u.size
    state = np.zeros((2, nidx, M), dtype=complex)
    state[0, 0, 0] = 1.0
    state = np.tensordot(Q, state, axes=(1, 0))                     # prepare c
    b0 = np.zeros((nidx, M), dtype=complex)                          # c = 0: A psi^k
    for j in range(nidx):
        b0[j] = Pk @ state[0, j]
    b0 = block_encode_apply(b0, alphas, units, P)
    b1 = np.zeros((nidx, M), dtype=complex)                          # c = 1: -psi^{k-1}
    for j in range(nidx):
        b1[j] = -(Pk1 @ state[1, j])
    state = np.stack([b0, b1])
    state = np.tensordot(Q.conj().T, state, axes=(1, 0))            # unprepare c
    total = float(np.sum(np.abs(state) ** 2))
    post = state[0, 0]
    p = float(np.sum(np.abs(post) ** 2))
    out = post * (w0 + w1)
    return np.real(out).reshape(shape), p, total
