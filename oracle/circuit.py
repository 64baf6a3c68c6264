"""Classical simulation of the shift circuits of Sec. 3.1.  TEST INFRASTRUCTURE.

The incrementer updates qubit m with x_m <- x_m XOR (x_0 AND ... AND x_{m-1})
(eq. 5), applying the multi-controlled X gates from the most significant qubit
down to the least significant one (Fig. 1 shows the 3-qubit case: the
Toffoli onto x_2, then CNOT onto x_1, then X on x_0).  The decrementer is its
adjoint, i.e. the same gates in reverse order.
"""
import numpy as np


def incrementer_gates(n):
    """Gate list in application order: (target, controls)."""
    return [(m, tuple(range(m))) for m in range(n - 1, -1, -1)]


def apply_gates(x, n, gates):
    bits = [(x >> b) & 1 for b in range(n)]
    for target, controls in gates:
        if all(bits[c] for c in controls):
            bits[target] ^= 1
    return sum(b << i for i, b in enumerate(bits))


def increment(x, n):
    return apply_gates(x, n, incrementer_gates(n))


def decrement(x, n):
    return apply_gates(x, n, list(reversed(incrementer_gates(n))))


def permutation_matrix(n, direction=+1):
    """Matrix P with P[f(x), x] = 1 for f = increment (+1) or decrement (-1)."""
    N = 1 << n
    P = np.zeros((N, N))
    f = increment if direction > 0 else decrement
    for x in range(N):
        P[f(x, n), x] = 1.0
    return P
