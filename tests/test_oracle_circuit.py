"""Pins of the shift operators: the incrementer circuit (Sec. 3.1, eq. 5, Fig. 1)
against integer arithmetic, and the shift MPO cores (Sec. 4.2, eqs. 9-13)
against the circuit."""
import os

import numpy as np
import pytest

from oracle import circuit as C
from oracle import mps as M


def _golden_fig1(repo_root):
    path = os.path.join(repo_root, "tests", "golden", "fig1_incrementer_3q.txt")
    gates = []
    with open(path) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            v = [int(t) for t in line.split()]
            gates.append((v[0], tuple(v[1:])))
    return gates


def test_fig1_gate_order(repo_root):
    assert C.incrementer_gates(3) == _golden_fig1(repo_root)


@pytest.mark.parametrize("n", range(1, 9))
def test_incrementer_truth_table(n):
    N = 1 << n
    for x in range(N):
        assert C.increment(x, n) == (x + 1) % N
        assert C.decrement(x, n) == (x - 1) % N
        assert C.decrement(C.increment(x, n), n) == x


@pytest.mark.parametrize("n", range(1, 7))
@pytest.mark.parametrize("direction", [+1, -1])
def test_periodic_shift_mpo_equals_circuit(n, direction):
    D = M.mpo_to_dense(M.shift_mpo_1d(n, direction, "periodic"))
    np.testing.assert_array_equal(D, C.permutation_matrix(n, direction))


@pytest.mark.parametrize("n", range(1, 7))
def test_open_shift_mpo_drops_wraparound(n):
    """Eq. 11 as printed keeps only carry-out 0: S^+|2^n-1> = 0 and S^-|0> = 0."""
    N = 1 << n
    P = C.permutation_matrix(n, +1)
    P[0, N - 1] = 0.0
    np.testing.assert_array_equal(M.mpo_to_dense(M.shift_mpo_1d(n, +1, "open")), P)
    Pm = C.permutation_matrix(n, -1)
    Pm[N - 1, 0] = 0.0
    np.testing.assert_array_equal(M.mpo_to_dense(M.shift_mpo_1d(n, -1, "open")), Pm)


@pytest.mark.parametrize("n", range(1, 6))
@pytest.mark.parametrize("boundary", ["periodic", "open"])
def test_backward_shift_is_adjoint(n, boundary):
    Sp = M.mpo_to_dense(M.shift_mpo_1d(n, +1, boundary))
    Sm = M.mpo_to_dense(M.shift_mpo_1d(n, -1, boundary))
    np.testing.assert_array_equal(Sm, Sp.T)


@pytest.mark.parametrize("n", range(2, 7))
def test_shift_mpo_bond_is_two(n):
    W = M.shift_mpo_1d(n, +1, "periodic")
    assert [w.shape[1] for w in W[:-1]] == [2] * (n - 1)
