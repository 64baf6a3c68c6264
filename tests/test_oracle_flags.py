"""Pins of the oracle's cut flags (mps.cut_flags): constructed spectra, and
the property the flags stand for, checked by brute force: an unflagged cut
moves by about the size of a rounding-level perturbation, a flagged one can
move by orders of magnitude more."""
import numpy as np

from oracle import mps as M


def truncate(A, eps, chi):
    U, s, Vt = np.linalg.svd(A, full_matrices=False)
    r = M.choose_rank(s, eps, chi)
    return (U[:, :r] * s[:r]) @ Vt[:r], s, r


def with_spectrum(s, seed):
    rng = np.random.default_rng(seed)
    m = len(s)
    U, _ = np.linalg.qr(rng.standard_normal((m + 4, m)))
    V, _ = np.linalg.qr(rng.standard_normal((m, m)))
    return (U * s) @ V.T


def test_constructed_spectra():
    s = np.array([1.0, 0.5, 0.2, 0.2 * (1 - 1e-5), 0.1])
    assert M.cut_flags(s, 3, 0.0) == {"gap"}            # the cap cuts a near tie
    assert M.cut_flags(s, 2, 0.0) == set()             # the cap cuts with a margin
    assert M.cut_flags(s, 4, 0.1) == {"cut"}           # 0.1 sits on the cutoff
    assert M.cut_flags(s, 4, 0.1 + 1e-14) == {"cut"}
    assert M.cut_flags(s, 4, 0.15) == set()            # the near tie is kept whole by the cutoff
    assert M.cut_flags(s, 5, 0.0) == set()             # nothing cut
    assert M.cut_flags(np.zeros(4), 1, 0.1) == set()   # zero matrix
    # exactly equal values dropped together by the cutoff
    assert M.cut_flags(np.array([1.0, 0.3, 1e-3, 1e-3]), 2, 1e-2) == set()


def test_flagged_cut_is_sensitive_unflagged_is_not():
    rng = np.random.default_rng(0)
    base = np.geomspace(1.0, 1e-6, 24)
    tie = base.copy()
    tie[8] = tie[7] * (1 - 1e-9)                   # the cap (8) cuts between equal-looking values
    for spec, flagged in ((base, False), (tie, True)):
        A = with_spectrum(spec, 1)
        T0, s, r = truncate(A, 0.0, 8)
        assert r == 8
        assert bool(M.cut_flags(s, r, 0.0)) == flagged
        moves = []
        for seed in range(4):
            E = np.random.default_rng(seed + 10).standard_normal(A.shape)
            E *= 1e-14 * np.linalg.norm(A, 2) / np.linalg.norm(E, 2)
            T1, _, _ = truncate(A + E, 0.0, 8)
            moves.append(np.linalg.norm(T1 - T0, 2) / np.linalg.norm(A, 2))
        if flagged:
            assert max(moves) > 1e-10
        else:
            assert max(moves) < 1e-12


def test_value_on_the_cutoff_flips():
    """A singular value on eps sigma_1 is kept or dropped by a rounding-level
    change: the rank moves by one and the truncation by about eps."""
    eps = 1e-6
    spec = np.geomspace(1.0, 1e-8, 20)
    spec[12] = eps * (1 + 1e-14)
    A = with_spectrum(spec, 2)
    T0, s, r0 = truncate(A, eps, 64)
    assert "cut" in M.cut_flags(s, r0, eps)
    ranks = {r0}
    for seed in range(8):
        E = np.random.default_rng(seed).standard_normal(A.shape)
        E *= 1e-13 / np.linalg.norm(E, 2)
        ranks.add(truncate(A + E, eps, 64)[2])
    assert len(ranks) == 2
