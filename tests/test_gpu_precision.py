"""Mixed-precision contractions (FP32 and split-BF16 matrix cores) against the
FP64 oracle.

Only the contractions change precision; QR, Jacobi SVD, truncation rule and
tail sums stay FP64, and storage is FP64.  The FP32 path rounds each operand
to FP32 (relative 2^-24) and accumulates in FP32; the BF16 path splits each
operand into three BF16 parts and keeps six of the nine partial products
(the dropped ones are below 2^-26 of a product), so its error is that of the
FP32 accumulation; the FP32 sums of each 16-deep slice are accumulated in
FP64.

Targets after 80 steps of a truncating run on the layered model: 1e-10 for
FP64, 1e-3 for BF16, and 1e-6 for FP32 unless the sensitivity floor of FP32
arithmetic is above it.  The floor at perturbation delta (two oracle runs, one
perturbed by delta relative noise before every rounding) is linear in delta,
about 23 delta here, and does not depend on eps: it is how the leapfrog scheme
carries per-step errors over 80 steps.  At FP32's unit roundoff u = 2^-24 it
is 1.4e-6, already above the 1e-6 target.  The GPU's FP32 rounding does not
enter once per entry of a rounding's input: a rounding chains about 3K FP32
contractions (operator apply, QR sweep, SVD sweep), each adding up to 6u per
entry (two operand roundings and the FP32 sums of up to four matrix-core
steps of a 16-deep slice), which add in norm to sqrt(3K) 6u = 36u at K = 12.
FP32 is held to the floor at delta = 32u = 2^-19.
"""
import sys

import numpy as np
import pytest

from oracle import stepper as S
import synth
import sensitivity

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def mpsw():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    from paper_2609_01904_amd import mpsw as m
    m.load()
    return m


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


@pytest.fixture(scope="module")
def reference():
    # no bond cap is reached (chi = 64 is the largest bond of n = 6), so the
    # eps cutoff alone truncates and the result is not sensitive to where a
    # capped cut falls
    n, eps, chi, steps = 6, 1e-6, 64, 80
    N = 1 << n
    cfg = synth.get_config("C2", n=n, steps=steps)
    return dict(n=n, eps=eps, chi=chi, steps=steps, lam=cfg["lam"], c2=cfg["c2"],
                src=(N // 2, 1), wav=synth.ricker(steps, cfg["dt"], 40.0), eps_c=cfg["eps_c"])


def _run(mpsw, ref, precision):
    st = mpsw.State(mpsw.make_config(ref["n"], ref["chi"], ref["eps"], ref["lam"], precision=precision))
    st.set_velocity_dense(ref["c2"], ref["eps_c"])
    st.set_source(0, ref["src"][0], ref["src"][1], ref["wav"])
    st.step(ref["steps"])
    out = st.to_dense(0, 0)
    c2r = st.to_dense(0, 2)
    st.close()
    return out, c2r


@pytest.fixture(scope="module")
def oracle_field(mpsw, reference):
    ref = reference
    _, c2r = _run(mpsw, ref, mpsw.MPSW_FP64)
    ds = S.DenseStepper(ref["n"], ref["lam"], ref["eps"], ref["chi"], c2r, src=ref["src"], wavelet=ref["wav"])
    for _ in range(ref["steps"]):
        ds.step()
    return ds.dense()


@pytest.fixture(scope="module")
def fp32_floor(mpsw, reference):
    ref = reference
    _, c2r = _run(mpsw, ref, mpsw.MPSW_FP64)
    return sensitivity.floor(ref["n"], ref["lam"], ref["eps"], ref["chi"], c2r, ref["src"], ref["wav"],
                             ref["steps"], delta=2.0 ** -19)


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_precision_against_fp64_oracle(mpsw, reference, oracle_field, fp32_floor, prec):
    tol = {0: 1e-10, 1: max(1e-6, fp32_floor), 2: 1e-3}[prec]
    _say("precision", prec, "tolerance", tol, "floor at 32 u32", fp32_floor)
    got, _ = _run(mpsw, reference, prec)
    err = rel(got, oracle_field)
    _say(f"precision {prec}: rel-L2 vs FP64 oracle after {reference['steps']} steps = {err:.3e}")
    assert np.all(np.isfinite(got))
    assert err < tol, err
