"""The measured workload at full size, in the launch configuration the
benchmark times: n = 10 (1024 x 1024), chi = 128, eps = 1e-6, the layered
velocity model, 256 shots advanced together with autotuned launch shapes,
starting from developed wavefields whose middle bonds sit at the chi cap.

The oracle cannot step 256 shots of this size in a test, so sampled shots are
checked one by one: each sampled shot's two fields before a step are handed to
the dense-detour oracle stepper (Sec. 4.3 roundings as right-to-left truncated
TT-SVDs of the dense tensors), which takes the same step; the GPU result must
agree to 1e-10 relative L2 and in every bond dimension.  The shots not sampled
are held to what holds at any size: finite fields and bonds within the caps.
"""
import sys

import numpy as np
import pytest

from oracle import stepper as S
import synth
from helpers import oracle_c2

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


def test_c3_batched_step_matches_oracle_on_sampled_shots(mpsw):
    import torch
    import bench
    B = 256
    _say("full-size C3 state,", B, "shots")
    cfg0 = synth.get_config("C3")
    bonds, cores, c2r = oracle_c2(cfg0["c2"], cfg0["eps_c"])
    st, cfg, fields = bench.make_state(mpsw, synth, "C3", B, "fp64", velocity=(bonds, cores))
    q, b = st.autotune(1)
    _say("autotuned: QR workgroups per shot", q, "Jacobi block", b)
    st.step(2)
    torch.cuda.synchronize()
    n, N, K = cfg["n"], 1 << cfg["n"], 2 * cfg["n"]
    sample = [0, 1, 45, 128, 200, 255]
    before = {s: (st.to_dense(s, 1), st.to_dense(s, 0), st.stats(s)["step"]) for s in sample}
    st.step(1)
    torch.cuda.synchronize()
    for s in range(B):
        bonds = st.bonds(s, 0)
        assert len(bonds) == K + 1 and bonds[0] == 1 and bonds[-1] == 1
        assert all(1 <= x <= min(cfg["chi"], 2 ** k, 2 ** (K - k)) for k, x in enumerate(bonds))
    for s in sample:
        up, u, k = before[s]
        g = st.to_dense(s, 0)
        assert np.all(np.isfinite(g))
        ds = S.DenseStepper(n, cfg["lam"], cfg["eps"], cfg["chi"], c2r, src=fields[s][2],
                            wavelet=cfg["wavelet_samples"])
        ds.u_prev, ds.u, ds.k = up, u, k
        ds.step()
        err = rel(g, ds.dense())
        _say(f"shot {s} (step {k + 1}): rel-L2 vs oracle {err:.2e}; bonds {st.bonds(s, 0)}")
        assert err < 1e-10, (s, err)
        assert st.bonds(s, 0) == ds.ranks[-1][2], s
    st.close()


def test_c5_step_matches_oracle(mpsw):
    """n = 11 (2048 x 2048), chi = 256: factors of up to 512 columns and QR
    panels of 4096 rows; one shot, one step after a warm-up step, against the
    oracle step from the same fields."""
    import torch
    import bench
    cfg0 = synth.get_config("C5")
    bonds, cores, c2r = oracle_c2(cfg0["c2"], cfg0["eps_c"])
    st, cfg, fields = bench.make_state(mpsw, synth, "C5", 1, "fp64", velocity=(bonds, cores))
    st.step(1)
    torch.cuda.synchronize()
    n = cfg["n"]
    up, u, k = st.to_dense(0, 1), st.to_dense(0, 0), st.stats(0)["step"]
    st.step(1)
    torch.cuda.synchronize()
    g = st.to_dense(0, 0)
    ds = S.DenseStepper(n, cfg["lam"], cfg["eps"], cfg["chi"], c2r, src=fields[0][2],
                        wavelet=cfg["wavelet_samples"])
    ds.u_prev, ds.u, ds.k = up, u, k
    ds.step()
    err = rel(g, ds.dense())
    _say(f"C5 step {k + 1}: rel-L2 vs oracle {err:.2e}; bonds {st.bonds(0, 0)}")
    assert err < 1e-10, err
    assert st.bonds(0, 0) == ds.ranks[-1][2]
    st.close()
