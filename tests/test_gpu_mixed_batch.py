"""The batched-shots workload (64 seeded shots on grids n = 8, 9, 10 with chi
caps 32/64/128, one state per grid, all stepped by one group graph), in FP64
from rest: sampled shots of every grid against the dense-detour oracle, and
every shot's bonds within its caps."""
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


def test_mixed_batch_group_matches_oracle_on_sampled_shots(mpsw):
    import torch
    import bench
    steps = 25
    ops = {n: oracle_c2(synth.get_config("C3", n=n)["c2"], 1e-6) for n in (8, 9, 10)}
    states, groups, shots = bench.make_mixed_states(mpsw, synth, "fp64", steps,
                                                    velocity={n: op[:2] for n, op in ops.items()})
    _say("shots per grid", {n: len(g) for n, g in groups.items()})
    grp = mpsw.Group(states)
    grp.step(steps)
    torch.cuda.synchronize()
    for st, (n, mine) in zip(states, sorted(groups.items())):
        K = 2 * n
        for i, sh in enumerate(mine):
            b = st.bonds(i, 0)
            assert all(1 <= x <= min(sh["chi"], 2 ** k, 2 ** (K - k)) for k, x in enumerate(b))
            assert st.stats(i)["step"] == steps
    for st, (n, mine) in zip(states, sorted(groups.items())):
        c2r = ops[n][2]
        lam = mine[0]["dt"] / mine[0]["dh"]
        for i in (0, len(mine) - 1):
            sh = mine[i]
            ds = S.DenseStepper(n, lam, sh["eps"], sh["chi"], c2r, src=(sh["ix"], sh["iz"]),
                                wavelet=sh["wavelet_samples"])
            for _ in range(steps):
                ds.step()
            err = rel(st.to_dense(i, 0), ds.dense())
            _say(f"n={n} shot {i} (chi {sh['chi']}, f0 {sh['f0']:.1f} Hz): rel-L2 vs oracle {err:.2e}")
            assert err < 1e-10, (n, i, err)
            assert st.bonds(i, 0) == ds.ranks[-1][2]
    grp.close()
    for st in states:
        st.close()
