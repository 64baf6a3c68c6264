"""Captured steps (HIP graphs) and groups of states through the C ABI.

A graph replays the same kernels on the same buffers, so graph mode and group
stepping must reproduce eager stepping bit for bit.  Every replay is checked,
with eager work (dense contractions, synchronisations) between replays, and
the end state is checked against the FP64 oracle.
"""
import sys

import numpy as np
import pytest

from oracle import stepper as S
import synth
from helpers import oracle_velocity

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


def _state(mpsw, n, chis, eps, lam, c2, srcs, wav):
    cfgs = [mpsw.make_config(n, chi, eps, lam) for chi in chis]
    st = mpsw.State(cfgs if len(cfgs) > 1 else cfgs[0])
    st.c2r = oracle_velocity(st, c2, 1e-8)
    for i, (ix, iz) in enumerate(srcs):
        st.set_source(i, ix, iz, wav)
    return st


def test_graph_mode_matches_eager(mpsw):
    import torch
    n, eps, lam = 5, 1e-9, 0.5
    N = 1 << n
    c2 = synth.layered_fault_velocity(n, dh=40.0) * 1e-8
    wav = synth.ricker(40, 0.004, 20.0)
    eager = _state(mpsw, n, [32], eps, lam, c2, [(N // 2, 1)], wav)
    graph = _state(mpsw, n, [32], eps, lam, c2, [(N // 2, 1)], wav)
    graph.set_graph_mode(True)
    done = 0
    for chunk in [3, 3, 1, 4, 6, 3]:   # replays of all three phases, eager remainders
        _say("graph chunk", chunk, "after", done)
        eager.step(chunk)
        graph.step(chunk)
        done += chunk
        torch.cuda.synchronize()
        a, b = eager.to_dense(0, 0), graph.to_dense(0, 0)
        assert np.array_equal(a, b), (done, rel(b, a))
        assert np.array_equal(eager.to_dense(0, 1), graph.to_dense(0, 1))
        assert graph.stats(0)["step"] == done
    ds = S.DenseStepper(n, lam, eps, 32, eager.c2r, src=(N // 2, 1), wavelet=wav)
    for _ in range(done):
        ds.step()
    assert rel(graph.to_dense(0, 0), ds.dense()) < 1e-10
    eager.close()
    graph.close()


def test_group_of_mixed_grids_matches_eager(mpsw):
    import torch
    eps, lam = 1e-9, 0.5
    wav = synth.ricker(40, 0.004, 20.0)
    specs = [  # (n, chis per shot, sources per shot)
        (4, [8, 16], [(3, 1), (12, 2)]),
        (5, [32], [(16, 1)]),
        (3, [4, 8, 8], [(0, 0), (5, 1), (7, 7)]),
    ]
    c2s = {n: synth.layered_fault_velocity(n, dh=40.0) * 1e-8 for n, _, _ in specs}
    grouped = [_state(mpsw, n, chis, eps, lam, c2s[n], srcs, wav) for n, chis, srcs in specs]
    single = [_state(mpsw, n, chis, eps, lam, c2s[n], srcs, wav) for n, chis, srcs in specs]
    grp = mpsw.Group(grouped)
    done = 0
    for chunk in [7, 3, 3, 2]:
        _say("group chunk", chunk, "after", done)
        grp.step(chunk)
        for st in single:
            st.step(chunk)
        done += chunk
        torch.cuda.synchronize()
        for (n, chis, _), g, s in zip(specs, grouped, single):
            for shot in range(len(chis)):
                assert np.array_equal(g.to_dense(shot, 0), s.to_dense(shot, 0)), (n, shot, done)
                assert g.bonds(shot, 0) == s.bonds(shot, 0)
                assert g.stats(shot)["step"] == done
    # a state stepped on its own leaves the group's graph stale; the group recaptures
    grouped[1].step(1)
    single[1].step(1)
    grp.step(3)
    for st in single:
        st.step(3)
    torch.cuda.synchronize()
    for g, s, (n, chis, _) in zip(grouped, single, specs):
        for shot in range(len(chis)):
            assert np.array_equal(g.to_dense(shot, 0), s.to_dense(shot, 0))
    grp.close()
    for st in grouped + single:
        st.close()


def test_autotune_restores_state_and_keeps_results(mpsw):
    import torch
    n, eps, lam = 5, 1e-9, 0.5
    N = 1 << n
    c2 = synth.layered_fault_velocity(n, dh=40.0) * 1e-8
    wav = synth.ricker(40, 0.004, 20.0)
    st = _state(mpsw, n, [32, 16], eps, lam, c2, [(N // 2, 1), (3, 2)], wav)
    st.step(5)
    torch.cuda.synchronize()
    before = [st.to_dense(s, w) for s in range(2) for w in (0, 1)]
    bonds = [st.bonds(s, 0) for s in range(2)]
    q, b = st.autotune(2)
    _say("autotune chose", q, b)
    assert q in (32, 16, 8, 4, 3, 2, 1) and b in (0, 8, 16, 32)
    after = [st.to_dense(s, w) for s in range(2) for w in (0, 1)]
    assert all(np.array_equal(x, y) for x, y in zip(before, after))
    assert [st.bonds(s, 0) for s in range(2)] == bonds
    assert st.stats(0)["step"] == 5
    st.step(10)
    ds = S.DenseStepper(n, lam, eps, 32, st.c2r, src=(N // 2, 1), wavelet=wav)
    for _ in range(15):
        ds.step()
    assert rel(st.to_dense(0, 0), ds.dense()) < 1e-10
    st.close()
