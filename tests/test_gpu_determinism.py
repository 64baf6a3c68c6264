"""Run-to-run determinism of the batched step in the shape the benchmark times:
the n = 10 workload (chi = 128, eps = 1e-6) with 256 shots, in the launch shapes
the autotuner picks there (1 workgroup per shot, Jacobi blocks of 32
columns) and in the 2- and 4-workgroup shapes (where the workgroups of one
shot share its QR panels through flags and its Jacobi block pairs through
round barriers), stepped twice from the same fields in two fresh states.
Every kernel sums in a fixed order and the workgroups of one shot only read
what the others have published, so the two runs must
agree bit for bit in every shot's bonds and in sampled fields (a race between
workgroups shows up here as shots whose truncation ranks differ between the
runs)."""
import sys

import numpy as np
import pytest

import synth

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


def _run(mpsw, shots, steps, sample, shapes):
    import torch
    import bench
    st, cfg, _ = bench.make_state(mpsw, synth, "C3", shots, "fp64")
    st.set_launch_shapes(*shapes)
    st.step(steps)
    torch.cuda.synchronize()
    bonds = [st.bonds(s, 0) for s in range(shots)]
    fields = {s: st.to_dense(s, 0) for s in sample}
    st.close()
    return bonds, fields


@pytest.mark.parametrize("shapes", [(1, 32), (2, 32), (4, 32)])
def test_batched_steps_are_bitwise_repeatable(mpsw, shapes):
    shots, steps, sample = 256, 6, (0, 37, 255)
    _say("256 shots, launch shapes", shapes)
    b1, f1 = _run(mpsw, shots, steps, sample, shapes)
    _say("run 1: bonds of shot 0", b1[0])
    b2, f2 = _run(mpsw, shots, steps, sample, shapes)
    _say("run 2: bonds of shot 0", b2[0])
    differ = [s for s in range(shots) if b1[s] != b2[s]]
    assert not differ, f"{len(differ)} shots with other bonds, first {differ[:8]}"
    for s in sample:
        assert np.array_equal(f1[s], f2[s]), s


def test_launch_shapes_are_checked(mpsw):
    st = mpsw.State(mpsw.make_config(3, 8, 1e-8, 0.1))
    for bad in ((0, 0), (33, 0), (4, 12), (4, -1)):
        with pytest.raises(mpsw.MpswError) as ei:
            st.set_launch_shapes(*bad)
        assert ei.value.name == "EINVAL", bad
    st.set_launch_shapes(4, 16)
    st.close()


def test_launch_shapes_agree_to_rounding(mpsw):
    """The same steps in 1, 2 and 4 workgroups per shot: with fewer Jacobi
    workgroups than block pairs each takes several pairs of a round in turn,
    and the QR panels move between workgroups through flags.  The shapes only
    change the order of some sums, so every shot keeps the same bonds and the
    sampled fields agree to rounding."""
    shots, steps, sample = 32, 4, (0, 13, 31)
    ref = None
    for shapes in ((4, 32), (2, 32), (1, 32)):
        import torch
        import bench
        st, cfg, _ = bench.make_state(mpsw, synth, "C3", shots, "fp64")
        st.set_launch_shapes(*shapes)
        st.step(steps)
        torch.cuda.synchronize()
        bonds = [st.bonds(s, 0) for s in range(shots)]
        fields = {s: st.to_dense(s, 0) for s in sample}
        st.close()
        _say("32 shots, launch shapes", shapes, "bonds of shot 0", bonds[0])
        if ref is None:
            ref = (bonds, fields)
            continue
        assert bonds == ref[0], shapes
        for s in sample:
            err = np.linalg.norm(fields[s] - ref[1][s]) / np.linalg.norm(ref[1][s])
            assert err < 1e-12, (shapes, s, err)
