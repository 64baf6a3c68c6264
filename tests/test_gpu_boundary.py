"""The C ABI's set-up and ownership calls on the GPU: checkpoint and resume
through mpsw_get_cores / mpsw_set_cores, device memory owned by the caller's
allocator (torch's caching allocator), and the error paths that need the
device (non-finite data, an allocator that runs dry)."""
import numpy as np
import pytest

import synth
from helpers import oracle_c2, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mpsw():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    from paper_2609_01904_amd import mpsw as m
    m.load()
    return m


def _state(mpsw, allocator=None, shots=1):
    n, chi, eps = 6, 16, 1e-7
    cfg = synth.get_config("C2", n=n, steps=40)
    cfgs = [mpsw.make_config(n, chi, eps, cfg["lam"]) for _ in range(shots)]
    st = mpsw.State(cfgs if shots > 1 else cfgs[0], allocator=allocator)
    bonds, cores, _ = oracle_c2(cfg["c2"], cfg["eps_c"])
    st.set_velocity_mpo(bonds, cores)
    for s in range(shots):
        st.set_source(s, (1 << n) // 2 - s, 1, synth.ricker(40, cfg["dt"], 40.0))
    return st


def test_checkpoint_resume_is_bitwise(mpsw):
    a = _state(mpsw, shots=2)
    a.step(15)
    prev, cur = a.get_cores(1, 1), a.get_cores(1, 0)
    step = a.stats(1)["step"]
    assert step == 15 and prev[0] == a.bonds(1, 1) and cur[0] == a.bonds(1, 0)
    b = _state(mpsw, shots=2)
    b.set_cores(1, step, prev, cur)
    assert np.array_equal(b.to_dense(1, 0), a.to_dense(1, 0))
    assert np.array_equal(b.to_dense(1, 1), a.to_dense(1, 1))
    a.step(12)
    b.step(12)
    say("resumed shot: bonds", b.bonds(1, 0))
    assert np.array_equal(b.to_dense(1, 0), a.to_dense(1, 0))   # same source clock, same arithmetic
    assert b.bonds(1, 0) == a.bonds(1, 0)
    with pytest.raises(mpsw.MpswError) as ei:
        bad = (list(cur[0]), cur[1])
        bad[0][3] = 99                                           # beyond min(chi, 2^k)
        b.set_cores(0, 0, prev, bad)
    assert ei.value.name == "EINVAL"
    a.close()
    b.close()


def test_torch_allocator_owns_device_memory(mpsw):
    import torch
    alloc = mpsw.TorchAllocator()
    before = torch.cuda.memory_allocated()
    st = _state(mpsw, allocator=alloc)
    held = alloc.bytes_held()
    say(f"allocator holds {held / 2**20:.1f} MiB in {len(alloc.blocks)} blocks")
    assert held > 1 << 20 and torch.cuda.memory_allocated() - before >= held
    ref = _state(mpsw)
    st.step(20)
    ref.step(20)
    assert np.array_equal(st.to_dense(0, 0), ref.to_dense(0, 0))
    st.close()
    ref.close()
    assert alloc.bytes_held() == 0


def test_allocator_that_runs_dry_reports_enomem(mpsw):
    class Dry(mpsw.TorchAllocator):
        def __init__(self):
            super().__init__()
            calls = {"n": 0}
            inner = self._fns[0]

            def _alloc(nbytes, ctx):
                calls["n"] += 1
                return None if calls["n"] > 3 else inner(nbytes, ctx)

            self._fns = (mpsw.ALLOC_FN(_alloc), self._fns[1])
            self.struct = mpsw.Allocator(self._fns[0], self._fns[1], None)

    dry = Dry()
    with pytest.raises(mpsw.MpswError) as ei:
        _state(mpsw, allocator=dry)
    assert ei.value.name == "ENOMEM"
    assert dry.bytes_held() == 0


def test_non_finite_values_are_reported(mpsw):
    """A non-finite field is refused on the host (EINVAL); values that
    overflow during the steps are reported at the next synchronising call
    (ENONFINITE), and the kernels that meet them still finish."""
    st = _state(mpsw)
    up, u = synth.random_fields(6, seed=2)
    bad = u.copy()
    bad[5, 7] = np.nan
    with pytest.raises(mpsw.MpswError) as ei:
        st.set_fields(0, up, bad)
    assert ei.value.name == "EINVAL"
    # sum of squares of the fields about 4e305 (finite); that of c^2 (L u),
    # with c^2 up to 2e7, about 2.5e318: its roundings overflow
    st.set_fields(0, up * 1e152, u * 1e152)
    st.step(2)
    with pytest.raises(mpsw.MpswError) as ei:
        st.stats(0)
    assert ei.value.name == "ENONFINITE"
    st.close()
