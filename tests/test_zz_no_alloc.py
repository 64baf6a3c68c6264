"""The allocation-free entry point (mpsw_mlp_grad_noalloc): device buffers
from the caller, partial sums in the library's static scratch array.  Two
calls in a row, the second on fewer samples, each against mpsw_mlp_grad (the
same kernels with library-allocated buffers): equal bit for bit."""
import numpy as np
import pytest

from oracle import mlp

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mpsw():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    from paper_2609_01904_amd import mpsw as m
    m.load()
    return m


def _data(m, seed):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((m, mlp.NIN)).astype(np.float32)
    X[:, :32] = -np.abs(X[:, :32]) * 3.0
    y = rng.uniform(0.05, 1.0, m).astype(np.float32)
    return X, y


def test_noalloc_gradient_equals_allocating_one(mpsw):
    import torch
    w = mlp.init(seed=3).astype(np.float32)
    w[-1] = 0.2
    wd = torch.from_numpy(w).cuda()
    grad = torch.empty(mpsw.MLP_NPARAM, dtype=torch.float32, device="cuda")
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    stream = torch.cuda.Stream()
    for m, seed in ((3000, 1), (257, 2)):   # the second call is smaller: stale scratch must not leak in
        X, y = _data(m, seed)
        Xd, yd = torch.from_numpy(X).cuda(), torch.from_numpy(y).cuda()
        torch.cuda.synchronize()
        with torch.cuda.stream(stream):
            mpsw.mlp_grad_noalloc(Xd, yd, wd, grad, loss, alpha=4.0, stream=stream)
        stream.synchronize()
        L, g = mpsw.mlp_grad(X, y, w, 4.0)
        assert np.array_equal(grad.cpu().numpy(), g), m
        assert loss.item() == L, m
        # and against the FP64 oracle to the FP32 bound of the gradient tests
        Lo, go = mlp.grad(w.astype(np.float64), X.astype(np.float64), y.astype(np.float64), 4.0)
        assert np.linalg.norm(g - go) <= 1e-4 * np.linalg.norm(go)
    with pytest.raises(mpsw.MpswError) as ei:
        X, y = _data(8193, 3)
        mpsw.mlp_grad_noalloc(torch.from_numpy(X).cuda(), torch.from_numpy(y).cuda(), wd, grad, loss, alpha=4.0)
    assert ei.value.name == "EINVAL"
