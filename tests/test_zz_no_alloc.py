"""The allocation-free gradient entry point (iblbm_nn_grad_noalloc) against
iblbm_nn_grad on the same samples and parameters: two calls in a row, the second with
fewer samples, so that the shared device scratch holds the first call's values when the
second starts.  The two entry points run the same kernels in the same order, so the
gradients and the loss agree exactly."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
NPARAM = 10 * 64 + 64 + 64 * 64 + 64 + 64 * 3 + 3


def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2002_08855_amd import binding
    return torch, binding


def _case(seed, n):
    rng = np.random.default_rng(seed)
    P = rng.normal(0, 0.25, NPARAM).astype(np.float32)
    x = rng.normal(size=(n, 10)).astype(np.float32)
    t = rng.normal(size=(n, 3)).astype(np.float32)
    return P, x, t


def _noalloc(torch, b, P, x, t):
    dev = torch.device("cuda", 0)
    dx = torch.from_numpy(x).to(dev)
    dt = torch.from_numpy(t).to(dev)
    dP = torch.from_numpy(P).to(dev)
    loss = torch.full((1,), float("nan"), dtype=torch.float32, device=dev)
    grad = torch.full((NPARAM,), float("nan"), dtype=torch.float32, device=dev)
    stream = torch.cuda.current_stream(dev)
    torch.cuda.synchronize()
    b.nn_grad_noalloc(dx.data_ptr(), dt.data_ptr(), x.shape[0], dP.data_ptr(), loss.data_ptr(),
                      grad.data_ptr(), stream.cuda_stream)
    torch.cuda.synchronize()
    return float(loss.cpu().numpy()[0]), grad.cpu().numpy()


def test_noalloc_gradient_matches_nn_grad_two_calls():
    torch, b = _gpu()
    for seed, n in ((31, 4096), (32, 1000)):
        print(f"case seed={seed} n={n}", flush=True)
        P, x, t = _case(seed, n)
        lref, gref = b.nn_grad(P, x, t)
        lna, gna = _noalloc(torch, b, P, x, t)
        print("loss", lref, lna, "max |dg|", np.abs(gna - gref).max(), flush=True)
        assert np.all(np.isfinite(gna))
        assert lna == lref
        assert np.array_equal(gna, gref)


def test_noalloc_rejects_sizes_beyond_the_scratch():
    """More samples than the scratch holds, or a NULL pointer: refused on the host before
    any device work."""
    torch, b = _gpu()
    cap = 8192
    dev = torch.device("cuda", 0)
    buf = torch.zeros(16, dtype=torch.float32, device=dev)
    with pytest.raises(b.IblbmError) as e:
        b.nn_grad_noalloc(buf.data_ptr(), buf.data_ptr(), cap + 1, buf.data_ptr(),
                          buf.data_ptr(), buf.data_ptr(), None)
    assert "E_CAPACITY" in str(e.value)
    with pytest.raises(b.IblbmError) as e:
        b.nn_grad_noalloc(None, buf.data_ptr(), 8, buf.data_ptr(), buf.data_ptr(),
                          buf.data_ptr(), None)
    assert "E_ARG" in str(e.value)
    assert ctypes.sizeof(ctypes.c_void_p) == 8
