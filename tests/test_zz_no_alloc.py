"""flash_mlp_grad_noalloc against flash_mlp_grad through the C ABI.

The no-allocation variant keeps its scratch in a static device array and takes the network
parameters as a device input; it must give the trainer's gradient and loss for the same
parameters and rows.  Two calls in a row, the second with fewer rows, so that the second call
runs on scratch that still holds the first call's values; a third call beyond the row limit
must be refused.
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_grad_noalloc_matches_trainer_gradient():
    import torch
    from paper_2604_17513_amd import flash as F
    L = F.lib()
    fn = L.flash_mlp_grad_noalloc
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(7)
    m = F.Mlp(4096, seed=3)
    theta = m.params()
    theta += rng.normal(scale=0.01, size=theta.shape).astype(np.float32)   # non-zero biases too
    m.set_params(theta)
    params = torch.tensor(theta, device=dev)
    grad = torch.empty(F.MLP_PARAMS, dtype=torch.float32, device=dev)
    loss = torch.empty(1, dtype=torch.float32, device=dev)
    stream = torch.cuda.current_stream(dev).cuda_stream
    for n in (2048, 333):
        x = torch.tensor(rng.normal(size=(n, F.MLP_FEATURES)).astype(np.float32), device=dev)
        t = torch.tensor(rng.normal(size=(n, F.MLP_OUTPUTS)).astype(np.float32), device=dev)
        torch.cuda.synchronize()
        g_ref, l_ref = m.grad(x, t, n)
        grad.fill_(float("nan"))
        st = fn(params.data_ptr(), x.data_ptr(), t.data_ptr(), n, grad.data_ptr(), loss.data_ptr(), stream)
        assert st == F.FLASH_OK, L.flash_last_error().decode()
        torch.cuda.synchronize()
        g = grad.cpu().numpy()
        lo = float(loss.cpu().numpy()[0])
        err = float(np.abs(g - g_ref).max())
        _say(f"rows {n}: loss {lo:.6e} vs {l_ref:.6e}, max |dgrad| {err:.3e}, bitwise {np.array_equal(g, g_ref)}")
        assert np.all(np.isfinite(g))
        assert np.array_equal(g, g_ref) and lo == l_ref
    # beyond the scratch's row limit: refused before anything is launched
    n = 2049
    x = torch.zeros((n, F.MLP_FEATURES), dtype=torch.float32, device=dev)
    t = torch.zeros((n, F.MLP_OUTPUTS), dtype=torch.float32, device=dev)
    st = fn(params.data_ptr(), x.data_ptr(), t.data_ptr(), n, grad.data_ptr(), loss.data_ptr(), stream)
    assert st == F.FLASH_ERR_CAPACITY
    assert "2048" in L.flash_last_error().decode()
