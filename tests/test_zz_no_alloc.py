"""The no-allocation entry point mlp_loss_grad_noalloc (library-held
workspace) against mlp_loss_grad with a caller workspace, through the C
interface: two calls in a row on the same device, the second with a
smaller batch (the library's workspace then holds the first call's
contents), and the batch limit."""
import ctypes as ct

import numpy as np
import pytest

from paper_1904_02108_amd import workload as W

pytestmark = pytest.mark.gpu
NP = 9347


@pytest.fixture(scope="module")
def L():
    import torch
    assert torch.cuda.is_available()
    torch.cuda.set_device(0)
    from paper_1904_02108_amd import lbmibm
    return lbmibm


def _dev(a):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32), device="cuda")


def _case(n, seed):
    rng = np.random.default_rng(seed)
    th = W.mlp_init(seed, scale=1.5)
    x = rng.normal(size=(n, 12)).astype(np.float32)
    t = rng.normal(size=(n, 3)).astype(np.float32)
    return th, x, t


def _with_workspace(L, th, x, t):
    import torch
    n = x.shape[0]
    dth, dx, dt = _dev(th), _dev(x), _dev(t)
    grad = torch.empty(NP, dtype=torch.float32, device="cuda")
    loss = torch.empty(1, dtype=torch.float64, device="cuda")
    ws = torch.empty(L.mlp_workspace_size(n), dtype=torch.uint8, device="cuda")
    st = torch.cuda.current_stream().cuda_stream
    L.mlp_loss_grad(dth.data_ptr(), n, dx.data_ptr(), dt.data_ptr(), grad.data_ptr(),
                    loss.data_ptr(), ws.data_ptr(), st)
    torch.cuda.synchronize()
    return grad.cpu().numpy(), float(loss.cpu().numpy()[0])


def _noalloc(L, th, x, t):
    import torch
    n = x.shape[0]
    dth, dx, dt = _dev(th), _dev(x), _dev(t)
    grad = torch.full((NP,), float("nan"), dtype=torch.float32, device="cuda")
    loss = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
    st = torch.cuda.current_stream().cuda_stream
    L.mlp_loss_grad_noalloc(dth.data_ptr(), n, dx.data_ptr(), dt.data_ptr(), grad.data_ptr(),
                            loss.data_ptr(), st)
    torch.cuda.synchronize()
    return grad.cpu().numpy(), float(loss.cpu().numpy()[0])


def test_noalloc_matches_workspace_entry_point_twice(L):
    """Same kernels, same fixed-order reductions: bit-identical gradient and
    loss, on a full batch and then on a smaller one."""
    for n, seed in ((L.MLP_NOALLOC_MAX_BATCH, 7), (333, 8)):
        print("mlp_loss_grad_noalloc n =", n, flush=True)
        th, x, t = _case(n, seed)
        g_ref, l_ref = _with_workspace(L, th, x, t)
        g, l = _noalloc(L, th, x, t)
        assert np.isfinite(g).all() and np.isfinite(l)
        assert np.array_equal(g, g_ref)
        assert l == l_ref


def test_noalloc_rejects_batches_beyond_the_limit(L):
    import torch
    n = L.MLP_NOALLOC_MAX_BATCH + 1
    dummy = torch.zeros(16, dtype=torch.float32, device="cuda")
    p = dummy.data_ptr()
    with pytest.raises(L.LbmError) as ei:
        L.mlp_loss_grad_noalloc(p, n, p, p, p, 0, torch.cuda.current_stream().cuda_stream)
    assert ei.value.status == L.LBM_ERR_ARG
    assert "exceeds" in str(ei.value)
