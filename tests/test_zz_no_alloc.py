"""acm_cnn_loss_noalloc (the entry point that allocates nothing) against
acm_cnn_loss (caller workspace) through the C ABI: same loss bits and same
gradient bytes on two calls in a row, the second on a smaller grid, and a
clear error beyond the static scratch's limit."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available()
    from paper_2012_03525_amd import acm
    acm.lib()
    return acm, torch


def _vp(t):
    return ctypes.c_void_p(t.data_ptr())


def _case(torch, nx, ny, seed):
    g = torch.Generator(device="cpu").manual_seed(seed)
    raw = torch.randn((ny, nx, 16), generator=g, dtype=torch.float32).cuda()
    base = [torch.randn((ny, nx), generator=g, dtype=torch.float32).cuda() * 0.01 for _ in range(3)]
    target = [b + torch.randn((ny, nx), generator=g, dtype=torch.float32).cuda() * 1e-3 for b in base]
    return raw, base, target


def _call(acm, torch, nx, ny, raw, base, target, scale, noalloc):
    L = acm.lib()
    grad = torch.full((ny, nx, 16), 7.0, dtype=torch.bfloat16, device="cuda")  # overwritten
    loss = torch.full((1,), -1.0, dtype=torch.float64, device="cuda")
    b = (ctypes.c_void_p * 3)(*[t.data_ptr() for t in base])
    t = (ctypes.c_void_p * 3)(*[x.data_ptr() for x in target])
    sc = (ctypes.c_float * 3)(*scale)
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if noalloc:
        st = L.acm_cnn_loss_noalloc(nx, ny, _vp(raw), b, t, sc, _vp(grad), _vp(loss), s)
    else:
        ws = torch.empty(L.acm_cnn_loss_workspace(nx, ny), dtype=torch.uint8, device="cuda")
        st = L.acm_cnn_loss(nx, ny, _vp(raw), b, t, sc, _vp(grad), _vp(ws), _vp(loss), s)
    acm.check(st)
    torch.cuda.synchronize()
    return loss.cpu().numpy().copy(), grad.view(torch.int16).cpu().numpy().copy()


def test_noalloc_loss_equals_workspace_loss_twice(env):
    acm, torch = env
    L = acm.lib()
    L.acm_cnn_loss_noalloc.restype = ctypes.c_int
    L.acm_cnn_loss_noalloc.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p,
                                       ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_void_p),
                                       ctypes.POINTER(ctypes.c_float), ctypes.c_void_p, ctypes.c_void_p,
                                       ctypes.c_void_p]
    # first a large grid (4096 partial sums), then a smaller one whose partials
    # occupy only the front of the shared static array
    for nx, ny, scale, seed in [(1024, 1024, (0.5, 2.0, 1.5), 1), (96, 40, (0.0, 1.0, 3.0), 2)]:
        raw, base, target = _case(torch, nx, ny, seed)
        ref_loss, ref_grad = _call(acm, torch, nx, ny, raw, base, target, scale, noalloc=False)
        got_loss, got_grad = _call(acm, torch, nx, ny, raw, base, target, scale, noalloc=True)
        assert np.isfinite(ref_loss[0]) and ref_loss[0] > 0
        assert got_loss.tobytes() == ref_loss.tobytes(), (nx, ny, got_loss, ref_loss)
        assert np.array_equal(got_grad, ref_grad), (nx, ny)
    # beyond the static scratch: ACM_EINVAL before any launch
    big_nx, big_ny = 2048, 1040  # 2,129,920 pixels > 8192 * 256
    raw = torch.empty(1, device="cuda")
    p3 = (ctypes.c_void_p * 3)(raw.data_ptr(), raw.data_ptr(), raw.data_ptr())
    sc = (ctypes.c_float * 3)(1.0, 1.0, 1.0)
    st = L.acm_cnn_loss_noalloc(big_nx, big_ny, _vp(raw), p3, p3, sc, _vp(raw), _vp(raw), None)
    assert st == acm.EINVAL
    assert b"static scratch" in L.acm_last_error()
