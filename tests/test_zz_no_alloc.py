"""The allocation-free weight gradient (lbmnn_conv_wgrad_noalloc) against the
workspace entry point (lbmnn_conv_wgrad), through the C ABI: the same kernels
on the same inputs, so the results agree bit for bit.  Two calls in a row,
the second on a smaller layer (the shared scratch keeps the first call's
partials), and a size beyond the scratch is refused before any launch."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _layer(n, h, w, cin, rows, seed):
    g = torch.Generator().manual_seed(seed)
    x = torch.randn(n, 1, h, w, cin, generator=g).to(torch.bfloat16).cuda()
    gy = torch.randn(n, 1, h, w, rows, generator=g).to(torch.bfloat16).cuda()
    return x, gy


def _wgrad(x, gy, rows, splits, noalloc):
    from paper_2310_00810_amd import _lib as C
    L = C.nnlib()
    n, d, h, w, cin = x.shape
    K = 9 * cin
    desc = C.lbmnn_conv_desc(n, d, h, w, 2, 3, cin, 0, 0, x.data_ptr(), cin, 0, None, None, 0, 0)
    dw = torch.full((rows, K), float("nan"), dtype=torch.float32, device="cuda")
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if noalloc:
        rc = L.lbmnn_conv_wgrad_noalloc(ctypes.byref(desc), ctypes.c_void_p(gy.data_ptr()), rows, 0, rows,
                                        ctypes.c_void_p(dw.data_ptr()), 0, splits, stream)
    else:
        need = L.lbmnn_wgrad_workspace_bytes(n * d * h * w, rows, K, splits)
        ws = torch.empty(need // 4 + 1, dtype=torch.float32, device="cuda")
        rc = L.lbmnn_conv_wgrad(ctypes.byref(desc), ctypes.c_void_p(gy.data_ptr()), rows, 0, rows,
                                ctypes.c_void_p(dw.data_ptr()), 0, ctypes.c_void_p(ws.data_ptr()), ws.numel() * 4,
                                splits, stream)
    C.check(rc, "wgrad")
    torch.cuda.synchronize()
    return dw


def test_noalloc_weight_gradient_matches_the_workspace_entry_point():
    big = (_layer(4, 64, 64, 64, 128, seed=1), 128, 9)
    small = (_layer(1, 24, 40, 16, 32, seed=2), 32, 3)
    for (x, gy), rows, splits in (big, small):
        ref = _wgrad(x, gy, rows, splits, noalloc=False)
        got = _wgrad(x, gy, rows, splits, noalloc=True)
        assert torch.isfinite(ref).all()
        assert torch.equal(got, ref)


def test_noalloc_weight_gradient_refuses_partials_beyond_its_scratch():
    from paper_2310_00810_amd import _lib as C
    L = C.nnlib()
    x, gy = _layer(1, 256, 256, 256, 256, seed=3)
    K, splits = 9 * 256, 64
    assert L.lbmnn_wgrad_workspace_bytes(256 * 256, 256, K, splits) > C.LBMNN_NOALLOC_SCRATCH_BYTES
    desc = C.lbmnn_conv_desc(1, 1, 256, 256, 2, 3, 256, 0, 0, x.data_ptr(), 256, 0, None, None, 0, 0)
    dw = torch.zeros(256, K, dtype=torch.float32, device="cuda")
    rc = L.lbmnn_conv_wgrad_noalloc(ctypes.byref(desc), ctypes.c_void_p(gy.data_ptr()), 256, 0, 256,
                                    ctypes.c_void_p(dw.data_ptr()), 0, splits,
                                    ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == C.LBM_ENOMEM
    assert b"scratch" in L.lbm_last_error()
    assert torch.count_nonzero(dw).item() == 0
