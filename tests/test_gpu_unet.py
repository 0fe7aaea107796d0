"""GPU parity of the BF16 MFMA network operators against the FP64 oracle.

Inputs and weights are rounded to BF16 first and the same rounded values go
to the oracle; the kernels accumulate in FP32, so FP32 outputs agree to
~1e-6 and BF16 outputs to one BF16 rounding.
"""
import ctypes

import numpy as np
import pytest

from oracle import nn as N

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def C_():
    from paper_2310_00810_amd import _lib as C
    return C


def bf(a):
    """Round to BF16 and back (float64), via torch."""
    return torch.from_numpy(np.asarray(a, np.float32)).to(torch.bfloat16).to(torch.float64).numpy()


def dev_bf(a):
    return torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(torch.bfloat16).cuda()


def rel(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def conv_call(x, W, bias, ks, dims, cout, flags=0, out32=True, grid=None, cin=None, in_cs=None, in_co=0,
              out=None, out_cs=None, out_co=0):
    C = C_()
    L = C.nnlib()
    n, d, h, w = grid if grid is not None else x.shape[:4]
    cin = cin if cin is not None else x.shape[-1]
    in_cs = in_cs if in_cs is not None else x.shape[-1]
    if out is None:
        out_shape = (n, d, h, w, cout)
        out = torch.zeros(out_shape, dtype=torch.float32 if out32 else torch.bfloat16, device="cuda")
    out_cs = out_cs if out_cs is not None else out.shape[-1]
    desc = C.lbmnn_conv_desc(n, d, h, w, dims, ks, cin, cout, flags, x.data_ptr(), in_cs, in_co,
                             None if out32 else out.data_ptr(), out.data_ptr() if out32 else None, out_cs, out_co)
    b = ctypes.c_void_p(bias.data_ptr()) if bias is not None else None
    C.check(L.lbmnn_conv(ctypes.byref(desc), ctypes.c_void_p(W.data_ptr()), b, stream()), "conv")
    torch.cuda.synchronize()
    return out


def wgrad_call(x, g, ks, dims, rows, flags=0, grid=None, splits=7, g_cs=None, cin=None, in_co=0, g_co=0):
    C = C_()
    L = C.nnlib()
    n, d, h, w = grid if grid is not None else x.shape[:4]
    cin = cin or x.shape[-1]
    K = cin * ks ** dims
    need = L.lbmnn_wgrad_workspace_bytes(n * d * h * w, rows, K, splits)
    ws = torch.empty(need // 4 + 1, dtype=torch.float32, device="cuda")
    dw = torch.zeros(rows, K, dtype=torch.float32, device="cuda")
    desc = C.lbmnn_conv_desc(n, d, h, w, dims, ks, cin, 0, flags, x.data_ptr(), x.shape[-1], in_co, None, None, 0, 0)
    C.check(L.lbmnn_conv_wgrad(ctypes.byref(desc), ctypes.c_void_p(g.data_ptr()), g_cs or g.shape[-1], g_co, rows,
                               ctypes.c_void_p(dw.data_ptr()), 0, ctypes.c_void_p(ws.data_ptr()), ws.numel() * 4,
                               splits, stream()), "wgrad")
    torch.cuda.synchronize()
    return dw


def transpose_call(W, rows, taps, cols, flip):
    C = C_()
    out = torch.empty_like(W)
    C.check(C.nnlib().lbmnn_weight_transpose(ctypes.c_void_p(W.data_ptr()), ctypes.c_void_p(out.data_ptr()), rows,
                                             taps, cols, flip, stream()), "transpose")
    return out


# 3 x 3 (x 3) layers with input channels in multiples of 32, on planes of multiples of 8 x 32 pixels
# and with at least 512 blocks, take the halo-tiled kernel: entries 3 (64 columns, two chunks), 6
# (40 of 64 columns), 7 (32 columns), 8 (3D, 32 columns, planes on both z faces) and 9 (3D, 40 of
# 64 columns, two chunks), and the input gradients of 3, 7 and 8; the others (among them 10, a 3D
# layer of 256 tiles) the im2col kernel
CASES = [(2, 3, (2, 1, 20, 24), 16, 24), (2, 1, (2, 1, 8, 16), 32, 8), (2, 3, (2, 1, 256, 256), 64, 64),
         (3, 3, (1, 6, 8, 10), 8, 16), (2, 3, (1, 1, 64, 64), 64, 32), (2, 3, (2, 1, 256, 256), 32, 40),
         (2, 3, (2, 1, 256, 256), 32, 32), (3, 3, (2, 16, 64, 64), 32, 32), (3, 3, (4, 8, 64, 64), 64, 40),
         (3, 3, (2, 32, 32, 32), 32, 64), (2, 3, (2, 1, 256, 256), 8, 32), (2, 3, (2, 1, 256, 256), 24, 32),
         (3, 3, (2, 16, 64, 64), 8, 32)]


@pytest.mark.parametrize("dims,ks,grid,cin,cout", CASES)
def test_conv_forward_fp32(dims, ks, grid, cin, cout):
    rng = np.random.default_rng(1)
    x = bf(rng.standard_normal(grid + (cin,)))
    W = bf(rng.standard_normal((cout, ks ** dims, cin)) / np.sqrt(cin * ks ** dims))
    b = rng.standard_normal(cout).astype(np.float32)
    y = conv_call(dev_bf(x), dev_bf(W.reshape(cout, -1)), torch.from_numpy(b).cuda(), ks, dims, cout)
    ref = N.conv_fwd(x, W, b.astype(np.float64), ks, dims)
    assert rel(y.cpu().numpy(), ref) <= 1e-5


@pytest.mark.parametrize("dims,ks,grid,cin,cout", CASES[:3])
def test_conv_forward_bf16_relu_and_accumulate(dims, ks, grid, cin, cout):
    rng = np.random.default_rng(2)
    x = bf(rng.standard_normal(grid + (cin,)))
    W = bf(rng.standard_normal((cout, ks ** dims, cin)) / np.sqrt(cin * ks ** dims))
    C = C_()
    y = conv_call(dev_bf(x), dev_bf(W.reshape(cout, -1)), None, ks, dims, cout, flags=C.NN_RELU, out32=False)
    ref = np.maximum(N.conv_fwd(x, W, None, ks, dims), 0)
    got = y.to(torch.float64).cpu().numpy()
    # BF16 rounding of the output, plus the FP32 accumulation error before it, which dominates
    # for outputs near zero (about 1e-6 over K = 576 for unit-variance outputs)
    assert np.all(np.abs(got - ref) <= 2 ** -7 * np.abs(ref) + 1e-5)
    # accumulate into an existing BF16 tensor, writing a channel slice of a wider buffer
    base = bf(rng.standard_normal(grid + (2 * cout,)))
    buf = dev_bf(base)
    conv_call(dev_bf(x), dev_bf(W.reshape(cout, -1)), None, ks, dims, cout, flags=C.NN_ACCUMULATE, out32=False,
              out=buf, out_cs=2 * cout, out_co=cout)
    got = buf.to(torch.float64).cpu().numpy()
    assert np.array_equal(got[..., :cout], base[..., :cout])
    exp = base[..., cout:] + N.conv_fwd(x, W, None, ks, dims)
    assert np.all(np.abs(got[..., cout:] - exp) <= 2 ** -7 * np.abs(exp) + 1e-5)


@pytest.mark.parametrize("dims,ks,grid,cin,cout", CASES)
def test_conv_input_gradient(dims, ks, grid, cin, cout):
    rng = np.random.default_rng(3)
    g = bf(rng.standard_normal(grid + (cout,)))
    W = bf(rng.standard_normal((cout, ks ** dims, cin)) / np.sqrt(cin))
    Wt = transpose_call(dev_bf(W.reshape(-1)), cout, ks ** dims, cin, 1)
    dx = conv_call(dev_bf(g), Wt, None, ks, dims, cin)
    ref = N.conv_dgrad(g, W, ks, dims, cin)
    assert rel(dx.cpu().numpy(), ref) <= 1e-5


@pytest.mark.parametrize("dims,ks,grid,cin,cout", CASES)
def test_conv_weight_gradient(dims, ks, grid, cin, cout):
    rng = np.random.default_rng(4)
    x = bf(rng.standard_normal(grid + (cin,)))
    g = bf(rng.standard_normal(grid + (cout,)))
    dw = wgrad_call(dev_bf(x), dev_bf(g), ks, dims, cout)
    ref, _ = N.conv_wgrad(x, g, ks, dims)
    assert rel(dw.cpu().numpy(), ref.reshape(cout, -1)) <= 1e-5


# 3x3 (2D) and 3x3x3 (3D, one launch per plane offset) layers whose rows and
# channels come in multiples of 32 take the halo-staged kernel: 64-row blocks,
# 32-row blocks of 64 channels, and 32-row blocks of 32 channels with the taps
# split over two wavefront pairs, 8-channel layers with the taps split over
# the four wavefronts; patches of 4 x 32 pixels (w > 16) or 8 x 16 (w <= 16),
# ragged at the right and bottom edges, several per block (splits) or all in
# one (splits = 1); the operands are channel slices of wider buffers.  w < 16
# takes the generic kernel.
HALO = [(2, (3, 1, 18, 45), 64, 64, 7), (2, (2, 1, 13, 16), 32, 32, 5), (2, (1, 1, 30, 40), 128, 32, 3),
        (2, (1, 1, 16, 16), 64, 128, 1), (2, (2, 1, 37, 70), 32, 32, 64), (2, (2, 1, 9, 12), 32, 64, 2),
        (2, (1, 1, 5, 33), 96, 64, 1), (2, (2, 1, 20, 40), 8, 32, 3), (2, (1, 1, 16, 16), 8, 64, 1),
        (3, (2, 5, 12, 40), 32, 32, 7), (3, (1, 3, 9, 16), 64, 64, 3), (3, (1, 4, 6, 20), 8, 32, 2),
        (3, (2, 2, 8, 33), 64, 32, 1)]


@pytest.mark.parametrize("dims,grid,cin,cout,splits", HALO)
def test_halo_weight_gradient(dims, grid, cin, cout, splits):
    rng = np.random.default_rng(14)
    x = bf(rng.standard_normal(grid + (cin + 16,)))
    g = bf(rng.standard_normal(grid + (cout + 8,)))
    dw = wgrad_call(dev_bf(x), dev_bf(g), 3, dims, cout, splits=splits, cin=cin, in_co=16, g_co=8)
    ref, _ = N.conv_wgrad(x[..., 16:], g[..., 8:], 3, dims)
    assert rel(dw.cpu().numpy(), ref.reshape(cout, -1)) <= 1e-5


# Deep, low-resolution layers (few output tiles, long K) split their K loop
# through the workspace entry point: FP32 output with accumulate, BF16 output
# with bias and ReLU, a D2S transposed convolution and an S2D input gradient
# (both accumulating).
SPLITK = [(3, 3, (2, 8, 8, 8), 64, 128, "f32acc"), (3, 3, (1, 4, 8, 8), 128, 64, "bf16relu"),
          (2, 3, (1, 1, 8, 8), 256, 256, "f32acc"), (2, 1, (1, 1, 4, 4), 512, 128, "d2s"),
          (3, 1, (1, 2, 4, 4), 256, 64, "s2d")]


@pytest.mark.parametrize("dims,ks,grid,cin,cout,mode", SPLITK)
def test_split_k_convolution(dims, ks, grid, cin, cout, mode):
    C = C_()
    L = C.nnlib()
    rng = np.random.default_rng(21)
    n, d, h, w = grid
    S = 1 << dims
    if mode == "s2d":
        fine = (n, 2 * d if dims == 3 else 1, 2 * h, 2 * w)
        x = bf(rng.standard_normal(fine + (cin,)))
        W = bf(rng.standard_normal((S * cin, cout)) / np.sqrt(S * cin))        # transposed-conv weights [S*cr][cin]
        Wt = transpose_call(dev_bf(W.reshape(-1)), S * cin, 1, cout, 0)
        flags, wdev, ocols = C.NN_S2D | C.NN_ACCUMULATE, Wt, cout
    elif mode == "d2s":
        x = bf(rng.standard_normal(grid + (cin,)))
        W = bf(rng.standard_normal((cout, cin)) / np.sqrt(cin))
        flags, wdev, ocols = C.NN_D2S | C.NN_ACCUMULATE, dev_bf(W), cout
    else:
        x = bf(rng.standard_normal(grid + (cin,)))
        W = bf(rng.standard_normal((cout, ks ** dims, cin)) / np.sqrt(cin * ks ** dims))
        flags, wdev, ocols = (C.NN_ACCUMULATE if mode == "f32acc" else C.NN_RELU), dev_bf(W.reshape(cout, -1)), cout
    bias = rng.standard_normal(cout >> dims if mode == "d2s" else cout).astype(np.float32)
    ogrid = (n, 2 * d if dims == 3 else 1, 2 * h, 2 * w) if mode == "d2s" else grid
    ch = cout >> dims if mode == "d2s" else cout
    base = rng.standard_normal(ogrid + (ch,)).astype(np.float32).astype(np.float64)
    outs = []
    for entry in ("ws", "plain"):
        o32 = mode != "bf16relu"
        out = torch.from_numpy(base.astype(np.float32)).cuda() if o32 else \
            torch.zeros(ogrid + (ch,), dtype=torch.bfloat16, device="cuda")
        xd = dev_bf(x)
        desc = C.lbmnn_conv_desc(n, d, h, w, dims, ks, cin, ocols, flags, xd.data_ptr(), cin, 0,
                                 None if o32 else out.data_ptr(), out.data_ptr() if o32 else None, ch, 0)
        bd = torch.from_numpy(bias).cuda()
        if entry == "ws":
            need = L.lbmnn_conv_workspace_bytes(ctypes.byref(desc))
            assert need > 0, "the layer should take the split path"
            ws = torch.empty(need // 4, dtype=torch.float32, device="cuda")
            wp, bp, wsp = (ctypes.c_void_p(t.data_ptr()) for t in (wdev, bd, ws))
            C.check(L.lbmnn_conv_ws(ctypes.byref(desc), wp, bp, wsp, need, stream()), "conv_ws")
            assert L.lbmnn_conv_ws(ctypes.byref(desc), wp, bp, wsp, need - 4, stream()) == C.LBM_ENOMEM
        else:
            C.check(L.lbmnn_conv(ctypes.byref(desc), ctypes.c_void_p(wdev.data_ptr()),
                                 ctypes.c_void_p(bd.data_ptr()), stream()), "conv")
        torch.cuda.synchronize()
        outs.append(out.to(torch.float64).cpu().numpy())
    got, plain = outs
    if mode == "s2d":
        ref = N.tconv_dgrad(x, W.reshape(S, cin, cout), dims) + bias + base
    elif mode == "d2s":
        ref = N.tconv_fwd(x, W.reshape(S, cout >> dims, cin), bias.astype(np.float64), dims) + base
    else:
        ref = N.conv_fwd(x, W, bias.astype(np.float64), ks, dims)
        ref = ref + base if mode == "f32acc" else np.maximum(ref, 0.0)
    if mode == "bf16relu":
        assert np.all(np.abs(got - ref) <= 2 ** -7 * np.abs(ref) + 1e-5)
        assert np.all(np.abs(got - plain) <= 2 ** -7 * np.abs(plain) + 1e-6)
    else:
        assert rel(got, ref) <= 1e-5
        assert rel(got, plain) <= 1e-6


@pytest.mark.parametrize("dims", [2, 3])
def test_transposed_conv_all_passes(dims):
    C = C_()
    rng = np.random.default_rng(5)
    grid = (2, 1, 6, 8) if dims == 2 else (1, 3, 4, 6)
    cin, cr = 16, 8
    S = 1 << dims
    x = bf(rng.standard_normal(grid + (cin,)))
    W = bf(rng.standard_normal((S, cr, cin)) / np.sqrt(cin))
    b = rng.standard_normal(cr).astype(np.float32)
    n, d, h, w = grid
    fine = (n, 2 * d if dims == 3 else 1, 2 * h, 2 * w)
    # forward into the lower half of a concatenated buffer
    out = torch.zeros(fine + (2 * cr,), dtype=torch.float32, device="cuda")
    conv_call(dev_bf(x), dev_bf(W.reshape(S * cr, cin)), torch.from_numpy(b).cuda(), 1, dims, S * cr,
              flags=C.NN_D2S, out=out, out_cs=2 * cr, out_co=0)
    ref = N.tconv_fwd(x, W, b.astype(np.float64), dims)
    assert rel(out[..., :cr].cpu().numpy(), ref) <= 1e-5
    assert torch.count_nonzero(out[..., cr:]).item() == 0
    # input gradient: S2D gather of the fine gradient
    g = bf(rng.standard_normal(fine + (cr,)))
    Wt = transpose_call(dev_bf(W.reshape(-1)), S * cr, 1, cin, 0)
    dx = conv_call(dev_bf(g), Wt, None, 1, dims, cin, flags=C.NN_S2D, grid=grid, cin=cr, in_cs=cr)
    assert rel(dx.cpu().numpy(), N.tconv_dgrad(g, W, dims)) <= 1e-5
    # weight gradient with the gradient rows gathered on the fine grid
    dw = wgrad_call(dev_bf(x), dev_bf(g), 1, dims, S * cr, flags=C.NN_S2D_G, grid=grid, g_cs=cr)
    refw, _ = N.tconv_wgrad(x, g, dims)
    assert rel(dw.cpu().numpy(), refw.reshape(S * cr, cin)) <= 1e-5


# 16-byte kernels (channel count, strides and offsets multiples of 8) and the
# per-element ones, overwriting and accumulating, on channel slices of wider buffers.
POOL = [(8, 8, 0, 0), (16, 24, 8, 1), (12, 12, 0, 1), (6, 10, 2, 0)]


@pytest.mark.parametrize("dims", [2, 3])
@pytest.mark.parametrize("Cn,cs,co,acc", POOL)
def test_pooling_forward_backward(dims, Cn, cs, co, acc):
    C = C_()
    L = C.nnlib()
    rng = np.random.default_rng(6)
    fine = (2, 1, 8, 12) if dims == 2 else (1, 4, 6, 8)
    xw = bf(rng.standard_normal(fine + (cs,)))
    x = xw[..., co:co + Cn]
    n, fd, fh, fw = fine
    coarse = (n, fd // 2 if dims == 3 else 1, fh // 2, fw // 2)
    xd = dev_bf(xw)
    y = torch.zeros(coarse + (cs,), dtype=torch.bfloat16, device="cuda")
    C.check(L.lbmnn_pool_fwd(xd.data_ptr(), cs, co, y.data_ptr(), cs, co, *coarse, Cn, dims, stream()), "pool")
    torch.cuda.synchronize()
    yh = y.to(torch.float64).cpu().numpy()
    assert np.array_equal(yh[..., co:co + Cn], N.pool_fwd(x, dims))
    assert np.all(np.delete(yh, np.s_[co:co + Cn], axis=-1) == 0)
    gw = bf(rng.standard_normal(coarse + (cs,)))
    g = gw[..., co:co + Cn]
    base = bf(rng.standard_normal(fine + (cs,)))
    gi = dev_bf(base)
    gd = dev_bf(gw)
    C.check(L.lbmnn_pool_bwd(xd.data_ptr(), cs, co, gd.data_ptr(), cs, co, gi.data_ptr(), cs, co, *coarse, Cn,
                             dims, acc, stream()), "pool_bwd")
    torch.cuda.synchronize()
    got = gi.to(torch.float64).cpu().numpy()
    routed = N.pool_bwd(x, g, dims)
    if acc:
        exp = np.where(routed != 0, N.bf16_round(base[..., co:co + Cn] + routed), base[..., co:co + Cn])
    else:
        exp = routed
    assert np.array_equal(got[..., co:co + Cn], exp)
    assert np.array_equal(np.delete(got, np.s_[co:co + Cn], axis=-1), np.delete(base, np.s_[co:co + Cn], axis=-1))


def _oracle_params(net):
    P = {}
    for name, (kind, ci, co, ks) in net.layers.items():
        W = net.weight(name, master=False).to(torch.float64).cpu().numpy()
        b = net.bias(name).to(torch.float64).cpu().numpy()
        if kind == "tconv":
            P[name] = (W.reshape(1 << net.dims, co, ci), b)
        else:
            P[name] = (W.reshape(co, ks ** net.dims, ci), b)
    return P


@pytest.mark.parametrize("dims,shape,base,levels,wscale,bias,bar_f,bar_g", [
    (2, (2, 1, 32, 48), 8, 3, 1.0, 0.0, 2e-3, 5e-3),      # narrow: short accumulations
    (3, (1, 16, 16, 8), 8, 3, 1.0, 0.0, 2e-3, 5e-3),
    (2, (2, 1, 32, 48), 32, 4, 0.1, 1.0, 2e-3, 1e-2),     # full width, every ReLU active
    (3, (1, 16, 16, 8), 32, 4, 0.1, 1.0, 2e-3, 1e-2),
    (2, (2, 1, 32, 48), 32, 4, 1.0, 0.0, 2e-2, 0.25),     # full width at random initialisation
    (3, (1, 16, 16, 8), 32, 4, 1.0, 0.0, 2e-2, 0.25),
    (2, (1, 1, 256, 256), 32, 4, 0.1, 1.0, 2e-3, 1e-2),   # the 2D warm start's input size (halo-tiled layers)
    (3, (1, 32, 32, 32), 32, 4, 0.1, 1.0, 2e-3, 1e-2),    # 3D at half the warm start's 64^3 per axis
])
def test_unet_forward_and_gradients_match_the_oracle(dims, shape, base, levels, wscale, bias, bar_f, bar_g):
    """Whole U-Net composition: FP32 head output and every parameter gradient
    against the oracle network on the same BF16 weights and input, the oracle
    storing activations and activation gradients in BF16 where the GPU path
    does.  What remains is FP32-vs-FP64 accumulation flipping BF16
    roundings.  Where a flip changes the sign of a pre-activation, the ReLU
    derivative switches between 0 and 1 and that gradient entry differs
    wholesale, so the gradient gap scales like the square root of the flipped
    fraction: small for the narrow network (short accumulations) and for a
    full-width network with small weights and unit biases (every
    pre-activation positive, so no flips), of order 10% for the full-width
    network at random initialisation."""
    from paper_2310_00810_amd.unet import UNet
    net = UNet(dims, base=base, levels=levels, seed=3)
    torch.manual_seed(0)
    with torch.no_grad():
        net.master[:net.n_params] += 0.02 * torch.randn(net.n_params, device="cuda")  # nonzero biases
        for name in net.layers:
            net.weight(name).mul_(wscale)
            if name != "head":
                net.bias(name).add_(bias)
    net.sync_bf16()
    rng = np.random.default_rng(7)
    x = bf(rng.standard_normal(shape + (8,)))
    out = net.forward(dev_bf(x))
    P = _oracle_params(net)
    kw = dict(base=base, levels=levels)
    ref, cache = N.unet_forward(x, P, dims, quantize=N.bf16_round, **kw)
    ef = rel(out.cpu().numpy(), ref)
    g = bf(rng.standard_normal(shape + (8,)))
    net.backward(dev_bf(g))
    torch.cuda.synchronize()
    grads = N.unet_backward(g, P, cache, dims, quantize=N.bf16_round, **kw)
    errs = {}
    for name in net.layers:
        gw = net.grad[net.woff[name]:net.woff[name] + np.prod(net.wshape[name])].cpu().numpy()
        gb = net.grad[net.boff[name]:net.boff[name] + net.layers[name][2]].cpu().numpy()
        errs[name] = (rel(gw, grads[name][0].ravel()), rel(gb, grads[name][1]))
    print(f"forward {ef:.2e}", {k: (float(f"{a:.2e}"), float(f"{b:.2e}")) for k, (a, b) in errs.items()})
    assert ef <= bar_f
    for name, (ew, eb) in errs.items():
        assert ew <= bar_g and eb <= bar_g, (name, ew, eb)


# (n, d, h, w, D): ragged sections, several row groups per section (w < 1024), two section chunks
# (w = 2048, the largest accepted), and 3D
FLUX = [(3, 1, 37, 300, 2), (2, 5, 6, 64, 3), (1, 1, 4, 2048, 2), (2, 64, 64, 64, 3), (1, 1, 256, 256, 2)]


@pytest.mark.parametrize("n,d,h,w,D", FLUX)
def test_flux_balance_matches_the_oracle(n, d, h, w, D):
    C = C_()
    rng = np.random.default_rng(n * 1000 + w)
    solid = (rng.random((n, d, h, w)) > 0.6).astype(np.uint8)
    u = (rng.random((n, d, h, w, D)) + 0.05).astype(np.float32)
    u[..., 1:] -= 0.55
    u[..., 0] *= rng.uniform(0.02, 3.0, (n, 1, 1, w)).astype(np.float32)   # uneven sections, some clamped
    u[solid == 1] = 7.0                                                     # not counted in the fluxes
    if n > 1:
        u[1, ..., 0] *= -1.0                                                # a sample with no forward flow
    ud = torch.from_numpy(u).cuda()
    sd = torch.from_numpy(solid).cuda()
    L = C.nnlib()
    nb = L.lbmnn_flux_balance_workspace_bytes(n, d, h, w)
    ws = torch.full((nb // 8 + 1,), float("nan"), dtype=torch.float64, device="cuda")   # nothing read before written
    C.check(L.lbmnn_flux_balance(sd.data_ptr(), n, d, h, w, D, ud.data_ptr(), ws.data_ptr(), nb, stream()),
            "flux balance")
    torch.cuda.synchronize()
    got = ud.cpu().numpy()
    for b in range(n):
        exp = N.flux_balance(u[b].astype(np.float64), solid[b])
        assert np.allclose(got[b], exp, rtol=3e-7, atol=0), b
    if n > 1:
        assert np.array_equal(got[1], u[1])
    args = (sd.data_ptr(), n, d, h)
    assert L.lbmnn_flux_balance(*args, w, D, None, ws.data_ptr(), nb, stream()) == C.LBM_EINVAL
    assert L.lbmnn_flux_balance(*args, 2049, D, ud.data_ptr(), ws.data_ptr(), nb, stream()) == C.LBM_EINVAL
    assert L.lbmnn_flux_balance(*args, w, 4, ud.data_ptr(), ws.data_ptr(), nb, stream()) == C.LBM_EINVAL
    assert L.lbmnn_flux_balance(*args, w, D, ud.data_ptr(), ws.data_ptr(), nb - 8, stream()) == C.LBM_ENOMEM


def test_mse_adam_and_feature_maps():
    C = C_()
    L = C.nnlib()
    rng = np.random.default_rng(8)
    P, pcs, creal = 1000, 8, 3
    pred = rng.standard_normal((P, pcs)).astype(np.float32)
    tgt = rng.standard_normal((P, creal)).astype(np.float32)
    wp = (rng.uniform(size=P) > 0.3).astype(np.float32)
    dp = torch.empty(P, pcs, dtype=torch.bfloat16, device="cuda")
    part = torch.empty(8, dtype=torch.float64, device="cuda")
    loss = torch.empty(1, dtype=torch.float64, device="cuda")
    pd, td, wd = [torch.from_numpy(a).cuda() for a in (pred, tgt, wp)]
    C.check(L.lbmnn_mse(pd.data_ptr(), pcs, td.data_ptr(), wd.data_ptr(), creal, P, 0.5, dp.data_ptr(),
                        part.data_ptr(), loss.data_ptr(), stream()), "mse")
    torch.cuda.synchronize()
    lexp, gexp = N.masked_mse(pred, tgt, wp, creal, 0.5)
    assert np.isclose(loss.item(), lexp, rtol=1e-6)
    assert np.allclose(dp.to(torch.float64).cpu().numpy(), gexp, rtol=1e-2, atol=1e-6)
    # Adam: two steps against the oracle's update in float64
    n = 777
    w = rng.standard_normal(n).astype(np.float32)
    gs = [rng.standard_normal(n).astype(np.float32) for _ in range(2)]
    wd_ = torch.from_numpy(w).cuda()
    m1 = torch.zeros(n, device="cuda")
    m2 = torch.zeros(n, device="cuda")
    wb = torch.empty(n, dtype=torch.bfloat16, device="cuda")
    mm, vv, ww = np.zeros(n), np.zeros(n), w.astype(np.float64)
    for t, gg in enumerate(gs, 1):
        gdev = torch.from_numpy(gg).cuda()      # kept alive until the kernel has run
        C.check(L.lbmnn_adam(wd_.data_ptr(), gdev.data_ptr(), m1.data_ptr(), m2.data_ptr(),
                             wb.data_ptr(), n, 1e-2, 0.9, 0.999, 1e-8, t, stream()), "adam")
        torch.cuda.synchronize()
        ww, mm, vv = N.adam(ww, gg, mm, vv, 1e-2, 0.9, 0.999, 1e-8, t)
    torch.cuda.synchronize()
    assert np.allclose(wd_.cpu().numpy(), ww, atol=1e-5)
    assert torch.equal(wb, wd_.to(torch.bfloat16))
    # Stokes normalisation round trip
    Pn, D = 64, 2
    solid = (rng.uniform(size=Pn) > 0.7).astype(np.uint8)
    prm = np.array([[0.004, 0.0, 0.8]], np.float32)
    drho = rng.uniform(0, 0.004, Pn).astype(np.float32)
    u = rng.standard_normal((Pn, D)).astype(np.float32) * 1e-3
    tg = torch.empty(Pn, 1 + D, device="cuda")
    wpx = torch.empty(Pn, device="cuda")
    sd, pr = torch.from_numpy(solid).cuda(), torch.from_numpy(prm).cuda()
    drho_d, u_d = torch.from_numpy(drho).cuda(), torch.from_numpy(u).cuda()
    C.check(L.lbmnn_normalize(drho_d.data_ptr(), u_d.data_ptr(), sd.data_ptr(), pr.data_ptr(), Pn, D, Pn,
                              tg.data_ptr(), wpx.data_ptr(), stream()), "norm")
    pred8 = torch.zeros(Pn, 8, device="cuda")
    pred8[:, :1 + D] = tg
    r2 = torch.empty(Pn, device="cuda")
    u2 = torch.empty(Pn, D, device="cuda")
    C.check(L.lbmnn_denormalize(pred8.data_ptr(), 8, sd.data_ptr(), pr.data_ptr(), Pn, D, Pn, r2.data_ptr(),
                                u2.data_ptr(), stream()), "denorm")
    torch.cuda.synchronize()
    fl = solid == 0
    texp = N.stokes_targets(drho, u, solid, 0.004, 0.0, 0.8)
    assert np.allclose(tg.cpu().numpy(), texp, rtol=1e-5, atol=1e-9)
    r_exp, u_exp = N.stokes_fields(pred8.cpu().numpy(), solid, 0.004, 0.0, 0.8, D)
    assert np.allclose(r2.cpu().numpy(), r_exp, rtol=1e-5, atol=1e-9)
    assert np.allclose(u2.cpu().numpy(), u_exp, rtol=1e-5, atol=1e-10)
    assert np.allclose(r2.cpu().numpy()[fl], drho[fl], rtol=1e-5, atol=1e-9)
    assert np.allclose(u2.cpu().numpy()[fl], u[fl], rtol=1e-5, atol=1e-10)
    assert np.all(wpx.cpu().numpy() == fl)


@pytest.mark.parametrize("npix,cs,co,Cn", [(5000, 64, 32, 32), (3001, 16, 0, 16), (777, 24, 3, 12)])
def test_fused_relu_backward_and_bias_gradient(npix, cs, co, Cn):
    """One pass (ReLU backward, then the bias gradient of the masked g) gives
    bit for bit what the two separate operations give, on the 16-byte path
    and on layouts that fall back to the separate kernels; the bias gradient
    against a float64 sum of the masked BF16 values."""
    C = C_()
    L = C.nnlib()
    rng = np.random.default_rng(npix)
    g0 = dev_bf(rng.standard_normal((npix, cs)))
    y = dev_bf(rng.standard_normal((npix, cs)))
    splits = 11
    ws = torch.empty(splits * Cn, dtype=torch.float32, device="cuda")
    ga, gb = g0.clone(), g0.clone()
    da = torch.zeros(Cn, dtype=torch.float32, device="cuda")
    db = torch.zeros(Cn, dtype=torch.float32, device="cuda")
    C.check(L.lbmnn_relu_bwd(ga.data_ptr(), y.data_ptr(), cs, co, npix, Cn, stream()), "relu_bwd")
    C.check(L.lbmnn_bias_grad(ga.data_ptr(), cs, co, npix, Cn, da.data_ptr(), 0, ws.data_ptr(), splits, stream()),
            "bias_grad")
    C.check(L.lbmnn_relu_bwd_bias_grad(gb.data_ptr(), y.data_ptr(), cs, co, npix, Cn, db.data_ptr(), 0,
                                       ws.data_ptr(), splits, stream()), "relu_bwd_bias_grad")
    torch.cuda.synchronize()
    assert torch.equal(ga, gb) and torch.equal(da, db)
    gm = g0.float().cpu().numpy()[:, co:co + Cn].astype(np.float64)
    gm[y.float().cpu().numpy()[:, co:co + Cn] <= 0] = 0
    assert np.array_equal(gb.float().cpu().numpy()[:, co:co + Cn], gm)
    assert np.allclose(db.cpu().numpy(), gm.sum(0), rtol=1e-5, atol=1e-4)
