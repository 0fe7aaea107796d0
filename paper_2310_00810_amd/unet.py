"""Warm-start U-Net on the lbmnn_* MFMA kernels.

A 4-level U-Net (base 32 channels, two 3x3 / 3x3x3 convolutions with ReLU
per level, 2x2(x2) max pooling, 2x2(x2) stride-2 transposed convolutions,
skip connections by concatenation, 1x1 head) maps the solid mask and the
boundary / viscosity parameters to the Stokes-scaled steady density and
velocity.  Its output only initialises the LBM (the paper's proposed
neural-network initial guess, Section 3.1.2 end and Section 3.5).

Weights: FP32 master copy + BF16 mirror used by the kernels; activations
BF16 channels-last; every operator is a liblbm.so kernel, torch only holds
the buffers.  Concatenation is by layout: the encoder's second convolution
writes its output into the upper half of the decoder's concatenated buffer
and the transposed convolution into the lower half.
"""
from __future__ import annotations

import ctypes
import math

import torch

from . import _lib as C

BF16 = torch.bfloat16


def _ptr(t, elem_off=0):
    return ctypes.c_void_p(t.data_ptr() + elem_off * t.element_size()) if t is not None else None


class UNet:
    def __init__(self, dims, base=32, levels=4, cin=8, cout=8, creal=None, seed=0, device="cuda"):
        assert dims in (2, 3)
        self.dims, self.base, self.levels, self.cin, self.cout = dims, base, levels, cin, cout
        self.creal = creal if creal is not None else 1 + dims
        self.device = torch.device(device)
        self.L = C.nnlib()
        # layer table: name -> (kind, ci, co, ks); weights W [rows][K] with
        # rows = co (conv) or 2^dims co (transposed conv)
        self.layers = {}
        c = cin
        for lv in range(levels):
            co = base << lv
            self.layers[f"e{lv}c0"] = ("conv", c, co, 3)
            self.layers[f"e{lv}c1"] = ("conv", co, co, 3)
            c = co
        for lv in range(levels - 2, -1, -1):
            co = base << lv
            self.layers[f"d{lv}t"] = ("tconv", 2 * co, co, 1)
            self.layers[f"d{lv}c0"] = ("conv", 2 * co, co, 3)
            self.layers[f"d{lv}c1"] = ("conv", co, co, 3)
        self.layers["head"] = ("conv", base, cout, 1)
        self.woff, self.boff, self.wshape = {}, {}, {}
        off = 0
        for name, (kind, ci, co, ks) in self.layers.items():
            rows = co * (1 << dims) if kind == "tconv" else co
            K = ci * (ks ** dims)
            self.wshape[name] = (rows, K)
            self.woff[name] = off
            off += rows * K
        for name, (kind, ci, co, ks) in self.layers.items():
            self.boff[name] = off
            off += co
        self.n_params = off
        n8 = (off + 7) // 8 * 8
        dev = self.device
        self.master = torch.zeros(n8, dtype=torch.float32, device=dev)
        self.grad = torch.zeros(n8, dtype=torch.float32, device=dev)
        self.m1 = torch.zeros(n8, dtype=torch.float32, device=dev)
        self.m2 = torch.zeros(n8, dtype=torch.float32, device=dev)
        self.wbf = torch.zeros(n8, dtype=BF16, device=dev)
        self.wT = torch.zeros(n8, dtype=BF16, device=dev)
        self.t = 0
        self._bufs = {}
        self._ws = torch.empty(0, dtype=torch.float32, device=dev)
        self._bws = torch.empty(1 << 18, dtype=torch.float32, device=dev)
        self._mse_part = torch.empty(0, dtype=torch.float64, device=dev)
        self.loss_dev = torch.zeros(1, dtype=torch.float64, device=dev)
        self.init_weights(seed)

    # ------------------------------------------------------------ params --
    def init_weights(self, seed=0):
        """He-normal weights (std sqrt(2 / fan_in)), zero biases."""
        g = torch.Generator().manual_seed(seed)
        w = torch.zeros(self.master.numel(), dtype=torch.float32)
        for name, (kind, ci, co, ks) in self.layers.items():
            rows, K = self.wshape[name]
            fan_in = ci * (ks ** self.dims)
            std = math.sqrt(2.0 / fan_in) if name != "head" else math.sqrt(1.0 / fan_in)
            w[self.woff[name]:self.woff[name] + rows * K] = torch.randn(rows * K, generator=g) * std
        self.master.copy_(w.to(self.device))
        self.sync_bf16()

    def sync_bf16(self):
        C.check(self.L.lbmnn_to_bf16(_ptr(self.master), _ptr(self.wbf), self.master.numel(), self._stream()),
                "lbmnn_to_bf16")

    def weight(self, name, master=True):
        rows, K = self.wshape[name]
        src = self.master if master else self.wbf
        return src[self.woff[name]:self.woff[name] + rows * K].view(rows, K)

    def bias(self, name):
        co = self.layers[name][2]
        return self.master[self.boff[name]:self.boff[name] + co]

    def state_dict(self):
        return {"master": self.master.detach().cpu(), "dims": self.dims, "base": self.base,
                "levels": self.levels, "t": self.t}

    def load_state_dict(self, sd):
        self.master.copy_(sd["master"].to(self.device))
        self.t = int(sd.get("t", 0))
        self.sync_bf16()

    def save(self, path, meta=None):
        """Weights as BF16 bits (the values the kernels use) + FP32 biases."""
        import numpy as np
        wb = self.wbf.view(torch.int16).cpu().numpy()
        np.savez(path, wbf=wb, master=self.master.cpu().numpy() if meta and meta.get("fp32") else np.zeros(0),
                 dims=self.dims, base=self.base, levels=self.levels, cin=self.cin, cout=self.cout,
                 n_params=self.n_params, bias=self.master[min(self.boff.values()):self.n_params].cpu().numpy())

    @classmethod
    def load(cls, path, device="cuda"):
        import numpy as np
        z = np.load(path, allow_pickle=False)
        net = cls(int(z["dims"]), base=int(z["base"]), levels=int(z["levels"]), cin=int(z["cin"]),
                  cout=int(z["cout"]), device=device)
        assert int(z["n_params"]) == net.n_params
        wb = torch.from_numpy(z["wbf"]).to(device).view(BF16)
        net.wbf.copy_(wb)
        net.master.copy_(wb.to(torch.float32))
        b0 = min(net.boff.values())
        net.master[b0:net.n_params] = torch.from_numpy(z["bias"]).to(device)
        return net

    def fold_output_scale(self, scale):
        """Multiplies head output channel c by scale[c] (weights and bias), so
        a network trained on standardised targets predicts them unscaled."""
        s = torch.as_tensor(scale, dtype=torch.float32, device=self.device)
        with torch.no_grad():
            W = self.weight("head")
            W[:s.numel()] *= s[:, None]
            self.bias("head")[:s.numel()] *= s
        self.sync_bf16()

    def _stream(self):
        return ctypes.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)

    # ------------------------------------------------------------ profiling --
    _prof = None

    def _timed(self, kind, name, flops, nbytes, fn):
        """Runs fn(); with profiling on (self._prof a list), between two HIP
        events on the current stream, recording the op's algorithmic flops and
        minimal bytes (operands read once, results written once)."""
        if self._prof is None:
            return fn()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        r = fn()
        b.record()
        self._prof.append((kind, name, flops, nbytes, a, b))
        return r

    # -------------------------------------------------------------- buffers --
    def _grid(self, shape, lv):
        n, d, h, w = shape
        return (n, d >> lv if self.dims == 3 else 1, h >> lv, w >> lv)

    def buffers(self, shape):
        key = tuple(shape)
        if key in self._bufs:
            return self._bufs[key]
        n, d, h, w = shape
        div = 1 << (self.levels - 1)
        if h % div or w % div or (self.dims == 3 and d % div):
            raise ValueError(f"spatial size must be divisible by {div}")
        B = {}
        dev = self.device

        def alloc(name, lv, ch, dtype=BF16):
            g = self._grid(shape, lv)
            B[name] = torch.empty(g + (ch,), dtype=dtype, device=dev)

        for lv in range(self.levels):
            Cl = self.base << lv
            for pre in ("", "g_"):
                alloc(pre + f"e{lv}c0", lv, Cl)
                if lv < self.levels - 1:
                    alloc(pre + f"cat{lv}", lv, 2 * Cl)
                    alloc(pre + f"p{lv}", lv + 1, Cl)
                    alloc(pre + f"d{lv}c0", lv, Cl)
                    alloc(pre + f"d{lv}c1", lv, Cl)
                else:
                    alloc(pre + "bott", lv, Cl)
        alloc("head", 0, self.cout, torch.float32)
        alloc("g_head", 0, self.cout)
        self._bufs[key] = B
        return B

    # ---------------------------------------------------------- primitives --
    def _conv(self, grid, ks, cin, cout, flags, inp, in_cs, in_co, name, out=None, out_cs=0, out_co=0,
              out32=None, transposed=False, use_bias=True):
        n, d, h, w = grid
        wsrc = self.wT if transposed else self.wbf
        desc = C.lbmnn_conv_desc(n, d, h, w, self.dims, ks, cin, cout, flags, inp.data_ptr(), in_cs, in_co,
                                 out.data_ptr() if out is not None else None,
                                 out32.data_ptr() if out32 is not None else None, out_cs, out_co)
        b = _ptr(self.master, self.boff[name]) if use_bias else None
        taps = (1 << self.dims) if flags & C.NN_S2D else ks ** self.dims
        M = n * d * h * w
        m_in = M << self.dims if flags & C.NN_S2D else M
        nbytes = 2 * m_in * cin + (4 if out32 is not None else 2) * M * cout + 2 * cout * taps * cin
        # the deep levels split their K loop: FP32 partials in the shared workspace
        need = self.L.lbmnn_conv_workspace_bytes(ctypes.byref(desc))
        if self._ws.numel() * 4 < need:
            self._ws = torch.empty(need // 4 + 1024, dtype=torch.float32, device=self.device)
        self._timed("dgrad" if transposed else "fwd", name, 2 * M * cout * taps * cin, nbytes,
                    lambda: C.check(self.L.lbmnn_conv_ws(ctypes.byref(desc), _ptr(wsrc, self.woff[name]), b,
                                                         _ptr(self._ws), self._ws.numel() * 4, self._stream()),
                                    "lbmnn_conv_ws"))

    def _wgrad(self, grid, ks, cin, flags, inp, in_cs, in_co, g, g_cs, g_co, rows, name):
        n, d, h, w = grid
        M = n * d * h * w
        K = cin * (ks ** self.dims) if not (flags & C.NN_S2D) else cin * (1 << self.dims)
        # blocks per pixel split: 32 x 128 tiles for at most 32 rows, else 64 x 64
        base_blocks = -(-K // 128) if rows <= 32 else -(-rows // 64) * -(-K // 64)
        splits = max(1, min(M // 512, max(1, 2048 // base_blocks)))
        need = self.L.lbmnn_wgrad_workspace_bytes(M, rows, K, splits)
        if self._ws.numel() * 4 < need:
            self._ws = torch.empty(need // 4 + 1024, dtype=torch.float32, device=self.device)
        desc = C.lbmnn_conv_desc(n, d, h, w, self.dims, ks, cin, 0, flags, inp.data_ptr(), in_cs, in_co,
                                 None, None, 0, 0)
        m_in = M << self.dims if flags & C.NN_S2D else M
        m_g = M << self.dims if flags & C.NN_S2D_G else M
        g_ch = rows >> self.dims if flags & C.NN_S2D_G else rows
        nbytes = 2 * m_in * cin + 2 * m_g * g_ch + 4 * rows * K
        self._timed("wgrad", name, 2 * M * rows * K, nbytes,
                    lambda: C.check(self.L.lbmnn_conv_wgrad(ctypes.byref(desc), ctypes.c_void_p(g.data_ptr()), g_cs,
                                                            g_co, rows, _ptr(self.grad, self.woff[name]), 0,
                                                            _ptr(self._ws), self._ws.numel() * 4, splits,
                                                            self._stream()), "lbmnn_conv_wgrad"))

    def _bgrad(self, g, cs, co, pixels, Cn, name):
        # about 16K elements (32 KB) per split, enough blocks to keep HBM busy at every level,
        # bounded by the partials buffer
        splits = max(1, min(-(-pixels * Cn // 16384), self._bws.numel() // Cn))
        self._timed("bgrad", name, pixels * Cn, 2 * pixels * Cn + 4 * Cn,
                    lambda: C.check(self.L.lbmnn_bias_grad(ctypes.c_void_p(g.data_ptr()), cs, co, pixels, Cn,
                                                           _ptr(self.grad, self.boff[name]), 0, _ptr(self._bws),
                                                           splits, self._stream()), "lbmnn_bias_grad"))

    def _relu_bgrad(self, g, y, cs, co, pixels, Cn, name):
        # ReLU backward and the bias gradient of the masked g in one pass (splits as in _bgrad)
        splits = max(1, min(-(-pixels * Cn // 16384), self._bws.numel() // Cn))
        self._timed("relu_bgrad", name, 2 * pixels * Cn, 6 * pixels * Cn + 4 * Cn,
                    lambda: C.check(self.L.lbmnn_relu_bwd_bias_grad(ctypes.c_void_p(g.data_ptr()),
                                                                    ctypes.c_void_p(y.data_ptr()), cs, co, pixels, Cn,
                                                                    _ptr(self.grad, self.boff[name]), 0,
                                                                    _ptr(self._bws), splits, self._stream()),
                                    "lbmnn_relu_bwd_bias_grad"))

    # -------------------------------------------------------------- forward --
    def forward(self, x):
        """x: BF16 (n, d, h, w, cin) -> FP32 head output (n, d, h, w, cout)."""
        shape = tuple(x.shape[:4])
        B = self.buffers(shape)
        self._x = x
        R = C.NN_RELU
        h, h_cs, h_co, Ch = x, self.cin, 0, self.cin
        for lv in range(self.levels):
            Cl = self.base << lv
            g = self._grid(shape, lv)
            self._conv(g, 3, Ch, Cl, R, h, h_cs, h_co, f"e{lv}c0", out=B[f"e{lv}c0"], out_cs=Cl)
            if lv < self.levels - 1:
                self._conv(g, 3, Cl, Cl, R, B[f"e{lv}c0"], Cl, 0, f"e{lv}c1", out=B[f"cat{lv}"],
                           out_cs=2 * Cl, out_co=Cl)
                gc = self._grid(shape, lv + 1)
                C.check(self.L.lbmnn_pool_fwd(_ptr(B[f"cat{lv}"]), 2 * Cl, Cl, _ptr(B[f"p{lv}"]), Cl, 0, *gc, Cl,
                                              self.dims, self._stream()), "lbmnn_pool_fwd")
                h, h_cs, h_co, Ch = B[f"p{lv}"], Cl, 0, Cl
            else:
                self._conv(g, 3, Cl, Cl, R, B[f"e{lv}c0"], Cl, 0, f"e{lv}c1", out=B["bott"], out_cs=Cl)
                h, h_cs, h_co, Ch = B["bott"], Cl, 0, Cl
        for lv in range(self.levels - 2, -1, -1):
            Cl = self.base << lv
            gc, g = self._grid(shape, lv + 1), self._grid(shape, lv)
            self._conv(gc, 1, 2 * Cl, Cl << self.dims, C.NN_D2S, h, h_cs, h_co, f"d{lv}t", out=B[f"cat{lv}"],
                       out_cs=2 * Cl, out_co=0)
            self._conv(g, 3, 2 * Cl, Cl, R, B[f"cat{lv}"], 2 * Cl, 0, f"d{lv}c0", out=B[f"d{lv}c0"], out_cs=Cl)
            self._conv(g, 3, Cl, Cl, R, B[f"d{lv}c0"], Cl, 0, f"d{lv}c1", out=B[f"d{lv}c1"], out_cs=Cl)
            h, h_cs, h_co, Ch = B[f"d{lv}c1"], Cl, 0, Cl
        g0 = self._grid(shape, 0)
        self._conv(g0, 1, self.base, self.cout, 0, h, h_cs, h_co, "head", out32=B["head"], out_cs=self.cout)
        return B["head"]

    # ------------------------------------------------------------- backward --
    def _transpose_weights(self):
        for name, (kind, ci, co, ks) in self.layers.items():
            rows, K = self.wshape[name]
            if kind == "tconv":
                args = (rows, 1, ci, 0)              # [sub*co + c][ci] -> [ci][sub*co + c]
            else:
                args = (co, ks ** self.dims, ci, 1)  # flip taps, swap cin / cout
            C.check(self.L.lbmnn_weight_transpose(_ptr(self.wbf, self.woff[name]), _ptr(self.wT, self.woff[name]),
                                                  *args, self._stream()), "lbmnn_weight_transpose")

    def backward(self, g_head):
        """Gradients of <head, g_head> into self.grad (overwritten)."""
        x = self._x
        shape = tuple(x.shape[:4])
        B = self.buffers(shape)
        self._transpose_weights()
        dims = self.dims
        S = 1 << dims
        npix = lambda lv: math.prod(self._grid(shape, lv))
        g0 = self._grid(shape, 0)
        # head (1x1)
        self._wgrad(g0, 1, self.base, 0, B["d0c1"] if self.levels > 1 else B["bott"], self.base, 0,
                    g_head, self.cout, 0, self.cout, "head")
        self._bgrad(g_head, self.cout, 0, npix(0), self.cout, "head")
        self._conv(g0, 1, self.cout, self.base, 0, g_head, self.cout, 0, "head", out=B["g_d0c1"],
                   out_cs=self.base, transposed=True, use_bias=False)
        for lv in range(0, self.levels - 1):
            Cl = self.base << lv
            g = self._grid(shape, lv)
            P = npix(lv)
            # second decoder conv
            self._relu_bgrad(B[f"g_d{lv}c1"], B[f"d{lv}c1"], Cl, 0, P, Cl, f"d{lv}c1")
            self._wgrad(g, 3, Cl, 0, B[f"d{lv}c0"], Cl, 0, B[f"g_d{lv}c1"], Cl, 0, Cl, f"d{lv}c1")
            self._conv(g, 3, Cl, Cl, 0, B[f"g_d{lv}c1"], Cl, 0, f"d{lv}c1", out=B[f"g_d{lv}c0"], out_cs=Cl,
                       transposed=True, use_bias=False)
            # first decoder conv (input: concatenation)
            self._relu_bgrad(B[f"g_d{lv}c0"], B[f"d{lv}c0"], Cl, 0, P, Cl, f"d{lv}c0")
            self._wgrad(g, 3, 2 * Cl, 0, B[f"cat{lv}"], 2 * Cl, 0, B[f"g_d{lv}c0"], Cl, 0, Cl, f"d{lv}c0")
            self._conv(g, 3, Cl, 2 * Cl, 0, B[f"g_d{lv}c0"], Cl, 0, f"d{lv}c0", out=B[f"g_cat{lv}"],
                       out_cs=2 * Cl, transposed=True, use_bias=False)
            # transposed conv: input on the coarser grid
            gc = self._grid(shape, lv + 1)
            hin = B[f"d{lv + 1}c1"] if lv + 1 < self.levels - 1 else B["bott"]
            g_hin = B[f"g_d{lv + 1}c1"] if lv + 1 < self.levels - 1 else B["g_bott"]
            self._wgrad(gc, 1, 2 * Cl, C.NN_S2D_G, hin, 2 * Cl, 0, B[f"g_cat{lv}"], 2 * Cl, 0, S * Cl, f"d{lv}t")
            self._bgrad(B[f"g_cat{lv}"], 2 * Cl, 0, P, Cl, f"d{lv}t")
            self._conv(gc, 1, Cl, 2 * Cl, C.NN_S2D, B[f"g_cat{lv}"], 2 * Cl, 0, f"d{lv}t", out=g_hin,
                       out_cs=2 * Cl, transposed=True, use_bias=False)
        for lv in range(self.levels - 1, -1, -1):
            Cl = self.base << lv
            g = self._grid(shape, lv)
            P = npix(lv)
            if lv < self.levels - 1:
                # skip gradient (already in the upper half of g_cat) + pooling path
                gc = self._grid(shape, lv + 1)
                C.check(self.L.lbmnn_pool_bwd(_ptr(B[f"cat{lv}"]), 2 * Cl, Cl, _ptr(B[f"g_p{lv}"]), Cl, 0,
                                              _ptr(B[f"g_cat{lv}"]), 2 * Cl, Cl, *gc, Cl, dims, 1,
                                              self._stream()), "lbmnn_pool_bwd")
                y1, gy1, cs1, co1 = B[f"cat{lv}"], B[f"g_cat{lv}"], 2 * Cl, Cl
            else:
                y1, gy1, cs1, co1 = B["bott"], B["g_bott"], Cl, 0
            self._relu_bgrad(gy1, y1, cs1, co1, P, Cl, f"e{lv}c1")
            self._wgrad(g, 3, Cl, 0, B[f"e{lv}c0"], Cl, 0, gy1, cs1, co1, Cl, f"e{lv}c1")
            self._conv(g, 3, Cl, Cl, 0, gy1, cs1, co1, f"e{lv}c1", out=B[f"g_e{lv}c0"], out_cs=Cl,
                       transposed=True, use_bias=False)
            self._relu_bgrad(B[f"g_e{lv}c0"], B[f"e{lv}c0"], Cl, 0, P, Cl, f"e{lv}c0")
            if lv == 0:
                xin, xcs, Cin = x, self.cin, self.cin
            else:
                xin, xcs, Cin = B[f"p{lv - 1}"], Cl >> 1, Cl >> 1
            self._wgrad(g, 3, Cin, 0, xin, xcs, 0, B[f"g_e{lv}c0"], Cl, 0, Cl, f"e{lv}c0")
            if lv > 0:
                self._conv(g, 3, Cl, Cin, 0, B[f"g_e{lv}c0"], Cl, 0, f"e{lv}c0", out=B[f"g_p{lv - 1}"],
                           out_cs=Cin, transposed=True, use_bias=False)

    # ------------------------------------------------------------ training --
    def loss_and_grad(self, out, target, wpix, scale):
        """Masked MSE on the first creal channels; returns the BF16 gradient
        of the head output (loss left on the device in self.loss_dev)."""
        B = self.buffers(tuple(out.shape[:4]))
        P = out.numel() // self.cout
        nb = -(-P // 256)
        if self._mse_part.numel() < nb:
            self._mse_part = torch.empty(nb, dtype=torch.float64, device=self.device)
        C.check(self.L.lbmnn_mse(_ptr(out), self.cout, _ptr(target), _ptr(wpix), self.creal, P, float(scale),
                                 _ptr(B["g_head"]), _ptr(self._mse_part), _ptr(self.loss_dev), self._stream()),
                "lbmnn_mse")
        return B["g_head"]

    def adam_step(self, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        self.t += 1
        C.check(self.L.lbmnn_adam(_ptr(self.master), _ptr(self.grad), _ptr(self.m1), _ptr(self.m2), _ptr(self.wbf),
                                  self.n_params, lr, beta1, beta2, eps, self.t, self._stream()), "lbmnn_adam")

    # ---------------------------------------------------------- accounting --
    def conv_flops(self, shape):
        """Algorithmic flops (2 M N K per implicit GEMM) of the convolutions of
        one forward pass, of the input gradients and of the weight gradients
        of one backward pass, for input shape (n, d, h, w)."""
        fwd = dgrad = wgrad = 0
        for name, (kind, ci, co, ks) in self.layers.items():
            rows, K = self.wshape[name]
            lv = 0 if name == "head" else int(name[1])
            if kind == "tconv":
                lv += 1                     # runs on the coarser grid
            M = math.prod(self._grid(shape, lv))
            f = 2 * M * rows * K
            fwd += f
            wgrad += f
            if name != "e0c0":              # no gradient of the network input
                dgrad += f
        return fwd, dgrad, wgrad

    def train_step(self, x, target, wpix, lr, n_fluid=None):
        """One Adam step on the masked MSE; n_fluid (the batch's number of
        fluid pixels, known on the host) avoids reading it back from wpix."""
        out = self.forward(x)
        if n_fluid is None:
            n_fluid = float(wpix.sum().item())
        scale = 1.0 / max(float(n_fluid), 1.0)
        g = self.loss_and_grad(out, target, wpix, scale)
        self.backward(g)
        self.adam_step(lr)
        return self.loss_dev


def measure(dims, batch, size, steps=5, warmup=2, base=32):
    """Throughput of the network's kernels on random inputs: milliseconds per
    training step (forward, loss, backward, Adam) and per forward pass, and the
    convolution flops per second of each against the dense BF16 MFMA peak
    (2.5 PFLOP/s)."""
    net = UNet(dims, base=base)
    shape = (batch, size if dims == 3 else 1, size, size)
    g = torch.Generator(device="cuda").manual_seed(0)
    x = torch.randn(shape + (net.cin,), generator=g, device="cuda").to(BF16)
    tgt = torch.randn(shape + (net.cout,), generator=g, device="cuda")
    wpix = torch.ones(shape, device="cuda")
    for _ in range(warmup):
        net.train_step(x, tgt, wpix, 1e-4)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record()
    for _ in range(steps):
        net.train_step(x, tgt, wpix, 1e-4)
    b.record()
    torch.cuda.synchronize()
    train_ms = a.elapsed_time(b) / steps
    a.record()
    for _ in range(steps):
        net.forward(x)
    b.record()
    torch.cuda.synchronize()
    fwd_ms = a.elapsed_time(b) / steps
    fwd, dgrad, wgrad = net.conv_flops(shape)
    layers = layer_roofline(net, x, tgt, wpix)
    peak = 2500.0
    tt = (fwd + dgrad + wgrad) / (train_ms * 1e-3) / 1e12
    tf = fwd / (fwd_ms * 1e-3) / 1e12
    return {"dims": dims, "batch": batch, "size": size, "base": base, "params": net.n_params,
            "train_step_ms": round(train_ms, 3), "forward_ms": round(fwd_ms, 3),
            "train_conv_gflop": round((fwd + dgrad + wgrad) / 1e9, 2), "forward_conv_gflop": round(fwd / 1e9, 2),
            "train_tflops": round(tt, 1), "forward_tflops": round(tf, 1), "peak_tflops": peak,
            "train_frac": round(tt / peak, 4), "forward_frac": round(tf / peak, 4), "ops": layers}


MFMA_PEAK_TFLOPS, HBM_PEAK_GBS = 2500.0, 8000.0


def layer_roofline(net, x, tgt, wpix, steps=3):
    """Per operation of a training step (layer forward, input gradient,
    weight gradient, bias / ReLU backward): HIP-event time on the current
    stream, averaged over `steps` steps, against its own roofline: the larger
    of flops / dense BF16 MFMA peak and minimal bytes / HBM peak.  Returns a
    list of dicts sorted by time, longest first."""
    acc = {}
    for _ in range(steps):
        net._prof = []
        net.train_step(x, tgt, wpix, 1e-4)
        torch.cuda.synchronize()
        for kind, name, flops, nbytes, a, b in net._prof:
            e = acc.setdefault((kind, name), [flops, nbytes, 0.0])
            e[2] += a.elapsed_time(b) / steps
        net._prof = None
    out = []
    for (kind, name), (flops, nbytes, ms) in acc.items():
        t_mfma = flops / (MFMA_PEAK_TFLOPS * 1e12) * 1e3 if kind in ("fwd", "dgrad", "wgrad") else 0.0
        t_hbm = nbytes / (HBM_PEAK_GBS * 1e9) * 1e3
        bound = "mfma" if t_mfma >= t_hbm else "hbm"
        out.append({"op": kind, "layer": name, "us": round(ms * 1e3, 2), "gflop": round(flops / 1e9, 3),
                    "mb": round(nbytes / 1e6, 2), "tflops": round(flops / (ms * 1e-3) / 1e12, 1),
                    "gbs": round(nbytes / (ms * 1e-3) / 1e9, 1), "bound": bound,
                    "frac": round(max(t_mfma, t_hbm) / ms, 4)})
    out.sort(key=lambda r: -r["us"])
    return out


def layer_table(m, command):
    """Markdown table of measure()'s per-operation roofline."""
    lines = [f"# U-Net per-operation roofline ({m['dims']}D, batch {m['batch']}, {m['size']}^{m['dims']})", "",
             "Command:", "", f"    {command}", "",
             f"Training step {m['train_step_ms']} ms ({m['train_tflops']} TFLOP/s of convolutions, "
             f"{100 * m['train_frac']:.1f} % of the dense BF16 peak); forward {m['forward_ms']} ms.  Each "
             "operation's time (HIP events, mean of 3 steps) against its own bound: max(flops / 2.5 PFLOP/s, "
             "minimal bytes / 8 TB/s); frac = that bound's time / measured time.", "",
             "| op | layer | us | GFLOP | MB | TFLOP/s | GB/s | bound | frac |", "|---|---|---|---|---|---|---|---|---|"]
    for r in m["ops"]:
        lines.append(f"| {r['op']} | {r['layer']} | {r['us']} | {r['gflop']} | {r['mb']} | {r['tflops']} | "
                     f"{r['gbs']} | {r['bound']} | {r['frac']} |")
    return "\n".join(lines) + "\n"


if __name__ == "__main__":
    import json
    import sys
    dims = int(sys.argv[1]) if len(sys.argv) > 1 else 2
    m = measure(dims, 16 if dims == 2 else 2, 256 if dims == 2 else 64)
    if len(sys.argv) > 2:
        with open(sys.argv[2], "w") as fh:
            fh.write(layer_table(m, "python -m paper_2310_00810_amd.unet " + " ".join(sys.argv[1:])))
    print(json.dumps(m), flush=True)
