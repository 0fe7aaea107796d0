"""FP64 reference of the warm-start network (TEST INFRASTRUCTURE ONLY).

Layer loops live in conv_oracle.c; this module marshals arrays and composes
the U-Net forward and backward from those layers in plain numpy (ReLU,
concatenation, the masked MSE).  Shapes are channels-last:
(n, d, h, w, C) with d = 1 in 2D.
"""
import ctypes

import numpy as np

from . import lib, _p, _f64


def bf16_round(a):
    """Round to the nearest BF16 value (ties to even), returned as float64:
    keep the upper 16 bits of the IEEE single, rounding on the lower 16."""
    f = np.ascontiguousarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def _ident(a):
    return a


def _taps(ks, dims):
    return ks ** dims


def conv_fwd(x, wt, bias, ks, dims):
    n, d, h, w, cin = x.shape
    cout = wt.shape[0]
    y = np.zeros((n, d, h, w, cout))
    lib().orc_conv_fwd(n, d, h, w, cin, cout, ks, dims, _p(_f64(x)), _p(_f64(wt)),
                       _p(_f64(bias) if bias is not None else None), _p(y))
    return y


def conv_dgrad(g, wt, ks, dims, cin):
    n, d, h, w, cout = g.shape
    dx = np.zeros((n, d, h, w, cin))
    lib().orc_conv_dgrad(n, d, h, w, cin, cout, ks, dims, _p(_f64(g)), _p(_f64(wt)), _p(dx))
    return dx


def conv_wgrad(x, g, ks, dims):
    n, d, h, w, cin = x.shape
    cout = g.shape[-1]
    dw = np.zeros((cout, _taps(ks, dims), cin))
    db = np.zeros(cout)
    lib().orc_conv_wgrad(n, d, h, w, cin, cout, ks, dims, _p(_f64(x)), _p(_f64(g)), _p(dw), _p(db))
    return dw, db


def tconv_fwd(x, wt, bias, dims):
    """wt: (2^dims, cout, cin)."""
    n, d, h, w, cin = x.shape
    cout = wt.shape[1]
    fd = 2 * d if dims == 3 else 1
    y = np.zeros((n, fd, 2 * h, 2 * w, cout))
    lib().orc_tconv_fwd(n, d, h, w, cin, cout, dims, _p(_f64(x)), _p(_f64(wt)),
                        _p(_f64(bias) if bias is not None else None), _p(y))
    return y


def tconv_dgrad(g, wt, dims):
    n, fd, fh, fw, cout = g.shape
    d = fd // 2 if dims == 3 else 1
    cin = wt.shape[2]
    dx = np.zeros((n, d, fh // 2, fw // 2, cin))
    lib().orc_tconv_dgrad(n, d, fh // 2, fw // 2, cin, cout, dims, _p(_f64(g)), _p(_f64(wt)), _p(dx))
    return dx


def tconv_wgrad(x, g, dims):
    n, d, h, w, cin = x.shape
    cout = g.shape[-1]
    dw = np.zeros((1 << dims, cout, cin))
    db = np.zeros(cout)
    lib().orc_tconv_wgrad(n, d, h, w, cin, cout, dims, _p(_f64(x)), _p(_f64(g)), _p(dw), _p(db))
    return dw, db


def pool_fwd(x, dims):
    n, fd, fh, fw, C = x.shape
    d = fd // 2 if dims == 3 else 1
    y = np.zeros((n, d, fh // 2, fw // 2, C))
    lib().orc_pool_fwd(n, d, fh // 2, fw // 2, C, dims, _p(_f64(x)), _p(y))
    return y


def pool_bwd(x, g, dims):
    n, fd, fh, fw, C = x.shape
    d = fd // 2 if dims == 3 else 1
    dx = np.zeros_like(x, dtype=np.float64)
    lib().orc_pool_bwd(n, d, fh // 2, fw // 2, C, dims, _p(_f64(x)), _p(_f64(g)), _p(dx))
    return dx


# ------------------------------------------------------------------ U-Net --
def unet_layout(dims, cin=8, base=32, levels=4, cout=8):
    """Layer list of the U-Net: ('conv', cin, cout, ks, relu) per encoder /
    decoder convolution, ('tconv', cin, cout) per up-sampling step."""
    enc, dec = [], []
    c = cin
    for lv in range(levels):
        co = base << lv
        enc.append([("conv", c, co, 3, True), ("conv", co, co, 3, True)])
        c = co
    for lv in range(levels - 2, -1, -1):
        co = base << lv
        dec.append([("tconv", c, co), ("conv", 2 * co, co, 3, True), ("conv", co, co, 3, True)])
        c = co
    head = ("conv", c, cout, 1, False)
    return enc, dec, head


def unet_forward(x, params, dims, quantize=None, base=32, levels=4):
    """params: dict name -> (W, b) in the GPU layouts (conv W (cout, taps, cin),
    tconv W (2^dims, cout, cin)).  Returns the head output and the cache.
    quantize (e.g. bf16_round) is applied to every stored activation, as a
    mixed-precision implementation stores them; None keeps FP64."""
    q = quantize or _ident
    enc, dec, head = unet_layout(dims, base=base, levels=levels)
    cache = {"x": x}
    h = x
    skips = []
    for lv, blk in enumerate(enc):
        for j, (_, ci, co, ks, relu) in enumerate(blk):
            W, b = params[f"e{lv}c{j}"]
            z = conv_fwd(h, W, b, ks, dims)
            h = q(np.maximum(z, 0) if relu else z)
            cache[f"e{lv}c{j}"] = h
        if lv < len(enc) - 1:
            skips.append(h)
            h = pool_fwd(h, dims)
            cache[f"p{lv}"] = h
    for k, blk in enumerate(dec):
        lv = len(enc) - 2 - k
        W, b = params[f"d{lv}t"]
        up = q(tconv_fwd(h, W, b, dims))
        h = np.concatenate([up, skips[lv]], axis=-1)
        cache[f"d{lv}cat"] = h
        for j in range(2):
            W, b = params[f"d{lv}c{j}"]
            h = q(np.maximum(conv_fwd(h, W, b, 3, dims), 0))
            cache[f"d{lv}c{j}"] = h
    W, b = params["head"]
    out = conv_fwd(h, W, b, 1, dims)
    return out, cache


def unet_backward(gout, params, cache, dims, quantize=None, base=32, levels=4):
    """Gradients of <out, gout> with respect to every (W, b); quantize is
    applied to every stored activation gradient (see unet_forward)."""
    q = quantize or _ident
    enc, dec, head = unet_layout(dims, base=base, levels=levels)
    grads = {}
    nl = len(enc)
    last = cache[f"d0c1"] if dec else cache[f"e{nl - 1}c1"]
    W, b = params["head"]
    grads["head"] = conv_wgrad(last, gout, 1, dims)
    g = q(conv_dgrad(gout, W, 1, dims, W.shape[2]))
    skip_g = {}
    # decoder levels in backward order: 0 (last in the forward), 1, ..., nl-2
    for lv in range(0, nl - 1):
        for j in (1, 0):
            y = cache[f"d{lv}c{j}"]
            g = g * (y > 0)
            xin = cache[f"d{lv}cat"] if j == 0 else cache[f"d{lv}c0"]
            W, b = params[f"d{lv}c{j}"]
            grads[f"d{lv}c{j}"] = conv_wgrad(xin, g, 3, dims)
            g = q(conv_dgrad(g, W, 3, dims, W.shape[2]))
        co = g.shape[-1] // 2
        g_up, skip_g[lv] = g[..., :co], g[..., co:]
        W, b = params[f"d{lv}t"]
        xin = cache[f"d{lv + 1}c1"] if lv + 1 < nl - 1 else cache[f"e{nl - 1}c1"]
        grads[f"d{lv}t"] = tconv_wgrad(xin, g_up, dims)
        g = q(tconv_dgrad(g_up, W, dims))
    for lv in range(nl - 1, -1, -1):
        if lv < nl - 1:
            g = q(pool_bwd(cache[f"e{lv}c1"], g, dims) + skip_g[lv])
        for j in (1, 0):
            y = cache[f"e{lv}c{j}"]
            g = g * (y > 0)
            if j == 0:
                xin = cache["x"] if lv == 0 else cache[f"p{lv - 1}"]
            else:
                xin = cache[f"e{lv}c0"]
            W, b = params[f"e{lv}c{j}"]
            grads[f"e{lv}c{j}"] = conv_wgrad(xin, g, 3, dims)
            g = q(conv_dgrad(g, W, 3, dims, W.shape[2]))
    return grads


# ------------------------------------------------------------ training ops --
# The warm-start network's loss, optimiser and target scaling (the network is
# the paper's future-work initial guess, Section 3.5; the scaling is the
# Stokes reading of its targets).

def masked_mse(pred, target, wpix, creal, scale):
    """Loss L = scale * sum_p wpix[p] * sum_{c < creal} (pred[p, c] - target[p, c])^2
    over pixels p (rows of pred, whose further columns are padding), and
    dL/dpred (zero in the padding columns)."""
    pred = np.asarray(pred, np.float64)
    d = pred[:, :creal] - np.asarray(target, np.float64)[:, :creal]
    w = np.asarray(wpix, np.float64)[:, None]
    g = np.zeros_like(pred)
    g[:, :creal] = 2.0 * scale * w * d
    return scale * float(np.sum(w * d * d)), g


def adam(w, g, m1, m2, lr, b1, b2, eps, t):
    """One Adam step (Kingma and Ba, Algorithm 1): the moment estimates, their
    bias corrections at step t (from 1) and the update; returns (w, m1, m2)."""
    g = np.asarray(g, np.float64)
    m1 = b1 * np.asarray(m1, np.float64) + (1.0 - b1) * g
    m2 = b2 * np.asarray(m2, np.float64) + (1.0 - b2) * g * g
    mh = m1 / (1.0 - b1 ** t)
    vh = m2 / (1.0 - b2 ** t)
    return np.asarray(w, np.float64) - lr * mh / (np.sqrt(vh) + eps), m1, m2


def stokes_targets(drho, u, solid, drho_in, drho_out, tau):
    """Network targets of one sample: t0 = (drho - drho_out) / (drho_in - drho_out)
    and t_a = u_a nu / (c_s^2 (drho_in - drho_out)) with nu = (tau - 1/2) / 3 and
    c_s^2 = 1/3 at fluid nodes, 0 at solid nodes; rows are nodes."""
    dr = drho_in - drho_out
    nu = (tau - 0.5) / 3.0
    fl = (np.asarray(solid).reshape(-1) == 0)[:, None]
    u = np.asarray(u, np.float64).reshape(fl.shape[0], -1)
    t = np.concatenate([(np.asarray(drho, np.float64).reshape(-1, 1) - drho_out) / dr, u * nu / (dr / 3.0)], axis=1)
    return np.where(fl, t, 0.0)


def stokes_fields(pred, solid, drho_in, drho_out, tau, dims):
    """Inverse of stokes_targets on the first 1 + dims columns of pred:
    (drho, u) at fluid nodes, 0 at solid nodes."""
    dr = drho_in - drho_out
    nu = (tau - 0.5) / 3.0
    fl = np.asarray(solid).reshape(-1) == 0
    p = np.asarray(pred, np.float64)
    drho = np.where(fl, drho_out + dr * p[:, 0], 0.0)
    u = np.where(fl[:, None], p[:, 1:1 + dims] * (dr / 3.0) / nu, 0.0)
    return drho, u


def flux_balance(u, solid, lo=0.25, hi=4.0, floor=0.1):
    """Cross-section flux balance of a predicted velocity field (one sample;
    an addition to the network initial guess of Section 3.5, from mass
    conservation: a steady flow carries the same flux through every
    cross-section normal to the flow direction x).

    solid: (d, h, w); u: (d, h, w, D), or (nodes, D) in that order.  With
    Q(x) the sum of u_x over the fluid nodes of section x (all y, z) and
    Qbar the mean of Q over the w sections, every velocity component of every
    node of section x is multiplied by
        s(x) = min(max(Qbar / max(Q(x), floor * Qbar), lo), hi);
    if Qbar <= 0 the field is returned unchanged."""
    solid = np.asarray(solid)
    d, h, w = solid.shape
    u = np.asarray(u, np.float64)
    shape = u.shape
    u = u.reshape(d, h, w, -1).copy()
    fluid = solid == 0
    Q = np.zeros(w)
    for x in range(w):
        Q[x] = np.sum(u[:, :, x, 0][fluid[:, :, x]])
    qbar = np.sum(Q) / w
    if not qbar > 0.0:
        return u.reshape(shape)
    for x in range(w):
        s = qbar / max(Q[x], floor * qbar)
        s = min(max(s, lo), hi)
        u[:, :, x, :] *= s
    return u.reshape(shape)
