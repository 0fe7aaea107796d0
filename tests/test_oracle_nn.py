"""Pins of the FP64 network-layer oracle: library correlation, adjoint
(dot-product) identities, special cases and finite differences."""
import numpy as np
import pytest
from scipy import signal

import oracle
from oracle import nn as N


def rnd(shape, seed):
    return np.random.default_rng(seed).standard_normal(shape)


@pytest.mark.parametrize("dims,ks", [(2, 3), (3, 3), (2, 1), (3, 1)])
def test_conv_matches_library_correlation(dims, ks):
    shape = (2, 5, 6, 7, 3) if dims == 3 else (2, 1, 6, 7, 3)
    x = rnd(shape, 1)
    W = rnd((4, ks ** dims, 3), 2)
    b = rnd(4, 3)
    y = N.conv_fwd(x, W, b, ks, dims)
    for bb in range(2):
        for co in range(4):
            ref = np.full(shape[1:4], b[co])
            for ci in range(3):
                kern = W[co, :, ci].reshape((ks,) * dims) if dims == 3 else W[co, :, ci].reshape(ks, ks)[None]
                ref += signal.correlate(x[bb, ..., ci], kern, mode="same")
            assert np.allclose(y[bb, ..., co], ref, atol=1e-12)


@pytest.mark.parametrize("dims,ks", [(2, 3), (3, 3), (2, 1)])
def test_conv_gradients_are_adjoints(dims, ks):
    shape = (2, 4, 5, 6, 3) if dims == 3 else (2, 1, 5, 6, 3)
    x = rnd(shape, 4)
    W = rnd((5, ks ** dims, 3), 5)
    g = rnd(shape[:-1] + (5,), 6)
    y = N.conv_fwd(x, W, None, ks, dims)
    lhs = np.sum(y * g)
    assert np.isclose(lhs, np.sum(x * N.conv_dgrad(g, W, ks, dims, 3)), rtol=1e-12)
    dw, db = N.conv_wgrad(x, g, ks, dims)
    assert np.isclose(lhs, np.sum(W * dw), rtol=1e-12)
    assert np.allclose(db, g.sum((0, 1, 2, 3)), rtol=1e-12)


@pytest.mark.parametrize("dims", [2, 3])
def test_transposed_conv(dims):
    shape = (2, 3, 4, 5, 4) if dims == 3 else (2, 1, 4, 5, 4)
    x = rnd(shape, 7)
    S = 1 << dims
    # identity weights: nearest-neighbour upsampling
    I = np.broadcast_to(np.eye(4), (S, 4, 4))
    y = N.tconv_fwd(x, I, None, dims)
    up = x.repeat(2, 2).repeat(2, 3)
    if dims == 3:
        up = up.repeat(2, 1)
    assert np.array_equal(y, up)
    W = rnd((S, 6, 4), 8)
    g = rnd(y.shape[:-1] + (6,), 9)
    yw = N.tconv_fwd(x, W, None, dims)
    lhs = np.sum(yw * g)
    assert np.isclose(lhs, np.sum(x * N.tconv_dgrad(g, W, dims)), rtol=1e-12)
    dw, db = N.tconv_wgrad(x, g, dims)
    assert np.isclose(lhs, np.sum(W * dw), rtol=1e-12)
    assert np.allclose(db, g.sum((0, 1, 2, 3)))


@pytest.mark.parametrize("dims", [2, 3])
def test_pooling(dims):
    shape = (2, 4, 6, 8, 3) if dims == 3 else (2, 1, 6, 8, 3)
    x = rnd(shape, 10)
    y = N.pool_fwd(x, dims)
    n, d, h, w, C = shape
    if dims == 3:
        ref = x.reshape(n, d // 2, 2, h // 2, 2, w // 2, 2, C).max((2, 4, 6))
    else:
        ref = x.reshape(n, 1, h // 2, 2, w // 2, 2, C).max((3, 5))
    assert np.array_equal(y, ref)
    g = rnd(y.shape, 11)
    dx = N.pool_bwd(x, g, dims)
    assert np.isclose(dx.sum(), g.sum())
    # the gradient lands exactly where the input equals the window maximum
    up = y.repeat(2, 2).repeat(2, 3)
    if dims == 3:
        up = up.repeat(2, 1)
    assert np.all((dx != 0) <= (x == up))


def _params(dims, seed=0, scale=0.3):
    enc, dec, head = N.unet_layout(dims)
    rng = np.random.default_rng(seed)
    P = {}
    for lv, blk in enumerate(enc):
        for j, (_, ci, co, ks, _) in enumerate(blk):
            P[f"e{lv}c{j}"] = (rng.standard_normal((co, ks ** dims, ci)) * scale / np.sqrt(ks ** dims * ci),
                              0.05 * rng.standard_normal(co))
    for k, blk in enumerate(dec):
        lv = len(enc) - 2 - k
        _, ci, co = blk[0]
        P[f"d{lv}t"] = (rng.standard_normal((1 << dims, co, ci)) * scale / np.sqrt(ci), 0.05 * rng.standard_normal(co))
        for j, (_, ci2, co2, ks, _) in enumerate(blk[1:]):
            P[f"d{lv}c{j}"] = (rng.standard_normal((co2, 9 if dims == 2 else 27, ci2)) * scale / np.sqrt(9 * ci2),
                              0.05 * rng.standard_normal(co2))
    _, ci, co, ks, _ = head
    P["head"] = (rng.standard_normal((co, 1, ci)) / np.sqrt(ci), 0.05 * rng.standard_normal(co))
    return P


def test_unet_backward_matches_central_differences():
    dims = 2
    P = _params(dims, seed=1, scale=1.5)
    x = rnd((1, 1, 8, 8, 8), 12)
    gout = rnd((1, 1, 8, 8, 8), 13)
    out, cache = N.unet_forward(x, P, dims)
    grads = N.unet_backward(gout, P, cache, dims)
    rng = np.random.default_rng(14)
    h = 1e-6
    for name in ["e0c0", "e1c1", "e3c0", "d2t", "d1c0", "d0c1", "head"]:
        W, b = P[name]
        for _ in range(2):
            idx = tuple(rng.integers(0, s) for s in W.shape)
            Wp, Wm = W.copy(), W.copy()
            Wp[idx] += h
            Wm[idx] -= h
            Pp, Pm = dict(P), dict(P)
            Pp[name], Pm[name] = (Wp, b), (Wm, b)
            fd = (np.sum(N.unet_forward(x, Pp, dims)[0] * gout) - np.sum(N.unet_forward(x, Pm, dims)[0] * gout)) / (2 * h)
            an = grads[name][0][idx]
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (name, idx, fd, an)
        k = rng.integers(0, b.shape[0])
        bp, bm = b.copy(), b.copy()
        bp[k] += h
        bm[k] -= h
        Pp, Pm = dict(P), dict(P)
        Pp[name], Pm[name] = (W, bp), (W, bm)
        fd = (np.sum(N.unet_forward(x, Pp, dims)[0] * gout) - np.sum(N.unet_forward(x, Pm, dims)[0] * gout)) / (2 * h)
        assert abs(fd - grads[name][1][k]) <= 1e-6 * max(1.0, abs(fd)), (name, "bias")


def test_bf16_rounding_definition():
    """Round-to-nearest-even onto the BF16 grid (8 significand bits)."""
    x = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, 1.0 + 2 ** -7 + 2 ** -9, -2.5, 0.0, 3.0e38])
    r = N.bf16_round(x)
    assert list(r[:4]) == [1.0, 1.0, 1.0 + 2 ** -6, 1.0 + 2 ** -7]
    assert r[4] == -2.5 and r[5] == 0.0
    rng = np.random.default_rng(0)
    v = rng.standard_normal(10000) * 10.0 ** rng.uniform(-5, 5, 10000)
    rv = N.bf16_round(v)
    assert np.all(np.abs(rv - v) <= 2.0 ** -8 * np.abs(v) * (1 + 1e-6))
    # values on the grid are fixed points
    assert np.array_equal(N.bf16_round(rv), rv)
