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


def test_masked_mse_gradient_and_special_cases():
    """Masked MSE: dL/dpred against central differences of L; a zero-weight
    pixel and the padding columns contribute nothing; one pixel, one column:
    L = scale (p - t)^2."""
    rng = np.random.default_rng(31)
    P, pcs, creal = 7, 5, 3
    pred = rng.standard_normal((P, pcs))
    tgt = rng.standard_normal((P, creal))
    w = rng.uniform(size=P)
    w[2] = 0.0
    L, g = N.masked_mse(pred, tgt, w, creal, 0.7)
    h = 1e-6
    for p in range(P):
        for c in range(pcs):
            e = np.zeros_like(pred)
            e[p, c] = h
            fd = (N.masked_mse(pred + e, tgt, w, creal, 0.7)[0] - N.masked_mse(pred - e, tgt, w, creal, 0.7)[0]) / (2 * h)
            assert abs(fd - g[p, c]) <= 1e-8 * max(1.0, abs(fd))
    assert np.all(g[2] == 0.0) and np.all(g[:, creal:] == 0.0)
    pred2 = pred.copy()
    pred2[2] += 5.0
    pred2[:, creal:] -= 3.0
    assert N.masked_mse(pred2, tgt, w, creal, 0.7)[0] == L
    assert np.isclose(N.masked_mse(np.array([[2.0]]), np.array([[0.5]]), np.array([1.0]), 1, 0.25)[0], 0.25 * 1.5 ** 2)


def test_adam_bias_corrections():
    """Adam from zero moments: with a constant gradient g the bias-corrected
    moments are exactly g and g^2 at every step, so each step moves a weight
    by lr g / (|g| + eps); with b1 = b2 = 0 the same holds for any gradient
    sequence; a zero gradient leaves the moments decaying and the step equal
    to the corrected ratio."""
    rng = np.random.default_rng(32)
    n = 9
    w0 = rng.standard_normal(n)
    g = rng.standard_normal(n)
    lr, eps = 1e-2, 1e-8
    w, m1, m2 = w0, np.zeros(n), np.zeros(n)
    for t in range(1, 6):
        w, m1, m2 = N.adam(w, g, m1, m2, lr, 0.9, 0.999, eps, t)
        assert np.allclose(w, w0 - t * lr * g / (np.abs(g) + eps), rtol=0, atol=1e-13)
    w, m1, m2 = w0, np.zeros(n), np.zeros(n)
    for t in range(1, 4):
        gt = rng.standard_normal(n)
        w_prev = w
        w, m1, m2 = N.adam(w, gt, m1, m2, lr, 0.0, 0.0, eps, t)
        assert np.allclose(w, w_prev - lr * gt / (np.abs(gt) + eps), rtol=0, atol=1e-15)
    w1, m1, m2 = N.adam(w0, g, np.zeros(n), np.zeros(n), lr, 0.9, 0.999, eps, 1)
    w2, m1b, m2b = N.adam(w1, np.zeros(n), m1, m2, lr, 0.9, 0.999, eps, 2)
    assert np.allclose(m1b, 0.9 * m1) and np.allclose(m2b, 0.999 * m2)
    mh, vh = m1b / (1 - 0.9 ** 2), m2b / (1 - 0.999 ** 2)
    assert np.allclose(w2, w1 - lr * mh / (np.sqrt(vh) + eps))


def test_stokes_scaling_round_trip_and_closed_form():
    """The target scaling and its inverse are inverse at fluid nodes and 0 at
    solid nodes; the density target is 1 at the inlet density and 0 at the
    outlet's; the velocity target is u nu / (c_s^2 drho) (nu = 0.1 at tau = 0.8)."""
    rng = np.random.default_rng(33)
    P, D = 50, 3
    solid = (rng.uniform(size=P) > 0.7).astype(np.uint8)
    drho = rng.uniform(0, 0.004, P)
    drho[0], drho[1] = 0.004, 0.001
    solid[:2] = 0
    u = rng.standard_normal((P, D)) * 1e-3
    t = N.stokes_targets(drho, u, solid, 0.004, 0.001, 0.8)
    assert t[0, 0] == 1.0 and t[1, 0] == 0.0
    fl = solid == 0
    assert np.allclose(t[fl, 1:], u[fl] * 0.1 / (0.003 / 3.0))
    assert np.all(t[~fl] == 0.0)
    r2, u2 = N.stokes_fields(np.concatenate([t, np.zeros((P, 2))], axis=1), solid, 0.004, 0.001, 0.8, D)
    assert np.allclose(r2[fl], drho[fl], rtol=1e-13) and np.allclose(u2[fl], u[fl], rtol=1e-12)
    assert np.all(r2[~fl] == 0.0) and np.all(u2[~fl] == 0.0)


# ---- cross-section flux balance of the warm start's predicted velocity ----

def _field(rng, d, h, w, D, porosity=0.6):
    solid = (rng.random((d, h, w)) > porosity).astype(np.uint8)
    u = rng.random((d, h, w, D)) + 0.1
    u[..., 1:] -= 0.6
    u[solid == 1] = 0.0
    return solid, u


def _fluxes(u, solid):
    return np.array([u[:, :, x, 0][solid[:, :, x] == 0].sum() for x in range(solid.shape[2])])


@pytest.mark.parametrize("d,D", [(1, 2), (3, 3)])
def test_flux_balance_makes_every_section_carry_the_mean_flux(d, D):
    rng = np.random.default_rng(4)
    solid, u = _field(rng, d, 9, 12, D)
    q0 = _fluxes(u, solid)
    out = N.flux_balance(u, solid)
    q1 = _fluxes(out, solid)
    # no factor is clamped for these fields: every section now carries the old mean flux
    assert q0.min() > 0.1 * q0.mean() and (q0.mean() / q0).max() < 4 and (q0.mean() / q0).min() > 0.25
    assert np.allclose(q1, q0.mean(), rtol=1e-13, atol=0)
    # one factor per section, the same for every component and node of the section
    for x in range(12):
        fl = solid[:, :, x] == 0
        r = out[:, :, x][fl] / u[:, :, x][fl]
        assert np.allclose(r, q0.mean() / q0[x], rtol=1e-13)
    assert np.all(out[solid == 1] == 0)


def test_flux_balance_keeps_a_balanced_field_and_ignores_solid_nodes():
    solid = np.zeros((1, 3, 4), np.uint8)
    solid[0, 1, 2] = 1
    u = np.zeros((1, 3, 4, 2))
    u[0, :, :, 0] = [[1.0, 2.0, 3.0, 1.0], [2.0, 2.0, 99.0, 2.0], [3.0, 2.0, 3.0, 3.0]]   # each section: 6
    u[0, :, :, 1] = 0.5
    out = N.flux_balance(u, solid)
    assert np.array_equal(out, u)                      # factors exactly 1: the solid node's 99 is not counted


def test_flux_balance_clamps_and_leaves_reverse_flow_alone():
    solid = np.zeros((1, 1, 3), np.uint8)
    u = np.zeros((1, 1, 3, 2))
    u[0, 0, :, 0] = [1.0, 1.9, 0.01]                   # Qbar = 0.97; sections scale by 0.97, 0.97/1.9, 4 (clamped)
    u[0, 0, :, 1] = 1.0
    out = N.flux_balance(u, solid)
    qb = 2.91 / 3
    assert np.allclose(out[0, 0, :, 0], [qb, 1.9 * qb / 1.9, 0.04], rtol=1e-14)
    assert np.allclose(out[0, 0, :, 1], [qb, qb / 1.9, 4.0], rtol=1e-14)
    u[0, 0, 2, 0] = 1.0                                  # Q = 1, 1.9, 1 -> factor 1.3 / 1.9 above the floor
    out = N.flux_balance(u, solid, lo=0.8)
    assert np.allclose(out[0, 0, :, 0], [1.3, 1.9 * 0.8, 1.3], rtol=1e-14)   # the middle factor clamped to lo
    u[0, 0, :, 0] = [-1.0, 0.5, 0.2]                     # no net forward flow: unchanged
    assert np.array_equal(N.flux_balance(u, solid), u)
