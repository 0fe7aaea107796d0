"""Pins of the oracle's time-windowed loss: the velocity mismatch summed over
several states of the trajectory (the periodic wake of Section 3.4 is
observed over time, not in one snapshot)."""
from itertools import product

import numpy as np
import pytest

import oracle as O
from tests.conftest import abb_lattices, mrt_velocity_lattices, tiny_lattices
from tests.test_oracle import _grad_case

T, K, TAU = 25, 6, 0.8


def _frame_times(frames, stride):
    return [T - (frames - 1 - m) * stride for m in range(frames)]


def _case(lat, frames, seed=0):
    rin, rout, tgt, wgt, f0 = _grad_case(lat, seed)
    if lat.bc_tuple[0] == O.BC_VELOCITY:
        rin = 0.02 + 0.002 * np.random.default_rng(seed + 1).standard_normal((lat.nz, lat.ny))
    rng = np.random.default_rng(seed + 2)
    tg = 0.004 * rng.standard_normal((frames,) + lat.shape + (3,))
    if lat.q == 9:
        tg[..., 2] = 0
    return rin, rout, tg, wgt, f0


def _lattices():
    pick = dict(tiny_lattices())
    out = [("d2q9_wall_grains", pick["d2q9_wall_grains"]), ("d3q19_periodic_yz", pick["d3q19_periodic_yz"])]
    out += [(n, l) for n, l in abb_lattices() if n == "abb_d2q9_wall_grains"]
    out += [(n, l) for n, l in mrt_velocity_lattices() if n == "mrt_vel_d2q9_wall_grains"]
    return out


@pytest.mark.parametrize("name,lat", _lattices())
@pytest.mark.parametrize("frames,stride", [(4, 3), (3, 6), (5, 1)])
@pytest.mark.parametrize("kind", [O.LOSS_VEC, O.LOSS_NORM])
def test_window_loss_is_the_sum_of_its_frames(name, lat, frames, stride, kind):
    """Brute force: run to each frame time separately and add the final-state
    losses against that frame's target."""
    rin, rout, tg, wgt, f0 = _case(lat, frames)
    ref = 0.0
    for m, t in enumerate(_frame_times(frames, stride)):
        ref += O.loss(lat, O.run(lat, TAU, rin, rout, f0, t), tg[m], wgt, kind, 0.5)
    L, _ = O.loss_complex_step(lat, TAU, rin, rout, f0, T, tg, wgt, kind, 0.5, frames=frames, stride=stride)
    g = O.grad(lat, TAU, rin, rout, f0, T, tg, wgt, kind, 0.5, K=K, frames=frames, stride=stride)
    assert L == pytest.approx(ref, rel=1e-13)
    assert g["loss"] == pytest.approx(ref, rel=1e-13)


@pytest.mark.parametrize("name,lat", _lattices())
@pytest.mark.parametrize("frames,stride", [(4, 3), (3, 6), (2, 7), (3, 1)])
def test_window_gradient_matches_complex_step(name, lat, frames, stride):
    """Every inlet and outlet component and dL/dtau of the windowed loss from
    the reverse pass against complex-step derivatives of the forward map
    (frames between checkpoints, and on them: with K = 6, (2, 7) has a frame
    at step 18 and (3, 1) one at step 24)."""
    rin, rout, tg, wgt, f0 = _case(lat, frames, seed=3)
    g = O.grad(lat, TAU, rin, rout, f0, T, tg, wgt, O.LOSS_VEC, 0.5, K=K, frames=frames, stride=stride)
    scale = max(np.abs(g["drho_in"]).max(), np.abs(g["drho_out"]).max())
    assert scale > 0
    kw = dict(frames=frames, stride=stride)
    for zi, yi in product(range(lat.nz), range(lat.ny)):
        e = np.zeros((lat.nz, lat.ny))
        e[zi, yi] = 1
        _, d_in = O.loss_complex_step(lat, TAU, rin, rout, f0, T, tg, wgt, O.LOSS_VEC, 0.5, drho_in=e, **kw)
        _, d_out = O.loss_complex_step(lat, TAU, rin, rout, f0, T, tg, wgt, O.LOSS_VEC, 0.5, drho_out=e, **kw)
        assert abs(d_in - g["drho_in"][zi, yi]) <= 1e-10 * scale
        assert abs(d_out - g["drho_out"][zi, yi]) <= 1e-10 * scale
    _, d_tau = O.loss_complex_step(lat, TAU, rin, rout, f0, T, tg, wgt, O.LOSS_VEC, 0.5, dtau=1.0, **kw)
    assert abs(d_tau - g["dtau"]) <= 1e-10 * abs(d_tau)


@pytest.mark.parametrize("name,lat", _lattices())
def test_window_gradient_is_the_sum_of_frame_gradients(name, lat):
    """Linearity: the windowed gradient is the sum of the final-state
    gradients of runs that end at each frame time."""
    frames, stride = 4, 5
    rin, rout, tg, wgt, f0 = _case(lat, frames, seed=5)
    g = O.grad(lat, TAU, rin, rout, f0, T, tg, wgt, O.LOSS_VEC, 1.0, K=K, frames=frames, stride=stride)
    acc = {k: 0.0 for k in ("drho_in", "drho_out", "dtau")}
    for m, t in enumerate(_frame_times(frames, stride)):
        gm = O.grad(lat, TAU, rin, rout, f0, t, tg[m], wgt, O.LOSS_VEC, 1.0, K=K)
        for k in acc:
            acc[k] = acc[k] + gm[k]
    for k in acc:
        assert np.allclose(g[k], acc[k], rtol=1e-10, atol=1e-13 * np.abs(acc[k]).max())


def test_one_frame_is_the_final_state_loss():
    name, lat = _lattices()[0]
    rin, rout, tg, wgt, f0 = _case(lat, 1)
    a = O.grad(lat, TAU, rin, rout, f0, T, tg[0], wgt, O.LOSS_VEC, 1.0, K=K)
    b = O.grad(lat, TAU, rin, rout, f0, T, tg, wgt, O.LOSS_VEC, 1.0, K=K, frames=1, stride=7)
    for k in ("loss", "drho_in", "drho_out", "dtau"):
        assert np.array_equal(a[k], b[k])
