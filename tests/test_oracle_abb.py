"""Pins of the oracle's anti-bounce-back density boundary (Eq. 6).

The rule read from the paper: at a fluid node x_b of an x face, the
population g_i arriving from outside the lattice is
  g_i(x_b) = -f*_opp(i)(x_b) + 2 w_i rho_w (1 + (u.c_i)^2 / (2 cs^4) - u.u / (2 cs^2)),
with rho_w the imposed density and u the velocity of x_b (Section 2.1).
"""
from itertools import product

import numpy as np
import pytest

import oracle as O
from paper_2310_00810_amd import geometry as G
from tests.conftest import abb_lattices
from tests.test_oracle import _grad_case, _mean_fields, _poiseuille_error, _run_to_residual


@pytest.mark.parametrize("q", [9, 19])
def test_abb_reproduces_the_equilibrium(q):
    """f_i^eq + f_opp(i)^eq is twice the even part of the equilibrium, so a
    face node whose outgoing populations are at equilibrium (rho_w, u)
    receives exactly the incoming equilibrium populations, for any u."""
    nz = 3 if q == 19 else 1
    lat = O.Lattice(q, 5, 4, nz, (O.BC_ABB, O.BC_PERIODIC, O.BC_PERIODIC))
    c, w, opp = O.velset(q)
    rng = np.random.default_rng(3)
    rin = 1.0 + 0.01 * rng.standard_normal((nz, 4))
    rout = 1.0 + 0.01 * rng.standard_normal((nz, 4))
    u = 0.05 * rng.standard_normal(lat.shape + (3,))
    if q == 9:
        u[..., 2] = 0
    # post-collision state: equilibrium at the face's rho_w and the node's u
    rho = np.ones(lat.shape)
    rho[:, :, 0] = rin
    rho[:, :, -1] = rout
    fs = O.init_eq(lat, rho, u)
    g = O.abb(lat, rin, rout, fs, np.zeros_like(fs))
    for x, s in ((0, 1), (lat.nx - 1, -1)):
        unk = c[:, 0] == s
        assert np.allclose(g[:, :, x][..., unk], fs[:, :, x][..., unk], atol=1e-15, rtol=0)
        # known slots are left alone
        assert np.all(g[:, :, x][..., ~unk] == 0)


def test_abb_rest_state():
    """Equal face densities keep the fluid at rest."""
    solid = G.rsa_disks(48, 24, (3.0, 5.0), 0.8, seed=11, x_margin=4, gap=1.0)[None]
    lat = O.Lattice(9, 48, 24, 1, (O.BC_ABB, O.BC_WALL, O.BC_PERIODIC), solid)
    f = O.run(lat, 0.8, 1.0, 1.0, O.init_eq(lat, 1.0, 0.0), 300)
    rho, u = O.macro(lat, f)
    assert np.abs(u).max() < 1e-14
    assert np.abs(rho[lat.fluid()] - 1.0).max() < 1e-14


@pytest.mark.parametrize("tau,tol", [(0.5 + np.sqrt(3 / 16), 1e-3), (0.8, 1e-2)])
def test_abb_poiseuille(tau, tol):
    """Channel driven by anti-bounce-back faces: the steady profile at
    mid-channel is the Poiseuille parabola of the local density gradient, the
    density varies linearly along x, and extrapolated to the faces (half a
    link outside the end nodes) it meets the imposed densities to within a
    few per cent of the density difference."""
    nx, ny, rin, rout = 64, 32, 1.002, 1.0
    lat = O.Lattice(9, nx, ny, 1, (O.BC_ABB, O.BC_WALL, O.BC_PERIODIC))
    fp, f, steps, r = _run_to_residual(lat, tau, rin, rout, O.init_eq(lat, 1.0, 0.0), 1e-9)
    assert r <= 1e-9
    rho, u = _mean_fields(lat, fp, f)
    assert _poiseuille_error(rho, u, ny, tau, nx // 2) <= tol
    xs = np.arange(nx)[8:-8]
    p = np.polyfit(xs, rho[0].mean(0)[8:-8], 1)
    assert np.abs(np.polyval(p, xs) - rho[0].mean(0)[8:-8]).max() < 1e-2 * (rin - rout)
    assert abs(np.polyval(p, -0.5) - rin) < 0.04 * (rin - rout)
    assert abs(np.polyval(p, nx - 0.5) - rout) < 0.04 * (rin - rout)


@pytest.mark.parametrize("name,lat", abb_lattices())
@pytest.mark.parametrize("kind", [O.LOSS_VEC, O.LOSS_NORM])
def test_abb_adjoint_matches_complex_step(name, lat, kind):
    """Every per-node inlet and outlet component and dL/dtau from the reverse
    pass equal the complex-step derivatives of the forward map."""
    T, tau = 40, 0.8
    rin, rout, tgt, wgt, f0 = _grad_case(lat)
    g = O.grad(lat, tau, rin, rout, f0, T, tgt, wgt, kind, 0.5, K=7)
    scale = max(np.abs(g["drho_in"]).max(), np.abs(g["drho_out"]).max())
    assert scale > 0
    for zi, yi in product(range(lat.nz), range(lat.ny)):
        e = np.zeros((lat.nz, lat.ny))
        e[zi, yi] = 1
        _, d_in = O.loss_complex_step(lat, tau, rin, rout, f0, T, tgt, wgt, kind, 0.5, drho_in=e)
        _, d_out = O.loss_complex_step(lat, tau, rin, rout, f0, T, tgt, wgt, kind, 0.5, drho_out=e)
        assert abs(d_in - g["drho_in"][zi, yi]) <= 1e-10 * scale
        assert abs(d_out - g["drho_out"][zi, yi]) <= 1e-10 * scale
    L, d_tau = O.loss_complex_step(lat, tau, rin, rout, f0, T, tgt, wgt, kind, 0.5, dtau=1.0)
    assert abs(d_tau - g["dtau"]) <= 1e-10 * abs(d_tau)
    assert abs(L - g["loss"]) <= 1e-13 * abs(L)
    sin = lat.solid[:, :, 0].astype(bool)
    assert np.all(g["drho_in"][sin] == 0)


def test_abb_adjoint_matches_central_differences():
    name, lat = abb_lattices()[0]
    T, tau, h = 40, 0.8, 1e-6
    rin, rout, tgt, wgt, f0 = _grad_case(lat, seed=4)
    g = O.grad(lat, tau, rin, rout, f0, T, tgt, wgt)

    def L(tau_, rin_, rout_):
        return O.loss(lat, O.run(lat, tau_, rin_, rout_, f0, T), tgt, wgt)

    fd_tau = (L(tau + h, rin, rout) - L(tau - h, rin, rout)) / (2 * h)
    assert abs(fd_tau - g["dtau"]) <= 1e-6 * abs(g["dtau"])
    fd_in = (L(tau, rin + h, rout) - L(tau, rin - h, rout)) / (2 * h)
    assert abs(fd_in - g["drho_in"].sum()) <= 1e-6 * abs(g["drho_in"]).sum()


@pytest.mark.parametrize("name,lat", abb_lattices())
@pytest.mark.parametrize("T", [1, 3])
def test_abb_step_adjoint_dot_product(name, lat, T):
    """<J v, w> = <v, J^T w> for the T-step map with anti-bounce-back faces;
    J^T composes the boundary, streaming and collision transposes, the
    boundary's contribution entering at the post-collision state."""
    c, wts, _ = O.velset(lat.q)
    fl = lat.fluid()[..., None]
    f0 = (wts + G.random_perturbation(lat.shape, lat.q, 0.01, seed=12)) * fl
    v = G.random_perturbation(lat.shape, lat.q, 1.0, seed=13) * fl
    wv = G.random_perturbation(lat.shape, lat.q, 1.0, seed=14) * fl
    tau, rin, rout = 0.75, 1.01, 0.995
    _, Jv = O.jvp_steps(lat, tau, rin, rout, f0, v, T)
    traj = [f0]
    for _ in range(T):
        traj.append(O.run(lat, tau, rin, rout, traj[-1], 1))
    a = wv.copy()
    for t in range(T, 0, -1):
        fs = O.collide(lat, tau, traj[t - 1])
        a, fsb, _, _ = O.abb_adj(lat, rin, rout, fs, a)
        b = O.stream_adj(lat, a) + fsb
        a, _ = O.collide_adj(lat, tau, traj[t - 1], b)
    lhs = np.sum(Jv * wv)
    rhs = np.sum(v * a)
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), 1.0)
