"""Pins of the oracle's D2Q9 multiple-relaxation-time collision (Section 3.4)
and of the Zou-He velocity inlet used with it (the cylinder wake experiment's
free-stream inflow)."""
import os
from itertools import product

import numpy as np
import pytest

import oracle as O
from paper_2310_00810_amd import geometry as G
from tests.test_oracle import _grad_case, _mean_fields, _poiseuille_error, _run_to_residual

HERE = os.path.dirname(os.path.abspath(__file__))


def _mrt_rates(tau=None):
    return np.array(O.MRT_RATES if tau is None else [1.0 / tau] * 9)


def _d2q9_lattices(bcx, mrt):
    """Small D2Q9 lattices with grains next to the faces, walls or periodic y."""
    s1 = np.zeros((1, 6, 8), np.uint8)
    s1[0, 2, 3] = s1[0, 3, 4] = s1[0, 0, 1] = 1
    s2 = np.zeros((1, 5, 7), np.uint8)
    s2[0, 1, 2] = 1
    return [("walls", O.Lattice(9, 8, 6, 1, (bcx, O.BC_WALL, O.BC_PERIODIC), s1, mrt=mrt)),
            ("periodic_y", O.Lattice(9, 7, 5, 1, (bcx, O.BC_PERIODIC, O.BC_PERIODIC), s2, mrt=mrt))]


def test_mrt_basis_matches_the_printed_matrix():
    printed = np.loadtxt(os.path.join(HERE, "golden", "mrt_d2q9_matrix.txt"))
    M = O.mrt_matrix()
    assert np.array_equal(M, printed)
    # orthogonal rows
    G_ = M @ M.T
    assert np.allclose(G_ - np.diag(np.diag(G_)), 0)


def test_mrt_with_equal_rates_is_bgk():
    """S = I / tau reduces MRT to BGK (Section 3.4)."""
    name, lat = _d2q9_lattices(O.BC_PRESSURE, None)[0]
    tau = 0.7
    mrt = O.Lattice(9, lat.nx, lat.ny, 1, lat.bc_tuple, lat.solid, mrt=_mrt_rates(tau))
    f0 = O.init_eq(lat, 1.0, 0.0)
    a = O.run(lat, tau, 1.01, 1.0, f0, 50)
    b = O.run(mrt, tau, 1.01, 1.0, f0, 50)
    assert np.abs(a - b).max() < 1e-14


def test_mrt_conserves_mass_and_momentum_and_relaxes_stress_at_one_over_tau():
    lat = O.Lattice(9, 4, 3, 1, (O.BC_PERIODIC,) * 3, mrt=_mrt_rates())
    c, w, _ = O.velset(9)
    f = w + G.random_perturbation(lat.shape, 9, 0.01, seed=15)
    tau = 0.8
    fs = O.collide(lat, tau, f)
    assert np.allclose(fs.sum(-1), f.sum(-1), atol=1e-15, rtol=0)
    assert np.allclose(fs @ c[:, :2], f @ c[:, :2], atol=1e-15, rtol=0)
    # stress moments: m* - m_eq = (1 - 1/tau) (m - m_eq)
    M = O.mrt_matrix()
    rho, u = O.macro(lat, f)
    feq = np.stack([O.equilibrium(9, r, v) for r, v in zip(rho.ravel(), u.reshape(-1, 3))]).reshape(f.shape)
    dm, dms = (f - feq) @ M.T, (fs - feq) @ M.T
    assert np.allclose(dms[..., 7:], (1 - 1 / tau) * dm[..., 7:], atol=1e-15, rtol=0)
    rates = np.array(O.MRT_RATES)
    assert np.allclose(dms[..., [1, 2, 4, 6]], (1 - rates[[1, 2, 4, 6]]) * dm[..., [1, 2, 4, 6]], atol=1e-15, rtol=0)


@pytest.mark.parametrize("tau,tol", [(0.8, 2e-2)])
def test_mrt_poiseuille(tau, tol):
    """The shear viscosity of the MRT scheme is (tau - 1/2)/3: steady channel
    flow follows the Poiseuille parabola of the local density gradient."""
    nx, ny = 64, 32
    lat = O.Lattice(9, nx, ny, 1, (O.BC_PRESSURE, O.BC_WALL, O.BC_PERIODIC), mrt=_mrt_rates())
    fp, f, steps, r = _run_to_residual(lat, tau, 1.002, 1.0, O.init_eq(lat, 1.0, 0.0), 1e-9)
    assert r <= 1e-9
    rho, u = _mean_fields(lat, fp, f)
    assert _poiseuille_error(rho, u, ny, tau, nx // 2) <= tol


def test_velocity_inlet_imposes_the_velocity():
    """After a step every fluid inlet node has u = (u_in, 0) exactly."""
    name, lat = _d2q9_lattices(O.BC_VELOCITY, None)[0]
    uin = np.array([[0.01, 0.02, 0.015, 0.0, 0.03, 0.025]]).T.reshape(1, 6)
    f = O.run(lat, 0.8, uin, 1.0, O.init_eq(lat, 1.0, 0.0), 7)
    rho, u = O.macro(lat, f)
    fl = lat.fluid()[0, :, 0]
    assert np.allclose(u[0, fl, 0, 0], uin[0, fl], atol=1e-15, rtol=0)
    assert np.allclose(u[0, fl, 0, 1], 0.0, atol=1e-15)
    # the outlet keeps its density
    assert np.allclose(rho[0, lat.fluid()[0, :, -1], -1], 1.0, atol=1e-15)


@pytest.mark.parametrize("bcx", [O.BC_PRESSURE, O.BC_VELOCITY])
@pytest.mark.parametrize("use_mrt", [False, True])
def test_adjoint_matches_complex_step(bcx, use_mrt):
    """Reverse-pass gradients (inlet values per node: density or velocity;
    outlet density; tau) against complex-step derivatives, for MRT and the
    velocity inlet."""
    T, tau = 30, 0.8
    for name, lat in _d2q9_lattices(bcx, _mrt_rates() if use_mrt else None):
        rin, rout, tgt, wgt, f0 = _grad_case(lat)
        if bcx == O.BC_VELOCITY:
            rin = 0.02 + 0.002 * np.random.default_rng(1).standard_normal((lat.nz, lat.ny))
        g = O.grad(lat, tau, rin, rout, f0, T, tgt, wgt, O.LOSS_VEC, 0.5, K=7)
        scale = max(np.abs(g["drho_in"]).max(), np.abs(g["drho_out"]).max())
        assert scale > 0
        for zi, yi in product(range(lat.nz), range(lat.ny)):
            e = np.zeros((lat.nz, lat.ny))
            e[zi, yi] = 1
            _, d_in = O.loss_complex_step(lat, tau, rin, rout, f0, T, tgt, wgt, O.LOSS_VEC, 0.5, drho_in=e)
            _, d_out = O.loss_complex_step(lat, tau, rin, rout, f0, T, tgt, wgt, O.LOSS_VEC, 0.5, drho_out=e)
            assert abs(d_in - g["drho_in"][zi, yi]) <= 1e-10 * scale
            assert abs(d_out - g["drho_out"][zi, yi]) <= 1e-10 * scale
        L, d_tau = O.loss_complex_step(lat, tau, rin, rout, f0, T, tgt, wgt, O.LOSS_VEC, 0.5, dtau=1.0)
        assert abs(d_tau - g["dtau"]) <= 1e-10 * abs(d_tau)
        assert abs(L - g["loss"]) <= 1e-13 * abs(L)


@pytest.mark.parametrize("bcx", [O.BC_PRESSURE, O.BC_VELOCITY])
def test_mrt_step_adjoint_dot_product(bcx):
    """<J v, w> = <v, J^T w> for 3 MRT steps, J^T from the oracle's stage
    transposes (boundary, streaming, collision)."""
    for name, lat in _d2q9_lattices(bcx, _mrt_rates()):
        c, wts, _ = O.velset(9)
        fl = lat.fluid()[..., None]
        f0 = (wts + G.random_perturbation(lat.shape, 9, 0.01, seed=12)) * fl
        v = G.random_perturbation(lat.shape, 9, 1.0, seed=13) * fl
        wv = G.random_perturbation(lat.shape, 9, 1.0, seed=14) * fl
        tau, rin, rout = 0.75, (0.02 if bcx == O.BC_VELOCITY else 1.01), 0.995
        T = 3
        _, Jv = O.jvp_steps(lat, tau, rin, rout, f0, v, T)
        traj = [f0]
        for _ in range(T):
            traj.append(O.run(lat, tau, rin, rout, traj[-1], 1))
        a = wv.copy()
        for t in range(T, 0, -1):
            a, _, _ = O.zouhe_adj(lat, a, g=traj[t], rho_in=rin)
            b = O.stream_adj(lat, a)
            a, _ = O.collide_adj(lat, tau, traj[t - 1], b)
        assert abs(np.sum(Jv * wv) - np.sum(v * a)) <= 1e-12 * max(abs(np.sum(Jv * wv)), 1.0)
