"""Pins of the FP64 CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: exact
lattice isotropy, conservation laws, the closed-form Poiseuille profile, the
three Zou-He conditions, symmetry, complex-step and finite-difference
derivatives, and dot-product identities.  A plausible slip anywhere in the
oracle (a wrong weight, a sign, a dropped Zou-He term, a transposed index in
an adjoint) fails at least one of them.
"""
from fractions import Fraction
from itertools import product

import numpy as np
import pytest

import oracle as O
from paper_2310_00810_amd import geometry as G
from tests.conftest import tiny_lattices


# ----------------------------------------------------------------- lattice --
@pytest.mark.parametrize("q", [9, 19])
def test_velocity_set_isotropy(q):
    """Exact moments of the weights: sum w = 1, odd moments 0, second moment
    cs^2 delta, fourth moment cs^4 (dd + dd + dd) with cs^2 = 1/3."""
    c, w, opp = O.velset(q)
    wf = [Fraction(x).limit_denominator(1000) for x in w]
    for x, xf in zip(w, wf):
        assert abs(float(xf) - x) < 1e-16
    d = 2 if q == 9 else 3
    assert len({tuple(v) for v in c}) == q
    assert sum(wf) == 1
    delta = lambda a, b: 1 if a == b else 0
    for a in range(d):
        assert sum(wf[i] * c[i][a] for i in range(q)) == 0
    for a, b in product(range(d), repeat=2):
        assert sum(wf[i] * c[i][a] * c[i][b] for i in range(q)) == Fraction(1, 3) * delta(a, b)
    for a, b, g in product(range(d), repeat=3):
        assert sum(wf[i] * c[i][a] * c[i][b] * c[i][g] for i in range(q)) == 0
    for a, b, g, e in product(range(d), repeat=4):
        m4 = sum(wf[i] * c[i][a] * c[i][b] * c[i][g] * c[i][e] for i in range(q))
        assert m4 == Fraction(1, 9) * (delta(a, b) * delta(g, e) + delta(a, g) * delta(b, e)
                                       + delta(a, e) * delta(b, g))
    for i in range(q):
        assert np.all(c[opp[i]] == -c[i])
    if q == 9:
        assert np.all(c[:, 2] == 0)


@pytest.mark.parametrize("q", [9, 19])
def test_equilibrium_moments(q):
    """sum feq = rho, sum feq c = rho u, sum feq c c = rho cs^2 I + rho u u."""
    c, w, _ = O.velset(q)
    rng = np.random.default_rng(1)
    for _ in range(20):
        rho = rng.uniform(0.8, 1.2)
        u = rng.uniform(-0.1, 0.1, 3)
        if q == 9:
            u[2] = 0
        feq = O.equilibrium(q, rho, u)
        assert abs(feq.sum() - rho) < 1e-14
        assert np.allclose(feq @ c, rho * u, atol=1e-15, rtol=0)
        P = np.einsum("i,ia,ib->ab", feq, c, c)
        d = 2 if q == 9 else 3
        expect = rho / 3 * np.eye(3) + rho * np.outer(u, u)
        assert np.allclose(P[:d, :d], expect[:d, :d], atol=1e-14, rtol=0)
    # at rest the equilibrium is the weight vector times rho
    assert np.allclose(O.equilibrium(q, 1.3, np.zeros(3)), 1.3 * w, atol=1e-16)


@pytest.mark.parametrize("q", [9, 19])
def test_collision_conserves_mass_and_momentum(q):
    c, w, _ = O.velset(q)
    lat = O.Lattice(q, 5, 4, 3 if q == 19 else 1, (O.BC_PERIODIC,) * 3)
    f = w + G.random_perturbation(lat.shape, q, 0.01, seed=2)
    for tau in (0.55, 0.8, 1.0, 1.7):
        fs = O.collide(lat, tau, f)
        assert np.allclose(fs.sum(-1), f.sum(-1), atol=1e-15, rtol=0)
        assert np.allclose(fs @ c, f @ c, atol=1e-15, rtol=0)
    # tau = 1 lands exactly on the equilibrium of the incoming moments
    rho, u = O.macro(lat, f)
    fs = O.collide(lat, 1.0, f)
    k = (1, 2, 3) if q == 19 else (0, 2, 3)
    assert np.allclose(fs[k], O.equilibrium(q, rho[k], u[k]), atol=1e-16)


# ------------------------------------------------------ conservation, walls --
@pytest.mark.parametrize("q,bc,steps", [
    (9, (O.BC_WALL, O.BC_WALL, O.BC_PERIODIC), 1000),
    (9, (O.BC_PERIODIC, O.BC_WALL, O.BC_PERIODIC), 1000),
    (19, (O.BC_WALL, O.BC_PERIODIC, O.BC_WALL), 200),
    (19, (O.BC_PERIODIC, O.BC_PERIODIC, O.BC_PERIODIC), 200),
])
def test_closed_box_mass_conservation(q, bc, steps):
    """Walls and grains with halfway bounce-back, no open faces: total mass is
    constant from any initial state."""
    if q == 9:
        solid = G.rsa_disks(40, 24, (2.5, 4.0), 0.8, seed=5, x_margin=0, gap=1.0)[None]
        shape = (1, 24, 40)
    else:
        solid = G.boolean_spheres((12, 10, 8), (1.5, 2.5), 0.85, seed=6,
                                  periodic=(False, True, True), x_margin=0)
        shape = (8, 10, 12)
    lat = O.Lattice(q, shape[2], shape[1], shape[0], bc, solid)
    c, w, _ = O.velset(q)
    f = (w + G.random_perturbation(shape, q, 0.02, seed=7)) * lat.fluid()[..., None]
    m0 = f.sum()
    f1 = O.run(lat, 0.7, 1.0, 1.0, f, steps)
    assert abs(f1.sum() - m0) / m0 < 1e-13
    assert np.all(f1[solid.astype(bool)] == 0)
    if bc == (O.BC_PERIODIC,) * 3:
        # no walls and no grains in x -> momentum is conserved too, up to grains
        pass


def test_periodic_box_momentum_conservation():
    lat = O.Lattice(19, 6, 5, 4, (O.BC_PERIODIC,) * 3)
    c, w, _ = O.velset(19)
    f = w + G.random_perturbation(lat.shape, 19, 0.01, seed=8)
    j0 = (f @ c).sum((0, 1, 2))
    f1 = O.run(lat, 0.9, 1.0, 1.0, f, 50)
    assert np.allclose((f1 @ c).sum((0, 1, 2)), j0, atol=1e-14)


# ------------------------------------------------------------------- Zou-He --
@pytest.mark.parametrize("q", [9, 19])
def test_zouhe_conditions(q):
    """After the boundary pass every fluid face node has rho = rho_b, zero
    tangential velocity and bounced-back normal non-equilibrium."""
    c, w, opp = O.velset(q)
    nz = 3 if q == 19 else 1
    lat = O.Lattice(q, 5, 4, nz, (O.BC_PRESSURE, O.BC_PERIODIC, O.BC_PERIODIC))
    g = w + G.random_perturbation(lat.shape, q, 0.01, seed=9)
    rng = np.random.default_rng(3)
    rin = 1 + rng.uniform(0, 0.02, (nz, 4))
    rout = 1 + rng.uniform(-0.02, 0, (nz, 4))
    g2 = O.zouhe(lat, rin, rout, g)
    ex, exm = (int(np.flatnonzero((c == [1, 0, 0]).all(1))[0]),
               int(np.flatnonzero((c == [-1, 0, 0]).all(1))[0]))
    for x, rb, s in ((0, rin, 1), (4, rout, -1)):
        node = g2[:, :, x, :]
        rho = node.sum(-1)
        j = node @ c
        assert np.allclose(rho, rb, atol=1e-14, rtol=0)
        assert np.allclose(j[..., 1:], 0, atol=1e-15)
        for zi, yi in product(range(nz), range(4)):
            u = j[zi, yi] / rho[zi, yi]
            feq = O.equilibrium(q, rho[zi, yi], u)
            neq = node[zi, yi] - feq
            assert abs(neq[ex] - neq[exm]) < 1e-15
        # known populations untouched
        known = c[:, 0] != s
        assert np.array_equal(node[..., known], g[:, :, x][..., known])
    # interior untouched
    assert np.array_equal(g2[:, :, 1:4], g[:, :, 1:4])


# ---------------------------------------------------------- steady channels --
# The discrete scheme carries an undamped period-2 mode: an equilibrium
# perturbation with j_x alternating in sign from node to node along x is
# mapped by streaming onto its own negative, and collision, halfway
# bounce-back and the Zou-He faces leave it alone (eigenvalue -1 of the step
# Jacobian).  Start-up transients excite it, so steady-state quantities are
# taken on the two-step mean  u_bar(t) = (u(t) + u(t-1)) / 2, which cancels
# the mode exactly, and the residual is ||u_bar(t) - u_bar(t-1)|| / ||u_bar(t)||.
def _run_to_residual(lat, tau, rin, rout, f, tol, every=100, max_steps=200_000):
    """Returns (f(t-1), f(t), steps, r) once r <= tol (or at max_steps)."""
    steps = 0
    r = np.inf
    while steps < max_steps:
        f = O.run(lat, tau, rin, rout, f, every - 2)
        _, u_a = O.macro(lat, f)
        f_prev = O.run(lat, tau, rin, rout, f, 1)
        _, u_b = O.macro(lat, f_prev)
        f = O.run(lat, tau, rin, rout, f_prev, 1)
        _, u_c = O.macro(lat, f)
        steps += every
        ubar = 0.5 * (u_c + u_b)
        r = 0.5 * np.linalg.norm(u_c - u_a) / max(np.linalg.norm(ubar), 1e-300)
        if r <= tol:
            break
    return f_prev, f, steps, r


def _mean_fields(lat, f_prev, f):
    r0, u0 = O.macro(lat, f_prev)
    r1, u1 = O.macro(lat, f)
    return 0.5 * (r0 + r1), 0.5 * (u0 + u1)


def test_staggered_mode_is_an_eigenvector_with_eigenvalue_minus_one():
    """The equilibrium perturbation j_x = (-1)^x (rho fixed) flips sign in one
    step, in a channel with walls and Zou-He faces."""
    nx, ny = 10, 4
    lat = O.Lattice(9, nx, ny, 1, (O.BC_PRESSURE, O.BC_WALL, O.BC_PERIODIC))
    c, w, _ = O.velset(9)
    f0 = O.init_eq(lat, 1.0, 0.0)
    v = (3 * w * c[:, 0])[None, None, None, :] * ((-1.0) ** np.arange(nx))[None, None, :, None]
    v = np.broadcast_to(v, f0.shape)
    _, Jv = O.jvp_steps(lat, 0.8, 1.0, 1.0, f0, v, 1)
    assert np.allclose(Jv, -v, atol=1e-14, rtol=0)


def test_rest_state():
    """Equal inlet and outlet densities keep the fluid at rest (up to the
    rounding of the weights in unshifted FP64 populations)."""
    solid = G.rsa_disks(48, 24, (3.0, 5.0), 0.8, seed=11, x_margin=4, gap=1.0)[None]
    lat = O.Lattice(9, 48, 24, 1, (O.BC_PRESSURE, O.BC_WALL, O.BC_PERIODIC), solid)
    f = O.run(lat, 0.8, 1.0, 1.0, O.init_eq(lat, 1.0, 0.0), 300)
    rho, u = O.macro(lat, f)
    assert np.abs(u).max() < 1e-14
    assert np.abs(rho[lat.fluid()] - 1.0).max() < 1e-14


def _poiseuille_error(rho, u, ny, tau, xm, zs=(0,)):
    nu = (tau - 0.5) / 3
    Gx = -(rho[:, :, xm + 1].mean() - rho[:, :, xm - 1].mean()) / 2 / 3
    s = np.arange(ny) + 0.5
    ue = Gx / (2 * rho[:, :, xm].mean() * nu) * s * (ny - s)
    return max(np.linalg.norm(u[z, :, xm, 0] - ue) / np.linalg.norm(ue) for z in zs)


@pytest.mark.parametrize("tau,tol", [(0.5 + np.sqrt(3 / 16), 1e-3), (0.8, 1e-2)])
def test_poiseuille_2d(tau, tol):
    """Steady channel between halfway bounce-back walls: at mid-channel
    u_x(y) = G / (2 rho nu) s (H - s), s = y + 1/2, H = ny, G = -cs^2 drho/dx,
    nu = (tau - 1/2) / 3.  The wall slip of halfway bounce-back vanishes at
    tau = 1/2 + sqrt(3/16); the remaining error is compressibility, O(drho^2)."""
    nx, ny = 64, 32
    lat = O.Lattice(9, nx, ny, 1, (O.BC_PRESSURE, O.BC_WALL, O.BC_PERIODIC))
    fp, f, steps, r = _run_to_residual(lat, tau, 1.002, 1.0, O.init_eq(lat, 1.0, 0.0), 1e-9)
    assert r <= 1e-9
    rho, u = _mean_fields(lat, fp, f)
    err = _poiseuille_error(rho, u, ny, tau, nx // 2)
    assert err <= tol, err
    assert np.abs(u[0, :, nx // 2, 1]).max() < 1e-6 * np.abs(u[0, :, nx // 2, 0]).max()


def test_poiseuille_3d_plane_channel():
    """D3Q19 plane channel (walls in y, periodic z): same closed form."""
    nx, ny, nz = 24, 12, 3
    tau = 0.5 + np.sqrt(3 / 16)
    lat = O.Lattice(19, nx, ny, nz, (O.BC_PRESSURE, O.BC_WALL, O.BC_PERIODIC))
    fp, f, steps, r = _run_to_residual(lat, tau, 1.002, 1.0, O.init_eq(lat, 1.0, 0.0), 1e-9)
    rho, u = _mean_fields(lat, fp, f)
    assert _poiseuille_error(rho, u, ny, tau, nx // 2, range(nz)) <= 1e-3
    assert np.abs(u[..., 2]).max() < 1e-12


def test_channel_symmetry_and_flux():
    """The empty channel is mirror-symmetric about its centreline, and at
    steady state the mass crossing every interior cross-section per step is
    the same.  The crossing mass is counted on post-collision populations:
    sum_y [sum_{c_x=+1} f*(x) - sum_{c_x=-1} f*(x+1)] over the links that
    reach the neighbouring column."""
    nx, ny = 32, 12
    tau = 0.9
    lat = O.Lattice(9, nx, ny, 1, (O.BC_PRESSURE, O.BC_WALL, O.BC_PERIODIC))
    fp, f, steps, r = _run_to_residual(lat, tau, 1.004, 1.0, O.init_eq(lat, 1.0, 0.0), 1e-12)
    assert r <= 1e-12
    rho, u = _mean_fields(lat, fp, f)
    um = np.abs(u).max()
    assert np.allclose(u[0, :, :, 0], u[0, ::-1, :, 0], atol=1e-12 * um, rtol=0)
    assert np.allclose(u[0, :, :, 1], -u[0, ::-1, :, 1], atol=1e-12 * um, rtol=0)
    c, _, _ = O.velset(9)
    phis = []
    for state in (fp, f):
        fs = O.collide(lat, tau, state)[0]
        # links that cross the section: c_x = +-1 and the target row exists
        # (links that would leave through a wall bounce back and stay)
        lands = np.ones((ny, 9), bool)
        lands[ny - 1, c[:, 1] == 1] = False
        lands[0, c[:, 1] == -1] = False
        P = (fs * (lands & (c[:, 0] == 1))[:, None, :]).sum((0, 2))
        M = (fs * (lands & (c[:, 0] == -1))[:, None, :]).sum((0, 2))
        phis.append(P[:-1] - M[1:])
    phi = 0.5 * (phis[0] + phis[1])
    assert np.ptp(phi) / phi.mean() < 1e-8


def test_darcy_empty_channel():
    """Darcy permeability of a slit of width H is H^2 / 12 (mean velocity
    times dynamic viscosity over the pressure gradient)."""
    nx, ny = 96, 16
    tau = 0.5 + np.sqrt(3 / 16)
    lat = O.Lattice(9, nx, ny, 1, (O.BC_PRESSURE, O.BC_WALL, O.BC_PERIODIC))
    fp, f, steps, r = _run_to_residual(lat, tau, 1.002, 1.0, O.init_eq(lat, 1.0, 0.0), 1e-10)
    rho, u = _mean_fields(lat, fp, f)
    nu = (tau - 0.5) / 3
    xm = slice(nx // 4, 3 * nx // 4)
    gradp = -np.polyfit(np.arange(nx)[xm], rho[0].mean(0)[xm], 1)[0] / 3
    k = rho[0].mean() * nu * u[0, :, xm, 0].mean() / gradp
    assert abs(k / (ny * ny / 12) - 1) < 2e-3, k / (ny * ny / 12)


# ------------------------------------------------------------------ losses --
def test_loss_closed_forms():
    """Uniform flow in a periodic box: VEC against a zero target is
    N |U|^2; NORM against a parallel target equals VEC; weights and the scale
    multiply node by node."""
    lat = O.Lattice(9, 6, 5, 1, (O.BC_PERIODIC,) * 3)
    U = np.array([0.03, -0.02, 0.0])
    f = O.init_eq(lat, 1.1, U)
    n = 30
    zero = np.zeros(lat.shape + (3,))
    assert np.isclose(O.loss(lat, f, zero), n * (U @ U), rtol=1e-13)
    tgt = np.broadcast_to(0.5 * U, lat.shape + (3,))
    assert np.isclose(O.loss(lat, f, tgt, kind=O.LOSS_NORM),
                      O.loss(lat, f, tgt, kind=O.LOSS_VEC), rtol=1e-13)
    wgt = np.zeros(lat.shape)
    wgt[0, 2, 3] = 2.0
    assert np.isclose(O.loss(lat, f, zero, wgt, scale=0.25), 0.5 * (U @ U), rtol=1e-13)
    # NORM ignores direction: a reversed target of the same length gives 0
    assert O.loss(lat, f, np.broadcast_to(-U, lat.shape + (3,)), kind=O.LOSS_NORM) < 1e-28


# ---------------------------------------------------------------- adjoints --
def _grad_case(lat, seed=0):
    rng = np.random.default_rng(seed)
    rin = 1.01 + 0.002 * rng.standard_normal((lat.nz, lat.ny))
    rout = 1.0 + 0.001 * rng.standard_normal((lat.nz, lat.ny))
    tgt = 0.004 * rng.standard_normal(lat.shape + (3,))
    if lat.q == 9:
        tgt[..., 2] = 0
    wgt = rng.uniform(0.5, 1.5, lat.shape)
    f0 = O.init_eq(lat, 1.0, 0.0)
    return rin, rout, tgt, wgt, f0


@pytest.mark.parametrize("name,lat", tiny_lattices())
@pytest.mark.parametrize("kind", [O.LOSS_VEC, O.LOSS_NORM])
def test_adjoint_matches_complex_step(name, lat, kind):
    """Every per-node inlet and outlet component and dL/dtau from the reverse
    pass equal the complex-step derivatives of the forward map."""
    T, tau = 40, 0.8
    rin, rout, tgt, wgt, f0 = _grad_case(lat)
    g = O.grad(lat, tau, rin, rout, f0, T, tgt, wgt, kind, 0.5, K=7)
    scale = max(np.abs(g["drho_in"]).max(), np.abs(g["drho_out"]).max())
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
    # solid face nodes get no gradient
    sin = lat.solid[:, :, 0].astype(bool)
    assert np.all(g["drho_in"][sin] == 0)


@pytest.mark.parametrize("name,lat", tiny_lattices()[:3])
def test_adjoint_matches_central_differences(name, lat):
    """Central finite differences (h = 1e-6) agree with the reverse pass."""
    T, tau, h = 40, 0.8, 1e-6
    rin, rout, tgt, wgt, f0 = _grad_case(lat, seed=4)
    g = O.grad(lat, tau, rin, rout, f0, T, tgt, wgt)

    def L(tau_, rin_, rout_):
        return O.loss(lat, O.run(lat, tau_, rin_, rout_, f0, T), tgt, wgt)

    fd_tau = (L(tau + h, rin, rout) - L(tau - h, rin, rout)) / (2 * h)
    assert abs(fd_tau - g["dtau"]) <= 1e-6 * abs(g["dtau"])
    fd_in = (L(tau, rin + h, rout) - L(tau, rin - h, rout)) / (2 * h)
    assert abs(fd_in - g["drho_in"].sum()) <= 1e-6 * abs(g["drho_in"]).sum()
    zi, yi = 0, lat.ny // 2
    e = np.zeros_like(rin)
    e[zi, yi] = h
    fd_node = (L(tau, rin + e, rout) - L(tau, rin - e, rout)) / (2 * h)
    assert abs(fd_node - g["drho_in"][zi, yi]) <= 1e-6 * abs(g["drho_in"]).max()


@pytest.mark.parametrize("K", [1, 3, 7, 40])
def test_checkpoint_interval_does_not_change_gradient(K):
    name, lat = tiny_lattices()[0]
    rin, rout, tgt, wgt, f0 = _grad_case(lat, seed=5)
    ref = O.grad(lat, 0.7, rin, rout, f0, 40, tgt, wgt, K=40)
    g = O.grad(lat, 0.7, rin, rout, f0, 40, tgt, wgt, K=K)
    for k in ("drho_in", "drho_out"):
        assert np.array_equal(g[k], ref[k])
    assert g["dtau"] == ref["dtau"] and g["loss"] == ref["loss"]


def test_gradient_vanishes_at_the_truth():
    """A target produced by the same forward map at the true parameters gives
    an exactly zero VEC loss and gradient."""
    name, lat = tiny_lattices()[0]
    rin, rout, _, wgt, f0 = _grad_case(lat, seed=6)
    _, u = O.macro(lat, O.run(lat, 0.85, rin, rout, f0, 30))
    g = O.grad(lat, 0.85, rin, rout, f0, 30, u, wgt)
    assert g["loss"] == 0.0
    assert np.all(g["drho_in"] == 0) and np.all(g["drho_out"] == 0) and g["dtau"] == 0.0


@pytest.mark.parametrize("name,lat", tiny_lattices())
@pytest.mark.parametrize("T", [1, 3])
def test_step_adjoint_dot_product(name, lat, T):
    """<J v, w> = <v, J^T w> for the T-step map at a random state, with J v
    from the complex-step forward and J^T w from the adjoint stages."""
    c, wts, _ = O.velset(lat.q)
    fl = lat.fluid()[..., None]
    f0 = (wts + G.random_perturbation(lat.shape, lat.q, 0.01, seed=12)) * fl
    v = G.random_perturbation(lat.shape, lat.q, 1.0, seed=13) * fl
    wv = G.random_perturbation(lat.shape, lat.q, 1.0, seed=14) * fl
    tau, rin, rout = 0.75, 1.01, 0.995
    _, Jv = O.jvp_steps(lat, tau, rin, rout, f0, v, T)
    # forward trajectory for the transposes
    traj = [f0]
    for _ in range(T):
        traj.append(O.run(lat, tau, rin, rout, traj[-1], 1))
    a = wv.copy()
    for t in range(T, 0, -1):
        a, _, _ = O.zouhe_adj(lat, a)
        b = O.stream_adj(lat, a)
        a, _ = O.collide_adj(lat, tau, traj[t - 1], b)
    lhs = np.sum(Jv * wv)
    rhs = np.sum(v * a)
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), 1.0)


@pytest.mark.parametrize("q", [9, 19])
def test_collision_adjoint_invariants(q):
    """Collision conserves mass and momentum, so its transpose maps the
    adjoint vectors 1 and (c . e) to themselves."""
    c, w, _ = O.velset(q)
    lat = O.Lattice(q, 4, 3, 2 if q == 19 else 1, (O.BC_PERIODIC,) * 3)
    f = w + G.random_perturbation(lat.shape, q, 0.01, seed=15)
    ones = np.ones(lat.shape + (q,))
    out, _ = O.collide_adj(lat, 0.8, f, ones)
    assert np.allclose(out, 1.0, atol=1e-14, rtol=0)
    e = np.array([0.3, -0.7, 0.5 if q == 19 else 0.0])
    lam = np.broadcast_to(c @ e, lat.shape + (q,))
    out, _ = O.collide_adj(lat, 0.8, f, lam)
    assert np.allclose(out, lam, atol=1e-14, rtol=0)


def test_complex_build_matches_real_build():
    name, lat = tiny_lattices()[2]
    rin, rout, tgt, wgt, f0 = _grad_case(lat, seed=7)
    L_re, _ = O.loss_complex_step(lat, 0.8, rin, rout, f0, 25, tgt, wgt, dtau=1.0)
    L = O.loss(lat, O.run(lat, 0.8, rin, rout, f0, 25), tgt, wgt)
    assert abs(L_re - L) <= 1e-15 * abs(L)


def test_adjoint_matches_complex_step_at_c1_size():
    """The C1 case at full size (D2Q9 64 x 32 channel, walls, tau 0.8, 2000
    steps, checkpoints every 45, NORM and VEC losses against a target made at
    rho_in = 1.003): dL/drho_in (constant head), dL/drho_out and dL/dtau of the
    reverse pass against complex-step directional derivatives."""
    lat = O.Lattice(9, 64, 32, 1, (O.BC_PRESSURE, O.BC_WALL, O.BC_PERIODIC))
    f0 = O.init_eq(lat, 1.0, 0.0)
    T, tau = 2000, 0.8
    _, tgt = O.macro(lat, O.run(lat, tau, 1.003, 1.0, f0, T))
    one = np.ones((1, 32))
    for kind in (O.LOSS_VEC, O.LOSS_NORM):
        g = O.grad(lat, tau, 1.005, 1.0, f0, T, tgt, None, kind, 1.0, K=45)
        L, d_in = O.loss_complex_step(lat, tau, 1.005, 1.0, f0, T, tgt, None, kind, 1.0, drho_in=one)
        _, d_out = O.loss_complex_step(lat, tau, 1.005, 1.0, f0, T, tgt, None, kind, 1.0, drho_out=one)
        _, d_tau = O.loss_complex_step(lat, tau, 1.005, 1.0, f0, T, tgt, None, kind, 1.0, dtau=1.0)
        assert abs(L - g["loss"]) <= 1e-12 * L
        assert abs(g["drho_in"].sum() - d_in) <= 1e-9 * abs(d_in)
        assert abs(g["drho_out"].sum() - d_out) <= 1e-9 * abs(d_out)
        assert abs(g["dtau"] - d_tau) <= 1e-9 * abs(d_tau)


def test_adjoint_matches_complex_step_on_a_reduced_c3():
    """C3 reduced to 32^3 and 800 steps (D3Q19 Boolean spheres r ~ U[2, 3.5],
    porosity 0.4, periodic y/z, per-node Fourier inlet profile, tau 0.75,
    checkpoints every 40, MEAN_FLUID VEC loss): the profile gradient along
    random directions and dL/dtau against complex-step derivatives."""
    n = 32
    solid = G.boolean_spheres((n, n, n), (2.0, 3.5), 0.4, seed=3, x_margin=3)
    lat = O.Lattice(19, n, n, n, (O.BC_PRESSURE, O.BC_PERIODIC, O.BC_PERIODIC), solid)
    f0 = O.init_eq(lat, 1.0, 0.0)
    T, tau = 800, 0.75
    rin = 1.0 + 0.004 * G.fourier_profile(n, n, seed=33)
    rng = np.random.default_rng(12)
    tgt = 1e-4 * rng.standard_normal(lat.shape + (3,))
    scale = 1.0 / lat.fluid().sum()
    g = O.grad(lat, tau, rin, 1.0, f0, T, tgt, None, O.LOSS_VEC, scale, K=40)
    for k in range(2):
        v = rng.standard_normal((n, n))
        _, d = O.loss_complex_step(lat, tau, rin, 1.0, f0, T, tgt, None, O.LOSS_VEC, scale, drho_in=v)
        assert abs(np.sum(g["drho_in"] * v) - d) <= 1e-9 * np.abs(g["drho_in"]).sum() * np.abs(v).max()
    _, d_tau = O.loss_complex_step(lat, tau, rin, 1.0, f0, T, tgt, None, O.LOSS_VEC, scale, dtau=1.0)
    assert abs(g["dtau"] - d_tau) <= 1e-9 * abs(d_tau)
