"""GPU parity of the HIP lattice Boltzmann path against the FP64 oracle.

Every case runs the kernels through the C ABI (liblbm.so) and compares with
the oracle on the same seeded inputs.  Bars: velocity relative L2 <= 1e-4,
gradients relative L2 <= 1e-3 (FP32 shifted populations against FP64).
"""
import numpy as np
import pytest

import oracle as O
from paper_2310_00810_amd import geometry as G
from tests.conftest import abb_lattices, mrt_velocity_lattices, multi_tile_lattices, tiny_lattices

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _lbm():
    from paper_2310_00810_amd import lbm
    return lbm


BC_NAMES = {O.BC_PRESSURE: "pressure", O.BC_PERIODIC: "periodic", O.BC_WALL: "wall", O.BC_ABB: "abb",
            O.BC_VELOCITY: "velocity"}


def oracle_pull_step(lat, tau, rin, rout, F):
    """One step in the GPU's state convention, F^t = C(B(S(F^{t-1}))), from
    the oracle's stages (B = Zou-He, or anti-bounce-back reading the
    post-collision state F^{t-1})."""
    g = O.stream(lat, F)
    g = O.abb(lat, rin, rout, F, g) if lat.bc_tuple[0] == O.BC_ABB else O.zouhe(lat, rin, rout, g)
    return g


def solver_for(lat, steps, tape=False, K=0, roi=None, target=None, loss_kind="vec",
               loss_scale="sum", inlet_mode="const", resident=1, frames=1, stride=1):
    lbm = _lbm()
    D = 2 if lat.q == 9 else 3
    tgt = None if target is None else np.asarray(target)[..., :D].astype(np.float32)
    ins = lbm.Instance(lat.nx, lat.ny, lat.nz, solid=lat.solid.copy(),
                       roi=None if roi is None else roi.astype(np.float32), target_u=tgt)
    kw = {} if lat.mrt is None else dict(collision="mrt", mrt_rates=tuple(lat.mrt))
    return lbm.Solver(lat.q, [ins], bc=tuple(BC_NAMES[b] for b in lat.bc_tuple), steps=steps,
                      ckpt_interval=K, tape=tape, loss_kind=loss_kind, loss_scale=loss_scale,
                      inlet_mode=inlet_mode, resident_segments=resident, loss_frames=frames,
                      loss_stride=stride, **kw)


def _inlet(lat, d):
    """The oracle's inlet face value for a GPU inlet parameter d: the density
    1 + d, or the velocity d itself for a velocity inlet."""
    return d if lat.bc_tuple[0] == O.BC_VELOCITY else 1 + d


def rel_l2(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def dense_shifted(lat, f):
    """oracle AoS (nz, ny, nx, q) -> GPU dense shifted (q, nz, ny, nx) float32."""
    _, w, _ = O.velset(lat.q)
    return np.ascontiguousarray(np.moveaxis(f - w, -1, 0)).astype(np.float32)


def from_dense(lat, flat, shifted=True):
    _, w, _ = O.velset(lat.q)
    a = flat.detach().cpu().numpy().astype(np.float64).reshape((lat.q,) + lat.shape)
    a = np.moveaxis(a, 0, -1)
    return a + w if shifted else a


def gpu_u(lat, solver, mean2=False):
    D = 2 if lat.q == 9 else 3
    _, u = solver.macro(mean2=mean2)
    return u.cpu().numpy().astype(np.float64).reshape(lat.shape + (D,))


def f32(x):
    return np.float64(np.float32(x))


# ---------------------------------------------------------------- forward --
@pytest.mark.parametrize("name,lat", tiny_lattices() + multi_tile_lattices() + abb_lattices() +
                         mrt_velocity_lattices())
@pytest.mark.parametrize("T", [1, 3])
def test_steps_from_random_state(name, lat, T):
    """T steps from a random non-equilibrium state, all boundary kinds."""
    _check_random_steps(lat, T)


def _long_rows(q):
    nx = (1 << 20) - 1                     # the longest row the ABI accepts
    ny, nz = (3, 1) if q == 9 else (2, 2)
    rng = np.random.default_rng(61 + q)
    solid = (rng.random((nz, ny, nx)) < 0.3).astype(np.uint8)
    solid[:, :, [0, -1]] = 0
    bc = (O.BC_PRESSURE, O.BC_WALL, O.BC_PERIODIC)
    return O.Lattice(q, nx, ny, nz, bc, solid)


@pytest.mark.parametrize("q", [9, 19])
def test_steps_on_the_longest_rows(q):
    """Rows of 2^20 - 1 nodes (x positions fill their 20-bit field): two
    steps from a random state against the oracle."""
    _check_random_steps(_long_rows(q), 2)


def test_largest_state_is_the_periodic_tiling_of_one_cell():
    """The largest D3Q19 instance state the library accepts, just below 4 GiB
    (384^3, 56.4 M fluid nodes, population offsets past 2^31 B): a fully
    periodic 12^3 tiling of a 32^3 cell holding one sphere, started from the
    tiled random equilibrium field of the cell, with the tiled target.  After
    T steps every cell's velocity equals the single cell's bit for bit, the
    loss and dL/dtau are 12^3 times the cell's, and the cell matches the
    oracle."""
    lbm = _lbm()
    cell, m, T, tau = 32, 12, 3, 0.8
    n = cell * m
    zz, yy, xx = np.mgrid[0:cell, 0:cell, 0:cell]
    sphere = (((xx - 15.5) ** 2 + (yy - 15.5) ** 2 + (zz - 15.5) ** 2) <= 3.5 ** 2).astype(np.uint8)
    fluid_big = int((sphere == 0).sum()) * m ** 3
    plane = -(-fluid_big // 64) * 64
    assert (1 << 31) < 19 * plane * 4 < (1 << 32)
    rng = np.random.default_rng(77)
    fl = (sphere == 0)
    drho = (0.01 * rng.standard_normal(sphere.shape) * fl).astype(np.float32)
    u = (0.01 * rng.standard_normal(sphere.shape + (3,)) * fl[..., None]).astype(np.float32)
    tgt = (0.01 * rng.standard_normal(sphere.shape + (3,))).astype(np.float32)
    bc = ("periodic", "periodic", "periodic")
    out = []
    for reps in (1, m):
        tile = lambda a: np.tile(a, (reps, reps, reps) + (1,) * (a.ndim - 3))
        k = cell * reps
        s = lbm.Solver(19, [lbm.Instance(k, k, k, solid=tile(sphere), target_u=tile(tgt))], bc=bc, steps=T,
                       ckpt_interval=T, tape=True)
        s.set_initial(torch.from_numpy(tile(drho).ravel()).cuda(), torch.from_numpy(tile(u).reshape(-1, 3)).cuda())
        loss = s.forward(tau, 0.0, 0.0, record_tape=True)[0]
        ug = s.macro()[1].cpu().numpy().reshape(k, k, k, 3)
        s.adjoint()
        out.append((loss, s.grad()["dtau"][0], ug))
        del s
        torch.cuda.empty_cache()
    (l1, d1, u1), (lm, dm, um) = out
    um = um.reshape(m, cell, m, cell, m, cell, 3).transpose(0, 2, 4, 1, 3, 5, 6).reshape(m ** 3, cell, cell, cell, 3)
    for c in range(m ** 3):
        assert np.array_equal(um[c], u1), c
    # per-block FP32 partial sums group the nodes differently in the two lattices
    assert lm == pytest.approx(m ** 3 * l1, rel=1e-6)
    assert dm == pytest.approx(m ** 3 * d1, rel=1e-4)
    lat = O.Lattice(19, cell, cell, cell, (O.BC_PERIODIC, O.BC_PERIODIC, O.BC_PERIODIC), sphere)
    f0 = O.init_eq(lat, 1.0 + drho.astype(np.float64), u.astype(np.float64))
    _, uo = O.macro(lat, O.run(lat, tau, 1.0, 1.0, f0, T))
    assert rel_l2(u1[fl], uo[fl]) <= 1e-5
    go = O.grad(lat, tau, 1.0, 1.0, f0, T, tgt.astype(np.float64), K=T)
    assert abs(l1 - go["loss"]) <= 1e-5 * go["loss"]
    assert abs(d1 - go["dtau"]) <= 1e-3 * abs(go["dtau"])


def test_pressure_faces_above_2_gib_are_the_tiling_of_one_cell():
    """A D3Q19 instance whose state spans more than 2 GiB (29.3 M fluid nodes,
    2.2 GB per state) with Zou-He pressure faces and a per-node inlet profile:
    a 64 x 32 x 32 cell holding one sphere, tiled 16 x 28 times in the
    periodic y and z.  The open links at the faces read past every accepted
    buffer range, so the gradient at the face nodes does not depend on where
    the state sits.  After T steps (the last segment resident, the first
    recomputed) every cell's velocity and every inlet and outlet node's
    gradient equal the single cell's bit for bit; loss and dL/dtau are the
    number of cells times the cell's; the cell matches the oracle."""
    lbm = _lbm()
    nx, cell, my, mz, T, K, tau = 64, 32, 16, 28, 4, 2, 0.8
    zz, yy, xx = np.mgrid[0:cell, 0:cell, 0:nx]
    sphere = (((xx - 31.5) ** 2 + (yy - 15.5) ** 2 + (zz - 15.5) ** 2) <= 5.5 ** 2).astype(np.uint8)
    fl = sphere == 0
    plane = -(-int(fl.sum()) * my * mz // 64) * 64
    assert (1 << 31) < 19 * plane * 4 < (1 << 32)
    rng = np.random.default_rng(78)
    drho = (0.01 * rng.standard_normal(sphere.shape) * fl).astype(np.float32)
    u = (0.01 * rng.standard_normal(sphere.shape + (3,)) * fl[..., None]).astype(np.float32)
    tgt = (0.01 * rng.standard_normal(sphere.shape + (3,))).astype(np.float32)
    prof = (0.004 * G.fourier_profile(cell, cell, n_modes=4, seed=5)).astype(np.float32)
    bc = ("pressure", "periodic", "periodic")
    out = []
    for ry, rz in ((1, 1), (my, mz)):
        tile = lambda a: np.tile(a, (rz, ry) + (1,) * (a.ndim - 2))
        s = lbm.Solver(19, [lbm.Instance(nx, cell * ry, cell * rz, solid=tile(sphere), target_u=tile(tgt))],
                       bc=bc, steps=T, ckpt_interval=K, tape=True, inlet_mode="profile")
        s.set_initial(torch.from_numpy(tile(drho).ravel()).cuda(), torch.from_numpy(tile(u).reshape(-1, 3)).cuda())
        loss = s.forward(tau, tile(prof).ravel(), 0.0, record_tape=True)[0]
        ug = s.macro()[1].cpu().numpy().reshape(cell * rz, cell * ry, nx, 3)
        s.adjoint()
        g = s.grad()
        out.append((loss, g["dtau"][0], g["drho_in"].reshape(cell * rz, cell * ry), ug))
        del s
        torch.cuda.empty_cache()
    (l1, d1, gi1, u1), (lm, dm, gim, um) = out
    for cz in range(mz):
        for cy in range(my):
            sl = (slice(cz * cell, (cz + 1) * cell), slice(cy * cell, (cy + 1) * cell))
            assert np.array_equal(um[sl], u1), (cz, cy)
            assert np.array_equal(gim[sl], gi1), (cz, cy)
    assert lm == pytest.approx(my * mz * l1, rel=1e-6)
    assert dm == pytest.approx(my * mz * d1, rel=1e-4)
    lat = O.Lattice(19, nx, cell, cell, (O.BC_PRESSURE, O.BC_PERIODIC, O.BC_PERIODIC), sphere)
    f0 = O.init_eq(lat, 1.0 + drho.astype(np.float64), u.astype(np.float64))
    rin = 1.0 + prof.astype(np.float64)
    _, uo = O.macro(lat, O.run(lat, tau, rin, 1.0, f0, T))
    assert rel_l2(u1[fl], uo[fl]) <= 1e-5
    go = O.grad(lat, tau, rin, 1.0, f0, T, tgt.astype(np.float64), K=K)
    assert abs(l1 - go["loss"]) <= 1e-5 * go["loss"]
    assert rel_l2(gi1, go["drho_in"]) <= 1e-3
    assert abs(d1 - go["dtau"]) <= 1e-3 * abs(go["dtau"])


def _check_random_steps(lat, T):
    _, w, _ = O.velset(lat.q)
    fl = lat.fluid()[..., None]
    F0 = (w + G.random_perturbation(lat.shape, lat.q, 0.01, seed=21)) * fl
    fb = dense_shifted(lat, F0)
    F0 = (np.moveaxis(fb.astype(np.float64), 0, -1) + w) * fl      # the same FP32 values
    rin = _inlet(lat, f32(0.004)) + np.zeros((lat.nz, lat.ny))
    rout = 1 + f32(-0.002) + np.zeros((lat.nz, lat.ny))
    tau = 0.7
    s = solver_for(lat, T)
    s.set_populations(torch.from_numpy(fb.ravel()).cuda())
    s.forward(tau, f32(0.004), f32(-0.002), want_loss=False)
    got = from_dense(lat, s.get_populations("state"))
    # GPU state convention: F^t = C(B(S(F^{t-1})))
    x = F0
    for _ in range(T):
        x = O.collide(lat, tau, oracle_pull_step(lat, tau, rin, rout, x))
    m = lat.fluid()
    assert rel_l2((got - w)[m], (x - w)[m]) < 1e-5
    assert np.all(np.isfinite(got))


def test_rest_state_stays_exactly_at_rest():
    solid = G.rsa_disks(96, 48, (4.0, 7.0), 0.75, seed=31)[None]
    lat = O.Lattice(9, 96, 48, 1, (O.BC_PRESSURE, O.BC_WALL, O.BC_PERIODIC), solid)
    s = solver_for(lat, 500)
    s.forward(0.8, 0.0, 0.0, want_loss=False)
    drho, u = s.macro()
    assert torch.count_nonzero(u).item() == 0 and torch.count_nonzero(drho).item() == 0


@pytest.mark.parametrize("q", [9, 19])
def test_closed_box_mass_conservation(q):
    if q == 9:
        solid = G.rsa_disks(80, 40, (3.0, 6.0), 0.8, seed=32, x_margin=0)[None]
        lat = O.Lattice(9, 80, 40, 1, (O.BC_WALL, O.BC_WALL, O.BC_PERIODIC), solid)
    else:
        solid = G.boolean_spheres((24, 20, 16), (2.0, 3.5), 0.8, seed=33, x_margin=0)
        lat = O.Lattice(19, 24, 20, 16, (O.BC_PERIODIC, O.BC_WALL, O.BC_PERIODIC), solid)
    _, w, _ = O.velset(q)
    fl = lat.fluid()[..., None]
    F0 = (w + G.random_perturbation(lat.shape, q, 0.01, seed=34)) * fl
    fb = dense_shifted(lat, F0)
    s = solver_for(lat, 1000)
    s.set_populations(torch.from_numpy(fb.ravel()).cuda())
    m0 = float(np.sum(fb.astype(np.float64)[:, lat.fluid()]))
    s.forward(0.75, 0.0, 0.0, want_loss=False)
    got = s.get_populations("state").double().sum().item()
    n_fluid = lat.fluid().sum()
    # deviation mass drift stays at FP32 rounding of the shifted populations
    assert abs(got - m0) < 1e-6 * n_fluid * 0.01 * q


def _c1(rin=1.005):
    lat = O.Lattice(9, 64, 32, 1, (O.BC_PRESSURE, O.BC_WALL, O.BC_PERIODIC))
    return lat


def test_c1_forward_parity_2000_steps():
    """2D channel 64 x 32, Zou-He rho_in = 1.005, rho_out = 1, tau = 0.8,
    2000 steps from rest: u(T) against the oracle."""
    lat = _c1()
    T = 2000
    s = solver_for(lat, T)
    s.forward(0.8, f32(0.005), 0.0, want_loss=False)
    ug = gpu_u(lat, s)
    fo = O.run(lat, 0.8, 1 + f32(0.005), 1.0, O.init_eq(lat, 1.0, 0.0), T)
    _, uo = O.macro(lat, fo)
    assert rel_l2(ug, uo[..., :2]) <= 1e-4


@pytest.mark.parametrize("kind", ["vec", "norm"])
def test_c1_gradient_parity(kind):
    """C1 loss against the target field of rho_in = 1.003; dL/drho_in,
    dL/dtau, dL/drho_out from the adjoint against the oracle's."""
    lat = _c1()
    T = 2000
    f0 = O.init_eq(lat, 1.0, 0.0)
    _, ut = O.macro(lat, O.run(lat, 0.8, 1 + f32(0.003), 1.0, f0, T))
    ut32 = ut.astype(np.float32).astype(np.float64)
    s = solver_for(lat, T, tape=True, K=45, target=ut32, loss_kind=kind)
    loss = s.forward(0.8, f32(0.005), 0.0, record_tape=True)
    s.adjoint()
    g = s.grad()
    ko = O.LOSS_VEC if kind == "vec" else O.LOSS_NORM
    go = O.grad(lat, 0.8, 1 + f32(0.005), 1.0, f0, T, ut32, kind=ko, K=45)
    assert abs(loss[0] - go["loss"]) <= 1e-4 * go["loss"]
    assert rel_l2(g["drho_in"], [go["drho_in"].sum()]) <= 1e-3
    assert rel_l2(g["drho_out"], [go["drho_out"].sum()]) <= 1e-3
    assert rel_l2(g["dtau"], [go["dtau"]]) <= 1e-3


def _driven(lats):
    """Lattices with inlet / outlet faces (the others stay at rest: zero gradients)."""
    return [(n, l) for n, l in lats if l.bc_tuple[0] in (O.BC_PRESSURE, O.BC_ABB, O.BC_VELOCITY)]


@pytest.mark.parametrize("name,lat", _driven(tiny_lattices() + multi_tile_lattices() + abb_lattices() +
                                             mrt_velocity_lattices()))
def test_tiny_profile_gradients(name, lat):
    """Per-node inlet profile gradients, dL/dtau and dL/drho_out on the tiny
    lattices (walls, periodic axes, grains touching the faces), T = 40."""
    T, tau = 40, 0.8
    rng = np.random.default_rng(0)
    din = (0.01 + 0.002 * rng.standard_normal((lat.nz, lat.ny))).astype(np.float32)
    solid_in = lat.solid[:, :, 0].astype(bool)
    tgt = (0.004 * rng.standard_normal(lat.shape + (3,))).astype(np.float32).astype(np.float64)
    if lat.q == 9:
        tgt[..., 2] = 0
    wgt = rng.uniform(0.5, 1.5, lat.shape).astype(np.float32).astype(np.float64)
    mode = "const" if solid_in.any() else "profile"
    s = solver_for(lat, T, tape=True, K=7, roi=wgt, target=tgt, inlet_mode=mode)
    dparam = din.ravel() if mode == "profile" else f32(0.01)
    s.forward(tau, dparam, f32(-0.001), record_tape=True)
    s.adjoint()
    g = s.grad()
    rin = _inlet(lat, din.astype(np.float64) if mode == "profile" else f32(0.01))
    go = O.grad(lat, tau, rin, 1 + f32(-0.001), O.init_eq(lat, 1.0, 0.0), T, tgt, wgt, K=7)
    if mode == "profile":
        assert rel_l2(g["drho_in"], go["drho_in"].ravel()) <= 1e-3
    else:
        assert rel_l2(g["drho_in"], [go["drho_in"].sum()]) <= 1e-3
    assert rel_l2(g["dtau"], [go["dtau"]]) <= 1e-3
    assert rel_l2(g["drho_out"], [go["drho_out"].sum()]) <= 1e-3


@pytest.mark.parametrize("name,lat", _driven(tiny_lattices() + multi_tile_lattices() + abb_lattices() +
                                             mrt_velocity_lattices()))
@pytest.mark.parametrize("frames,stride,resident", [(4, 5, 1), (3, 1, 2)])
def test_windowed_loss_gradients(name, lat, frames, stride, resident):
    """Time-windowed loss (frames at T - (frames - 1 - m) stride, one target
    per frame): loss, per-node inlet gradients, dL/dtau and dL/drho_out
    against the oracle.  T = 40, K = 7: frames inside and at the end of
    segments (step 35), in recomputed and in resident segments."""
    T, tau = 40, 0.8
    rng = np.random.default_rng(9)
    din = (0.01 + 0.002 * rng.standard_normal((lat.nz, lat.ny))).astype(np.float32)
    solid_in = lat.solid[:, :, 0].astype(bool)
    tgt = (0.004 * rng.standard_normal((frames,) + lat.shape + (3,))).astype(np.float32).astype(np.float64)
    if lat.q == 9:
        tgt[..., 2] = 0
    wgt = rng.uniform(0.5, 1.5, lat.shape).astype(np.float32).astype(np.float64)
    mode = "const" if solid_in.any() else "profile"
    s = solver_for(lat, T, tape=True, K=7, roi=wgt, target=tgt, inlet_mode=mode, resident=resident,
                   frames=frames, stride=stride)
    dparam = din.ravel() if mode == "profile" else f32(0.01)
    loss = s.forward(tau, dparam, f32(-0.001), record_tape=True)
    s.adjoint()
    g = s.grad()
    rin = _inlet(lat, din.astype(np.float64) if mode == "profile" else f32(0.01))
    go = O.grad(lat, tau, rin, 1 + f32(-0.001), O.init_eq(lat, 1.0, 0.0), T, tgt, wgt, K=7, frames=frames,
                stride=stride)
    assert abs(loss[0] - go["loss"]) <= 1e-4 * go["loss"]
    if mode == "profile":
        assert rel_l2(g["drho_in"], go["drho_in"].ravel()) <= 1e-3
    else:
        assert rel_l2(g["drho_in"], [go["drho_in"].sum()]) <= 1e-3
    assert rel_l2(g["dtau"], [go["dtau"]]) <= 1e-3
    assert rel_l2(g["drho_out"], [go["drho_out"].sum()]) <= 1e-3
    # a caller-given seed covers the final state only
    from paper_2310_00810_amd._lib import LBMError
    with pytest.raises(LBMError):
        s.adjoint(torch.zeros(lat.nx * lat.ny * lat.nz * (2 if lat.q == 9 else 3), device="cuda"))


@pytest.mark.parametrize("name,lat", tiny_lattices() + multi_tile_lattices() + abb_lattices() +
                         mrt_velocity_lattices())
@pytest.mark.parametrize("T", [1, 2, 3])
def test_adjoint_of_initial_state(name, lat, T):
    """dL/dF^0 from the GPU reverse sweep against the oracle's stage
    transposes composed in the GPU's state convention."""
    _, w, _ = O.velset(lat.q)
    fl = lat.fluid()[..., None]
    F0 = (w + G.random_perturbation(lat.shape, lat.q, 0.01, seed=41)) * fl
    fb = dense_shifted(lat, F0)
    F0 = (np.moveaxis(fb.astype(np.float64), 0, -1) + w) * fl
    rng = np.random.default_rng(42)
    tgt = (0.01 * rng.standard_normal(lat.shape + (3,))).astype(np.float32).astype(np.float64)
    if lat.q == 9:
        tgt[..., 2] = 0
    tau, rin, rout = 0.8, _inlet(lat, f32(0.003)), 1 + f32(-0.001)
    s = solver_for(lat, T, tape=True, K=2, target=tgt)
    s.set_populations(torch.from_numpy(fb.ravel()).cuda())
    s.forward(tau, f32(0.003), f32(-0.001), record_tape=True)
    s.adjoint()
    got = from_dense(lat, s.get_populations("adjoint"), shifted=False)
    # oracle: g^1 = B S F^0, then T-1 full steps, loss on g^T
    abb = lat.bc_tuple[0] == O.BC_ABB
    Fs = [F0]
    gs = [oracle_pull_step(lat, tau, rin, rout, F0)]
    for _ in range(T - 1):
        Fs.append(O.collide(lat, tau, gs[-1]))
        gs.append(oracle_pull_step(lat, tau, rin, rout, Fs[-1]))
    a = O.loss_seed(lat, gs[-1], tgt)
    for t in range(T, 0, -1):
        if abb:
            a, fsb, _, _ = O.abb_adj(lat, rin, rout, Fs[t - 1], a)
            a = O.stream_adj(lat, a) + fsb
        else:
            a, _, _ = O.zouhe_adj(lat, a, g=gs[t - 1], rho_in=rin)
            a = O.stream_adj(lat, a)
        if t > 1:
            a, _ = O.collide_adj(lat, tau, gs[t - 2], a)
    m = lat.fluid()
    assert rel_l2(got[m], a[m]) <= 1e-4


def test_checkpoint_interval_invariance_bitwise():
    lat = _c1()
    rng = np.random.default_rng(5)
    tgt = (0.001 * rng.standard_normal(lat.shape + (3,))).astype(np.float32)
    res = []
    for K in (1, 13, 100, 300):
        s = solver_for(lat, 300, tape=True, K=K, target=tgt)
        s.forward(0.9, 0.004, 0.0, record_tape=True)
        s.adjoint()
        res.append(s.grad())
    for r in res[1:]:
        for k in ("drho_in", "dtau", "drho_out"):
            assert np.array_equal(r[k], res[0][k])


def test_resident_segments_bitwise():
    """Keeping the taped forward's last R segments resident, so that the
    reverse sweep recomputes only the others, gives bit for bit the gradient
    of a sweep that recomputes every segment: for several R (one of them
    above the number of segments), on a second adjoint without a new forward
    (which must recompute), with graphs, direct launches and timing."""
    n = (24, 16, 12)
    solid = G.boolean_spheres(n, (2.5, 4.0), 0.6, seed=3, x_margin=3)
    lat = O.Lattice(19, n[0], n[1], n[2], (O.BC_PRESSURE, O.BC_PERIODIC, O.BC_PERIODIC), solid)
    T, K, tau = 50, 7, 0.75                      # 8 segments, the last one a single step
    din = (0.004 * G.fourier_profile(n[1], n[2], seed=33)).astype(np.float32).ravel()
    rng = np.random.default_rng(8)
    tgt = (1e-4 * rng.standard_normal(lat.shape + (3,))).astype(np.float32)

    def run(R, mode):
        s = solver_for(lat, T, tape=True, K=K, target=tgt, inlet_mode="profile", resident=R)
        assert s.resident_segments == min(R, 8)
        if mode == "direct":
            s.set_graphs(False)
        if mode == "timing":
            s.set_timing(True)
        out = []
        loss = s.forward(tau, din, 0.0, record_tape=True)
        for _ in range(2):
            s.adjoint()
            out.append((s.grad(), s.get_populations("adjoint").cpu().numpy()))
        return loss[0], out

    l0, ref = run(1, "graphs")
    for R, mode in [(1, "direct"), (2, "graphs"), (5, "direct"), (5, "timing"), (8, "graphs"), (12, "direct")]:
        l, out = run(R, mode)
        assert l == l0, (R, mode)
        for (g, a), (g0, a0) in zip(out, ref):
            for k in ("drho_in", "dtau", "drho_out"):
                assert np.array_equal(g[k], g0[k]), (R, mode, k)
            assert np.array_equal(a, a0), (R, mode)


def test_repeat_runs_are_bitwise_identical():
    lat = _c1()
    out = []
    for _ in range(2):
        s = solver_for(lat, 500, tape=True, K=50, target=np.zeros(lat.shape + (3,)))
        s.forward(0.8, 0.005, 0.0, record_tape=True)
        s.adjoint()
        out.append((s.get_populations("state").cpu().numpy(), s.grad()))
    assert np.array_equal(out[0][0], out[1][0])
    assert out[0][1]["dtau"][0] == out[1][1]["dtau"][0]


def test_d3q19_sphere_box_parity():
    """D3Q19 box of spheres, periodic y and z, per-node inlet profile:
    forward velocity and all gradients against the oracle."""
    n = (24, 16, 12)
    solid = G.boolean_spheres(n, (2.5, 4.0), 0.6, seed=3, x_margin=3)
    lat = O.Lattice(19, n[0], n[1], n[2], (O.BC_PRESSURE, O.BC_PERIODIC, O.BC_PERIODIC), solid)
    T, tau = 300, 0.75
    phi = G.fourier_profile(n[1], n[2], seed=33)
    din = (0.004 * phi).astype(np.float32)
    rng = np.random.default_rng(7)
    tgt = (1e-4 * rng.standard_normal(lat.shape + (3,))).astype(np.float32).astype(np.float64)
    s = solver_for(lat, T, tape=True, K=17, target=tgt, inlet_mode="profile", loss_scale="mean")
    loss = s.forward(tau, din.ravel(), 0.0, record_tape=True)
    ug = gpu_u(lat, s)
    s.adjoint()
    g = s.grad()
    f0 = O.init_eq(lat, 1.0, 0.0)
    rin = 1 + din.astype(np.float64)
    fo = O.run(lat, tau, rin, 1.0, f0, T)
    _, uo = O.macro(lat, fo)
    assert rel_l2(ug, uo) <= 1e-4
    nfl = lat.fluid().sum()
    go = O.grad(lat, tau, rin, 1.0, f0, T, tgt, scale=1.0 / nfl, K=17)
    assert abs(loss[0] - go["loss"]) <= 1e-4 * go["loss"]
    assert rel_l2(g["drho_in"], go["drho_in"].ravel()) <= 1e-3
    assert rel_l2(g["dtau"], [go["dtau"]]) <= 1e-3
    assert rel_l2(g["drho_out"], [go["drho_out"].sum()]) <= 1e-3


def test_batched_instances_match_single_runs():
    """Several lattices of different sizes in one problem give, bit for bit,
    what each gives alone."""
    lbm = _lbm()
    shapes = [(64, 32), (128, 64), (96, 40)]
    insts, singles = [], []
    taus, dins = [0.7, 0.9, 1.1], [0.002, 0.004, 0.006]
    for k, (nx, ny) in enumerate(shapes):
        solid = G.rsa_disks(nx, ny, (3.0, 6.0), 0.8, seed=100 + k)[None]
        tgt = np.zeros((1, ny, nx, 2), np.float32)
        insts.append(lbm.Instance(nx, ny, 1, solid=solid, target_u=tgt))
    bs = lbm.Solver(9, insts, steps=200, tape=True, ckpt_interval=20)
    lb = bs.forward(taus, dins, 0.0, record_tape=True)
    bs.adjoint()
    gb = bs.grad()
    ub = bs.split(bs.macro()[1].cpu().numpy())
    for k, ins in enumerate(insts):
        s = lbm.Solver(9, [ins], steps=200, tape=True, ckpt_interval=20)
        l1 = s.forward(taus[k], dins[k], 0.0, record_tape=True)
        s.adjoint()
        g1 = s.grad()
        assert l1[0] == lb[k]
        assert g1["dtau"][0] == gb["dtau"][k] and g1["drho_in"][0] == gb["drho_in"][k]
        assert np.array_equal(s.macro()[1].cpu().numpy(), ub[k])


def test_all_solid_instances():
    """An instance without a fluid node, alone or between two others in a
    batch: no tile is launched for it, its loss and gradients are zero, its
    velocity reads zero, and its neighbours in the batch are unaffected (bit
    for bit what they give alone)."""
    lbm = _lbm()
    shapes = [(64, 32), (40, 24), (96, 40)]
    insts = []
    for k, (nx, ny) in enumerate(shapes):
        solid = np.ones((1, ny, nx), np.uint8) if k == 1 else G.rsa_disks(nx, ny, (3.0, 6.0), 0.8, seed=200 + k)[None]
        tgt = np.full((1, ny, nx, 2), 1e-3, np.float32)
        insts.append(lbm.Instance(nx, ny, 1, solid=solid, target_u=tgt))
    taus, dins = [0.7, 0.9, 1.1], [0.002, 0.004, 0.006]
    for scale in ("sum", "mean"):
        bs = lbm.Solver(9, insts, steps=60, tape=True, ckpt_interval=7, loss_scale=scale)
        lb = bs.forward(taus, dins, 0.0, record_tape=True)
        bs.adjoint()
        gb = bs.grad()
        ub = bs.split(bs.macro()[1].cpu().numpy())
        assert lb[1] == 0.0 and gb["dtau"][1] == 0.0 and gb["drho_in"][1] == 0.0 and gb["drho_out"][1] == 0.0
        assert not np.any(ub[1])
        pa = bs.get_populations("adjoint").cpu().numpy()       # [inst][i][nz][ny][nx]
        o = 9 * insts[0].nodes
        assert not np.any(pa[o:o + 9 * insts[1].nodes])
        for k in (0, 2):
            s = lbm.Solver(9, [insts[k]], steps=60, tape=True, ckpt_interval=7, loss_scale=scale)
            l1 = s.forward(taus[k], dins[k], 0.0, record_tape=True)
            s.adjoint()
            g1 = s.grad()
            assert l1[0] == lb[k]
            assert g1["dtau"][0] == gb["dtau"][k] and g1["drho_in"][0] == gb["drho_in"][k]
            assert np.array_equal(s.macro()[1].cpu().numpy(), ub[k])
        # the solid instance alone: nothing to launch, zero loss and gradients
        s = lbm.Solver(9, [insts[1]], steps=60, tape=True, ckpt_interval=7, loss_scale=scale)
        assert s.forward(0.9, 0.004, 0.0, record_tape=True)[0] == 0.0
        s.adjoint()
        g = s.grad()
        assert g["dtau"][0] == 0.0 and g["drho_in"][0] == 0.0
        assert not torch.any(s.macro()[1]).item()


def test_error_paths():
    from paper_2310_00810_amd import _lib as C
    lat = _c1()
    s = solver_for(lat, 50, tape=True)
    with pytest.raises(C.LBMError) as e:
        s.forward(0.5, 0.001, 0.0)
    assert e.value.code == C.LBM_EINVAL
    with pytest.raises(C.LBMError) as e:
        s.adjoint()
    assert e.value.code == C.LBM_ESTATE
    s.forward(0.8, 0.001, 0.0, record_tape=False)
    with pytest.raises(C.LBMError) as e:
        s.adjoint()
    assert e.value.code == C.LBM_ESTATE
    with pytest.raises(C.LBMError) as e:
        s.grad()
    assert e.value.code == C.LBM_ESTATE
    # strongly compressible drive at tau near 1/2 blows up -> non-finite loss
    s2 = solver_for(lat, 3000, target=np.zeros(lat.shape + (3,)))
    with pytest.raises(C.LBMError) as e:
        s2.forward(0.5001, 0.9, -0.5)
    assert e.value.code == C.LBM_EUNSTABLE


# ------------------------------------------------------------ hipGraphs --
def test_graph_replays_match_direct_launches():
    """Forward and reverse sweeps replayed from captured graphs give, on
    every replay, bit for bit what direct launches give (eager work and
    synchronisations between the replays)."""
    lat = O.Lattice(9, 80, 40, 1, (O.BC_PRESSURE, O.BC_WALL, O.BC_PERIODIC),
                    G.rsa_disks(80, 40, (3.0, 6.0), 0.8, seed=51)[None])
    rng = np.random.default_rng(52)
    tgt = (1e-3 * rng.standard_normal(lat.shape + (3,))).astype(np.float32)
    sg = solver_for(lat, 240, tape=True, K=31, target=tgt)
    sd = solver_for(lat, 240, tape=True, K=31, target=tgt)
    sd.set_graphs(False)
    for rep, (tau, din) in enumerate([(0.8, 0.004), (0.9, 0.002), (0.8, 0.004), (1.1, 0.005)]):
        lg = sg.forward(tau, din, 0.0, record_tape=True)
        ld = sd.forward(tau, din, 0.0, record_tape=True)
        x = torch.randn(1000, device="cuda").sum()      # unrelated eager work
        torch.cuda.synchronize()
        sg.adjoint()
        sd.adjoint()
        gg, gd = sg.grad(), sd.grad()
        assert lg[0] == ld[0], rep
        for k in ("drho_in", "dtau", "drho_out"):
            assert np.array_equal(gg[k], gd[k]), (rep, k)
        assert torch.equal(sg.get_populations("adjoint"), sd.get_populations("adjoint"))
        del x


def test_run_to_residual_reaches_the_oracle_steady_state():
    """Two-step-mean residual criterion on the GPU; the converged mean
    velocity agrees with the oracle's steady state and with the Poiseuille
    closed form at tau = 1/2 + sqrt(3/16)."""
    nx, ny = 64, 32
    tau = 0.5 + np.sqrt(3 / 16)
    lat = O.Lattice(9, nx, ny, 1, (O.BC_PRESSURE, O.BC_WALL, O.BC_PERIODIC))
    s = solver_for(lat, 1)
    steps, r = s.run_to_residual(tau, f32(0.002), 0.0, tol=1e-6, max_steps=100_000, check_every=100)
    assert r <= 1e-6
    drho, u = s.macro(mean2=True)
    ug = u.cpu().numpy().astype(np.float64).reshape(1, ny, nx, 2)
    rg = 1 + drho.cpu().numpy().astype(np.float64).reshape(1, ny, nx)
    f = O.run(lat, tau, 1 + f32(0.002), 1.0, O.init_eq(lat, 1.0, 0.0), steps)
    f1 = O.run(lat, tau, 1 + f32(0.002), 1.0, f, 1)
    _, u0 = O.macro(lat, O.run(lat, tau, 1 + f32(0.002), 1.0, O.init_eq(lat, 1.0, 0.0), steps - 1))
    _, u1 = O.macro(lat, f)
    uo = 0.5 * (u0 + u1)
    assert rel_l2(ug, uo[..., :2]) <= 1e-4
    xm = nx // 2
    Gx = -(rg[0, :, xm + 1].mean() - rg[0, :, xm - 1].mean()) / 2 / 3
    sy = np.arange(ny) + 0.5
    ue = Gx / (2 * rg[0, :, xm].mean() * (tau - 0.5) / 3) * sy * (ny - sy)
    assert rel_l2(ug[0, :, xm, 0], ue) <= 2e-3
    del f1


def test_autograd_wrappers_match_the_builtin_gradient():
    """LBMLoss backward equals lbm_grad; LBMField with a torch VEC loss seeds
    the adjoint with dL/du and reproduces the built-in loss gradient."""
    lbm = _lbm()
    lat = _c1()
    rng = np.random.default_rng(9)
    tgt = (1e-3 * rng.standard_normal(lat.shape + (2,))).astype(np.float32)
    s = solver_for(lat, 300, tape=True, K=20, target=tgt)
    din = torch.tensor([0.004], dtype=torch.float64, requires_grad=True)
    tau = torch.tensor([0.8], dtype=torch.float64, requires_grad=True)
    dout = torch.tensor([0.0], dtype=torch.float64, requires_grad=True)
    loss = lbm.LBMLoss.apply(s, din, tau, dout)
    loss.sum().backward()
    ref = s.grad()
    assert din.grad.item() == ref["drho_in"][0] and tau.grad.item() == ref["dtau"][0]
    din2 = din.detach().clone().requires_grad_(True)
    tau2 = tau.detach().clone().requires_grad_(True)
    dout2 = dout.detach().clone().requires_grad_(True)
    u = lbm.LBMField.apply(s, din2, tau2, dout2)
    t = torch.from_numpy(tgt.reshape(-1, 2)).cuda()
    L2 = ((u - t) ** 2).sum()
    L2.backward()
    assert abs(L2.item() - loss.item()) <= 1e-5 * loss.item()
    assert abs(din2.grad.item() - ref["drho_in"][0]) <= 1e-4 * abs(ref["drho_in"][0])
    assert abs(tau2.grad.item() - ref["dtau"][0]) <= 1e-4 * abs(ref["dtau"][0])


# ------------------------------------------- obstructed pipe, anti-bounce-back --
def _e1_lattice():
    solid = G.obstructed_pipe(300, 50)
    return O.Lattice(9, 300, 50, 1, (O.BC_ABB, O.BC_WALL, O.BC_PERIODIC), solid)


def test_e1_forward_parity_40000_steps():
    """The obstructed pipe at full size (300 x 50, plate at x = 80, tau = 1,
    pressure difference 0.05 = density difference 0.15, 40000 steps): GPU
    velocity against the oracle."""
    lat = _e1_lattice()
    T, tau = 40000, 1.0
    s = solver_for(lat, T)
    s.forward(tau, 0.15, 0.0, want_loss=False)
    ug = gpu_u(lat, s)
    fo = O.run(lat, tau, 1.15, 1.0, O.init_eq(lat, 1.0, 0.0), T)
    _, uo = O.macro(lat, fo)
    m = lat.fluid()
    assert rel_l2(ug[m], uo[m][:, :2]) <= 1e-4


def test_e1_gradient_parity():
    """dL/d(rho_in) and dL/dtau of the obstructed pipe with the paper's
    outlet-region NORM loss (x >= 275), 1000 steps, against the oracle."""
    lat = _e1_lattice()
    T, tau = 1000, 1.0
    rng = np.random.default_rng(9)
    _, ut = O.macro(lat, O.run(lat, tau, 1.15, 1.0, O.init_eq(lat, 1.0, 0.0), T))
    tgt = (ut * (1 + 0.01 * rng.standard_normal(ut.shape))).astype(np.float32).astype(np.float64)
    roi = np.zeros(lat.shape)
    roi[:, :, 275:] = 1.0
    s = solver_for(lat, T, tape=True, roi=roi, target=tgt, loss_kind="norm")
    s.forward(tau, f32(0.1), 0.0, record_tape=True)
    s.adjoint()
    g = s.grad()
    go = O.grad(lat, tau, 1 + f32(0.1), 1.0, O.init_eq(lat, 1.0, 0.0), T, tgt, roi, O.LOSS_NORM)
    assert rel_l2(g["drho_in"], [go["drho_in"].sum()]) <= 1e-3
    assert rel_l2(g["dtau"], [go["dtau"]]) <= 1e-3


# ----------------------------------------- cylinder wake, MRT + velocity inlet --
def test_cylinder_wake_forward_parity():
    """D2Q9 MRT cylinder wake (800 x 320, D = 20, Zou-He velocity inlet
    u = 0.1, density outlet, periodic y, tau = 0.56, uniform start), 2000
    steps: GPU velocity against the oracle."""
    lbm = _lbm()
    nx, ny, U, T = 800, 320, 0.1, 2000
    solid = G.cylinder_channel(nx, ny, 20, 300, 160)
    s = lbm.Solver(9, [lbm.Instance(nx, ny, solid=solid)], bc=("velocity", "periodic", "periodic"), steps=T,
                   collision="mrt", mrt_rates=O.MRT_RATES)
    u0 = torch.zeros(nx * ny * 2, device="cuda")
    u0[0::2] = U
    s.set_initial(torch.zeros(nx * ny, device="cuda"), u0)
    s.forward(0.56, U, 0.0, want_loss=False)
    _, ug = s.macro()
    ug = ug.cpu().numpy().reshape(ny, nx, 2)
    lat = O.Lattice(9, nx, ny, 1, (O.BC_VELOCITY, O.BC_PERIODIC, O.BC_PERIODIC), solid, mrt=O.MRT_RATES)
    ua = np.zeros(lat.shape + (3,))
    ua[..., 0] = U
    fo = O.run(lat, 0.56, U, 1.0, O.init_eq(lat, 1.0, ua) * lat.fluid()[..., None], T)
    _, uo = O.macro(lat, fo)
    m = lat.fluid()[0]
    assert rel_l2(ug[m], uo[0][m][:, :2]) <= 1e-4


def test_cylinder_wake_windowed_gradient_parity():
    """The viscosity inversion's own configuration at full size: D2Q9 MRT,
    800 x 320 channel with a D = 20 cylinder, Zou-He velocity inlet u = 0.1,
    density outlet, periodic y, uniform start, loss summed over three frames
    (steps 20, 50, 80), K = 10 with two resident segments (the others
    recomputed beside the adjoint): loss, dL/du_in, dL/dtau and dL/drho_out
    against the oracle."""
    lbm = _lbm()
    nx, ny, U, T, K, tau = 800, 320, 0.1, 80, 10, 0.56
    frames, stride = 3, 30
    solid = G.cylinder_channel(nx, ny, 20, 300, 160)
    rng = np.random.default_rng(5)
    tg = (U + 0.01 * rng.standard_normal((frames, 1, ny, nx, 2))).astype(np.float32)
    s = lbm.Solver(9, [lbm.Instance(nx, ny, solid=solid, target_u=tg)], bc=("velocity", "periodic", "periodic"),
                   steps=T, ckpt_interval=K, tape=True, collision="mrt", mrt_rates=O.MRT_RATES,
                   resident_segments=2, loss_frames=frames, loss_stride=stride)
    u0 = torch.zeros(nx * ny * 2, device="cuda")
    u0[0::2] = U
    s.set_initial(torch.zeros(nx * ny, device="cuda"), u0)
    loss = s.forward(tau, f32(U), 0.0, record_tape=True)[0]
    s.adjoint()
    g = s.grad()
    del s
    torch.cuda.empty_cache()
    lat = O.Lattice(9, nx, ny, 1, (O.BC_VELOCITY, O.BC_PERIODIC, O.BC_PERIODIC), solid, mrt=O.MRT_RATES)
    ua = np.zeros(lat.shape + (3,))
    ua[..., 0] = U
    f0 = O.init_eq(lat, 1.0, ua) * lat.fluid()[..., None]
    t3 = np.zeros((frames,) + lat.shape + (3,))
    t3[..., :2] = tg
    go = O.grad(lat, tau, f32(U), 1.0, f0, T, t3, K=K, frames=frames, stride=stride)
    assert abs(loss - go["loss"]) <= 1e-4 * go["loss"]
    assert rel_l2(g["drho_in"], [go["drho_in"].sum()]) <= 1e-3
    assert rel_l2(g["dtau"], [go["dtau"]]) <= 1e-3
    assert rel_l2(g["drho_out"], [go["drho_out"].sum()]) <= 1e-3


@pytest.mark.parametrize("c,resident", [(1, 1), (2, 1), (2, 2)])
def test_overwritten_checkpoint_is_reported(c, resident):
    """A reverse sweep that recomputes a segment checks the step that ends it
    against the next checkpoint bit for bit: with checkpoint c overwritten in
    the caller's workspace after the taped forward, lbm_grad reports
    LBM_ECORRUPT, whether the recompute runs in sequence (one resident
    segment) or beside the adjoint on the second stream (two); the same sweep
    without the overwrite passes, and a
    following taped forward (which rewrites the checkpoints) passes again."""
    lbm = _lbm()
    from paper_2310_00810_amd._lib import LBM_ECORRUPT, LBMError
    solid = G.rsa_disks(96, 48, (4.0, 7.0), 0.75, seed=31)[None]
    rng = np.random.default_rng(5)
    tgt = (1e-3 * rng.standard_normal((1, 48, 96, 2))).astype(np.float32)
    s = lbm.Solver(9, [lbm.Instance(96, 48, solid=solid, target_u=tgt)], steps=40, ckpt_interval=10, tape=True,
                   resident_segments=resident)
    s.forward(0.8, 0.004, 0.0, record_tape=True)
    s.adjoint()
    clean = s.grad()
    s.forward(0.8, 0.004, 0.0, record_tape=True)
    ck = s.checkpoint(c)
    ck[7] = ck[7] + 1e-6
    torch.cuda.synchronize()
    s.adjoint()
    with pytest.raises(LBMError) as e:
        s.grad()
    assert e.value.code == LBM_ECORRUPT
    s.forward(0.8, 0.004, 0.0, record_tape=True)
    s.adjoint()
    again = s.grad()
    for k in clean:
        assert np.array_equal(clean[k], again[k]), k
