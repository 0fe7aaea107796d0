"""The 2D workloads at their full sizes against the FP64 oracle.

* The granular channel: D2Q9 512 x 256, RSA disks r ~ U[6, 14] to porosity
  0.70, tau 0.9, rho_in 1.004, walls in y.  The velocity after its full
  10 000 steps against the oracle's run; the gradient over 200 steps (K = 20,
  the recompute beside the adjoint) against the oracle's reverse sweep; and at
  the full T = 10 000, K = 500 the adjoint's dL/drho_in and dL/dtau against
  central differences of the GPU's own loss.
* The batch of 64 uneven D2Q9 media (11 M nodes) in one launch per step:
  every instance's velocity, loss and gradients over a few steps from a
  random equilibrium field, against the oracle run on that instance alone.
"""
import numpy as np
import pytest

import oracle as O
from paper_2310_00810_amd import geometry as G

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

NX, NY, TAU = 512, 256, 0.9
WALLS = (O.BC_PRESSURE, O.BC_WALL, O.BC_PERIODIC)


def f32(x):
    return np.float64(np.float32(x))


def rel(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.fixture(scope="module")
def channel():
    solid = G.rsa_disks(NX, NY, (6.0, 14.0), 0.70, seed=2)[None]
    return solid, O.Lattice(9, NX, NY, 1, WALLS, solid)


def test_granular_channel_velocity_after_10000_steps(channel):
    from paper_2310_00810_amd import lbm
    solid, lat = channel
    T, d = 10000, f32(0.004)
    s = lbm.Solver(9, [lbm.Instance(NX, NY, solid=solid)], steps=T)
    s.forward(TAU, d, 0.0, want_loss=False)
    ug = s.macro()[1].cpu().numpy().astype(np.float64).reshape(1, NY, NX, 2)
    fo = O.run(lat, TAU, 1.0 + d, 1.0, O.init_eq(lat, 1.0, 0.0), T)
    _, uo = O.macro(lat, fo)
    fl = lat.fluid()
    assert rel(ug[fl], uo[..., :2][fl]) <= 1e-4


def test_granular_channel_gradient_against_the_oracle(channel):
    from paper_2310_00810_amd import lbm
    solid, lat = channel
    T, K, d = 200, 20, f32(0.004)
    rng = np.random.default_rng(9)
    tgt = (1e-3 * rng.standard_normal((1, NY, NX, 2))).astype(np.float32)
    s = lbm.Solver(9, [lbm.Instance(NX, NY, solid=solid, target_u=tgt)], steps=T, ckpt_interval=K, tape=True,
                   resident_segments=2)
    loss = s.forward(TAU, d, 0.0, record_tape=True)[0]
    s.adjoint()
    g = s.grad()
    t3 = np.zeros((1, NY, NX, 3))
    t3[..., :2] = tgt
    go = O.grad(lat, TAU, 1.0 + d, 1.0, O.init_eq(lat, 1.0, 0.0), T, t3, K=K)
    assert abs(loss - go["loss"]) <= 1e-4 * go["loss"]
    assert rel(g["drho_in"], [go["drho_in"].sum()]) <= 1e-3
    assert rel(g["dtau"], [go["dtau"]]) <= 1e-3
    assert rel(g["drho_out"], [go["drho_out"].sum()]) <= 1e-3


def test_granular_channel_adjoint_at_10000_steps_matches_central_differences(channel):
    """The inverse problem's own setting: target from rho_in 1.004, evaluated
    half-way at 1.002, T = 10 000, K = 500."""
    from paper_2310_00810_amd import lbm
    solid, _ = channel
    T, K = 10000, 500
    s0 = lbm.Solver(9, [lbm.Instance(NX, NY, solid=solid)], steps=T)
    s0.forward(TAU, 0.004, 0.0, want_loss=False)
    tgt = s0.macro()[1].cpu().numpy().reshape(1, NY, NX, 2)
    s = lbm.Solver(9, [lbm.Instance(NX, NY, solid=solid, target_u=tgt)], steps=T, ckpt_interval=K, tape=True)
    d = 0.002
    s.forward(TAU, d, 0.0, record_tape=True)
    s.adjoint()
    g = s.grad()
    loss = lambda tau, din: s.forward(tau, din, 0.0, want_loss=True)[0]
    h = 2e-4
    fd_in = (loss(TAU, d + h) - loss(TAU, d - h)) / (2 * h)
    assert abs(g["drho_in"][0] - fd_in) <= 1e-3 * abs(fd_in)
    h = 1e-3
    fd_tau = (loss(TAU + h, d) - loss(TAU - h, d)) / (2 * h)
    assert abs(g["dtau"][0] - fd_tau) <= 1e-3 * abs(fd_tau)


def test_batch_of_64_media_against_the_oracle():
    from paper_2310_00810_amd import lbm, run
    insts, taus, dins = run.c4_instances(64)
    dins = [f32(x) for x in dins]
    T, K = 4, 2
    rng = np.random.default_rng(23)
    drho, u = [], []
    for ins in insts:
        fl = (ins.solid[0] == 0)
        drho.append((0.01 * rng.standard_normal((ins.ny, ins.nx)) * fl).astype(np.float32))
        u.append((0.01 * rng.standard_normal((ins.ny, ins.nx, 2)) * fl[..., None]).astype(np.float32))
    bs = lbm.Solver(9, insts, steps=T, ckpt_interval=K, tape=True)
    bs.set_initial(torch.from_numpy(np.concatenate([a.ravel() for a in drho])).cuda(),
                   torch.from_numpy(np.concatenate([a.reshape(-1, 2) for a in u])).cuda())
    lb = bs.forward(taus, dins, 0.0, record_tape=True)
    ub = bs.split(bs.macro()[1].cpu().numpy())
    bs.adjoint()
    gb = bs.grad()
    del bs
    torch.cuda.empty_cache()
    for k, ins in enumerate(insts):
        lat = O.Lattice(9, ins.nx, ins.ny, 1, WALLS, ins.solid)
        u3 = np.zeros((1, ins.ny, ins.nx, 3))
        u3[0, ..., :2] = u[k]
        f0 = O.init_eq(lat, 1.0 + drho[k][None].astype(np.float64), u3)
        t3 = np.zeros((1, ins.ny, ins.nx, 3))
        t3[..., :2] = ins.target_u
        rin = 1.0 + dins[k]
        _, uo = O.macro(lat, O.run(lat, taus[k], rin, 1.0, f0, T))
        fl = lat.fluid()
        ug = ub[k].astype(np.float64).reshape(1, ins.ny, ins.nx, 2)
        assert rel(ug[fl], uo[..., :2][fl]) <= 1e-4, k
        go = O.grad(lat, taus[k], rin, 1.0, f0, T, t3, K=K)
        assert abs(lb[k] - go["loss"]) <= 1e-4 * go["loss"], k
        assert abs(gb["drho_in"][k] - go["drho_in"].sum()) <= 1e-3 * abs(go["drho_in"].sum()), k
        assert abs(gb["dtau"][k] - go["dtau"]) <= 1e-3 * abs(go["dtau"]), k
        assert abs(gb["drho_out"][k] - go["drho_out"].sum()) <= 1e-3 * abs(go["drho_out"].sum()), k
