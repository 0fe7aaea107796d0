"""The benchmark's workload at full size, in the launch configuration the
benchmark times (D3Q19 128^3 Boolean spheres, porosity 0.40, periodic y/z,
per-node Fourier inlet profile, tau 0.75, T = 8000, K = 400, MEAN_FLUID VEC
loss against the velocity of a run at tau 0.9).  The oracle cannot follow
2 M nodes for 8000 steps, so at T = 8000 the checks are properties that hold
at any size: the tape layout does not change the gradient, and the adjoint's
derivatives match central differences of the GPU's own loss.  Over a few
steps the oracle does follow the full lattice, and there every population,
the loss and every gradient component are compared with it."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

N, T, K, TAU, TAU_TARGET = 128, 8000, 400, 0.75, 0.9


@pytest.fixture(scope="module")
def case():
    from paper_2310_00810_amd import geometry as G
    from paper_2310_00810_amd import lbm
    solid = G.boolean_spheres((N, N, N), (6.0, 10.0), 0.40, seed=3, periodic=(False, True, True), x_margin=4)
    din = (0.004 * G.fourier_profile(N, N, n_modes=8, seed=33)).astype(np.float32).ravel()
    bc = ("pressure", "periodic", "periodic")
    s0 = lbm.Solver(19, [lbm.Instance(N, N, N, solid=solid)], bc=bc, steps=T, inlet_mode="profile")
    s0.forward(TAU_TARGET, din, 0.0, want_loss=False)
    target = s0.macro()[1].cpu().numpy().reshape(N, N, N, 3)
    del s0
    torch.cuda.empty_cache()
    return solid, din, bc, target


def _solver(case, resident, tape=True):
    from paper_2310_00810_amd import lbm
    solid, din, bc, target = case
    return lbm.Solver(19, [lbm.Instance(N, N, N, solid=solid, target_u=target)], bc=bc, steps=T,
                      ckpt_interval=K, tape=tape, loss_scale="mean", inlet_mode="profile",
                      resident_segments=resident)


def test_resident_tape_segments_do_not_change_the_gradient(case):
    din = case[1]
    out = []
    for resident in (1, 3):
        s = _solver(case, resident)
        loss = s.forward(TAU, din, 0.0, record_tape=True)
        s.adjoint()
        out.append((loss[0], s.grad()))
        del s
        torch.cuda.empty_cache()
    (l1, g1), (l3, g3) = out
    assert l1 == l3
    for k in ("drho_in", "dtau", "drho_out"):
        assert np.array_equal(g1[k], g3[k]), k


def test_adjoint_matches_central_differences_of_the_gpu_loss(case):
    din = case[1].astype(np.float64)
    s = _solver(case, 2)
    s.forward(TAU, din, 0.0, record_tape=True)
    s.adjoint()
    g = s.grad()
    loss = lambda tau, d: s.forward(tau, d, 0.0, want_loss=True)[0]
    h = 1e-3
    fd_tau = (loss(TAU + h, din) - loss(TAU - h, din)) / (2 * h)
    assert abs(g["dtau"][0] - fd_tau) <= 1e-3 * abs(fd_tau)
    # along the profile itself: d/de L(din (1 + e))
    e = 2e-3
    fd_prof = (loss(TAU, din * (1 + e)) - loss(TAU, din * (1 - e))) / (2 * e)
    assert abs(float(np.dot(g["drho_in"], din)) - fd_prof) <= 1e-3 * abs(fd_prof)
    del s
    torch.cuda.empty_cache()


def test_full_size_steps_and_gradients_match_the_oracle(case):
    """The benchmark's lattice, boundaries, inlet profile, loss and launch
    configuration (graph replays, resident segments, the first segment
    recomputed on the second stream beside the adjoint) over T = 6 steps with
    K = 2, from a random equilibrium field set through the warm-start entry
    point, so the FP64 oracle can follow all 2 M nodes: the populations after
    T steps, the loss, and every gradient component.  An equilibrium start is
    left unchanged by collision at any tau, so the oracle's collide-first
    step convention and the solver's stream-first one give the same
    trajectory and the same dL/dtau."""
    import oracle as O
    from paper_2310_00810_amd import lbm
    solid, din, bc, _ = case
    steps, k_int = 6, 2
    lat = O.Lattice(19, N, N, N, (O.BC_PRESSURE, O.BC_PERIODIC, O.BC_PERIODIC), solid)
    fl = lat.fluid()
    rng = np.random.default_rng(17)
    drho = (0.01 * rng.standard_normal(lat.shape) * fl).astype(np.float32)
    u = (0.01 * rng.standard_normal(lat.shape + (3,)) * fl[..., None]).astype(np.float32)
    tgt = (1e-3 * rng.standard_normal(lat.shape + (3,))).astype(np.float32)
    s = lbm.Solver(19, [lbm.Instance(N, N, N, solid=solid, target_u=tgt)], bc=bc, steps=steps,
                   ckpt_interval=k_int, tape=True, loss_scale="mean", inlet_mode="profile",
                   resident_segments=2)
    assert s.resident_segments == 2           # of 3 segments: one is recomputed
    s.set_initial(torch.from_numpy(drho.ravel()).cuda(), torch.from_numpy(u.reshape(-1, 3)).cuda())
    loss = s.forward(TAU, din, 0.0, record_tape=True)[0]
    state = s.get_populations("state").cpu().numpy().astype(np.float64).reshape((19,) + lat.shape)
    s.adjoint()
    g = s.grad()
    del s
    torch.cuda.empty_cache()

    f0 = O.init_eq(lat, 1.0 + drho.astype(np.float64), u.astype(np.float64))
    rin = 1.0 + din.astype(np.float64).reshape(N, N)
    nfl = int(fl.sum())
    go = O.grad(lat, TAU, rin, 1.0, f0, steps, tgt.astype(np.float64), scale=1.0 / nfl, K=k_int)
    # solver state = post-collision populations of the oracle's state after T steps
    _, w, _ = O.velset(19)
    ref = O.collide(lat, TAU, O.run(lat, TAU, rin, 1.0, f0, steps)) - w
    got = np.moveaxis(state, 0, -1)
    err = np.linalg.norm((got - ref)[fl]) / np.linalg.norm(ref[fl])
    assert err <= 1e-5, err
    assert abs(loss - go["loss"]) <= 1e-4 * go["loss"]
    for key, ref_g in (("drho_in", go["drho_in"].ravel()), ("dtau", [go["dtau"]]),
                       ("drho_out", [go["drho_out"].sum()])):
        ref_g = np.asarray(ref_g, np.float64)
        e = np.linalg.norm(np.asarray(g[key], np.float64) - ref_g) / np.linalg.norm(ref_g)
        assert e <= 1e-3, (key, e)
