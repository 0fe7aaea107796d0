"""The trained warm-start network against the plain LBM (GPU).

The committed 2D and 3D weights were trained on solver-generated steady
states (seeds 500000+; the count is in each weight file's metadata).  On
held-out media (seeds
700000+) both starts must reach the 1e-6 residual, the warm start in fewer
steps and seconds (inference included) than the cold start, and both starts
must end at the same steady state."""
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

WDIR = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2310_00810_amd", "weights")
WEIGHTS = os.path.join(WDIR, "unet2d.npz")


def test_warm_start_beats_cold_start_on_held_out_media():
    from paper_2310_00810_amd import warmstart as W
    from paper_2310_00810_amd.unet import UNet
    net = UNet.load(WEIGHTS)
    res = [W.warm_vs_cold(net, W.sample(2, W.SEED_TEST + i), tol=1e-6, max_steps=100_000) for i in range(4)]
    print([(r["cold_steps"], r["warm_steps"], r["cold_s"], r["warm_s"]) for r in res])
    assert all(r["cold_r"] <= 1e-6 and r["warm_r"] <= 1e-6 for r in res)
    assert sum(r["warm_steps"] for r in res) < 0.8 * sum(r["cold_steps"] for r in res)
    assert sum(r["warm_s"] for r in res) < sum(r["cold_s"] for r in res)


def test_warm_and_cold_starts_reach_the_same_steady_state():
    """Both starts stepped far past the threshold agree to 1e-4 (relative L2
    of the two-step-mean velocity): the network only changes the path."""
    from paper_2310_00810_amd import geometry as G
    from paper_2310_00810_amd import warmstart as W
    from paper_2310_00810_amd.lbm import Instance, Solver
    from paper_2310_00810_amd.unet import UNet
    net = UNet.load(WEIGHTS)
    solid = G.boolean_disks(64, 64, (4.0, 8.0), 0.6, seed=11)[None].astype(np.uint8)
    din, tau = 0.004, 0.9
    s = Solver(9, [Instance(64, 64, 1, solid=solid)], bc=W.bc_of(2), steps=1)
    s.run_to_residual(tau, din, 0.0, tol=0.0, max_steps=60_000, check_every=100)
    _, uc = s.macro(mean2=True)
    uc = uc.clone()
    drho, u = W.predict_fields(net, solid, din, 0.0, tau)
    s.set_initial(drho, u)
    s.run_to_residual(tau, din, 0.0, tol=0.0, max_steps=60_000, check_every=100)
    _, uw = s.macro(mean2=True)
    fl = torch.from_numpy(solid.reshape(-1) == 0).cuda()
    assert ((uw - uc)[fl].norm() / uc[fl].norm()).item() <= 1e-4


def test_reversed_flow_matches_the_solver_on_the_reflected_medium():
    """The streamwise reflection that augments training (reversed_flow): the
    solver's steady state on the x-reflected medium equals the reflected and
    reversed steady state of the original on the nodes that flow (closed
    pockets keep their initial state), up to the flow's compressibility and
    inertia (density varies by drho_in across the channel)."""
    import ctypes
    from paper_2310_00810_amd import _lib as C
    from paper_2310_00810_amd import geometry as G
    from paper_2310_00810_amd import warmstart as W
    from paper_2310_00810_amd.lbm import Instance, Solver
    solid = G.boolean_disks(64, 48, (4.0, 8.0), 0.6, seed=11)[None].astype(np.uint8)
    pair = [solid, np.ascontiguousarray(solid[:, :, ::-1])]
    din, tau = 0.002, 0.9
    s = Solver(9, [Instance(64, 48, 1, solid=p) for p in pair], bc=W.bc_of(2), steps=1)
    s.run_to_residual(tau, din, 0.0, tol=0.0, max_steps=30_000, check_every=100)
    drho, u = s.macro(mean2=True)
    sd = torch.from_numpy(np.stack(pair)).cuda()
    prm = torch.tensor([[din, 0.0, tau]] * 2, dtype=torch.float32, device="cuda")
    per = 48 * 64
    tg = torch.empty((2 * per, 3), dtype=torch.float32, device="cuda")
    wp = torch.empty(2 * per, dtype=torch.float32, device="cuda")
    C.check(C.nnlib().lbmnn_normalize(ctypes.c_void_p(drho.data_ptr()), ctypes.c_void_p(u.data_ptr()),
                                      ctypes.c_void_p(sd.data_ptr()), ctypes.c_void_p(prm.data_ptr()), per, 2,
                                      2 * per, ctypes.c_void_p(tg.data_ptr()), ctypes.c_void_p(wp.data_ptr()),
                                      ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)),
            "lbmnn_normalize")
    tg, wp = tg.view(2, 1, 48, 64, 3), wp.view(2, 1, 48, 64)
    x = torch.zeros((1, 1, 48, 64, 8), dtype=torch.bfloat16, device="cuda")
    _, t_rev, w_rev = W.reversed_flow(x, tg[:1], wp[:1], 1.0)
    assert torch.equal(w_rev[0], wp[1])
    fl = torch.from_numpy(G.flowing(pair[1])).cuda().view(1, 48, 64)   # closed pockets keep their initial state
    assert bool((wp[1][fl] > 0).all())
    err_rho = (t_rev[0][..., 0] - tg[1][..., 0])[fl].abs().max().item()
    err_u = [((t_rev[0][..., c] - tg[1][..., c])[fl].norm() / tg[1][..., c][fl].norm()).item() for c in (1, 2)]
    print("reversed-flow mismatch: density", err_rho, "velocity", err_u)
    assert err_rho <= 1e-4 and max(err_u) <= 5e-3


def test_3d_warm_start_beats_cold_start_on_held_out_media():
    """D3Q19 64^3 sphere packings: the first four held-out media reach the
    1e-6 residual from both starts, the warm start in fewer steps, and the
    two converged fields agree to the accuracy the threshold leaves."""
    from paper_2310_00810_amd import warmstart as W
    from paper_2310_00810_amd.unet import UNet
    net = UNet.load(os.path.join(WDIR, "unet3d.npz"))
    res = [W.warm_vs_cold(net, W.sample(3, W.SEED_TEST + i), tol=1e-6, max_steps=100_000) for i in range(4)]
    print([(r["cold_steps"], r["warm_steps"], r["warm_cold_rel_l2"]) for r in res])
    assert all(r["cold_r"] <= 1e-6 and r["warm_r"] <= 1e-6 for r in res)
    assert sum(r["warm_steps"] for r in res) < 0.9 * sum(r["cold_steps"] for r in res)
    assert all(r["warm_cold_rel_l2"] <= 1e-3 for r in res)
