"""The trained warm-start network against the plain LBM (GPU).

The committed 2D and 3D weights were each trained on about 2000
solver-generated steady states (seeds 500000+).  On held-out media (seeds
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
