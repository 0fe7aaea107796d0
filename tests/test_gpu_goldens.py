"""GPU parity against the FP64 oracle at the workloads' stated step counts.

The expected values come from ``tests/golden/make_goldens.py``, which runs
only the oracle on the seeded inputs of the geometry module; the GPU runs the
same FP32 inputs here, in the launch configuration of the benchmark (graph
replays, resident tape segments, the recompute of the others beside the
adjoint on the second stream).  Bars: velocity relative L2 <= 1e-4, loss
relative 1e-4, gradients relative L2 <= 1e-3.

* 512 x 256 granular channel, T = 10 000, K = 500: the velocity at the truth
  (the golden's target) and at the guess, the loss and its three gradients.
* The sphere-box recipe on 64^3, T = 8000, K = 400: the velocity at the truth,
  then at the initial guess the loss, dL/drho_in at all 4096 inlet nodes,
  dL/dtau, dL/drho_out and the velocity at 20 000 sampled fluid nodes.
* The benchmark's 128^3 sphere box, T = 8000: the velocity at 20 000 sampled
  fluid nodes.
* The batch of 64 uneven channels in one launch per step, T = 5000, K = 71:
  loss, gradients and sampled velocity of 40 media.
"""
import os

import numpy as np
import pytest

from paper_2310_00810_amd import geometry as G

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def golden(name):
    path = os.path.join(GOLDEN, name + ".npz")
    if not os.path.exists(path):
        pytest.skip(f"{path} has not been generated (tests/golden/make_goldens.py {name})")
    return dict(np.load(path))


def rel(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def _release(s):
    del s
    torch.cuda.empty_cache()


def test_granular_channel_at_10000_steps():
    from paper_2310_00810_amd import lbm
    g = golden("c2")
    nx, ny, T = 512, 256, int(g["T"])
    solid = G.rsa_disks(nx, ny, (6.0, 14.0), 0.70, seed=2)[None]
    fl = solid[0] == 0
    target = g["target"]
    s = lbm.Solver(9, [lbm.Instance(nx, ny, solid=solid, target_u=target)], steps=T, ckpt_interval=500,
                   tape=True, resident_segments=2)
    s.forward(float(g["tau"]), float(g["drho_true"]), 0.0, want_loss=False)
    u = s.macro()[1].cpu().numpy().reshape(1, ny, nx, 2)
    assert rel(u[0][fl], target[0][fl]) <= 1e-4
    loss = s.forward(float(g["tau"]), float(g["drho_eval"]), 0.0, record_tape=True)[0]
    u = s.macro()[1].cpu().numpy().reshape(1, ny, nx, 2)
    assert rel(u[0][fl], g["u_eval"][0][fl]) <= 1e-4
    s.adjoint()
    gr = s.grad()
    assert abs(loss - g["loss"]) <= 1e-4 * g["loss"]
    for k in ("drho_in", "dtau", "drho_out"):
        assert rel(gr[k], [g[k]]) <= 1e-3, k
    _release(s)


def _box(n):
    solid = G.boolean_spheres((n, n, n), (6.0, 10.0), 0.40, seed=3, periodic=(False, True, True), x_margin=4)
    prof = (0.004 * G.fourier_profile(n, n, n_modes=8, seed=33)).astype(np.float32)
    return solid, prof


BOX = ("pressure", "periodic", "periodic")


def test_sphere_box_64_at_8000_steps():
    from paper_2310_00810_amd import lbm
    g = golden("c3_64")
    n, T = int(g["n"]), int(g["T"])
    solid, prof = _box(n)
    assert np.array_equal(prof, g["profile"])
    fl = solid == 0
    target = g["target"]
    s = lbm.Solver(19, [lbm.Instance(n, n, n, solid=solid, target_u=target)], bc=BOX, steps=T, ckpt_interval=400,
                   tape=True, loss_scale="mean", inlet_mode="profile", resident_segments=4)
    s.forward(float(g["tau_true"]), prof.ravel(), 0.0, want_loss=False)
    u = s.macro()[1].cpu().numpy().reshape(n, n, n, 3)
    assert rel(u[fl], target[fl]) <= 1e-4
    guess = np.full(n * n, float(g["drho_eval"]))
    loss = s.forward(float(g["tau_eval"]), guess, 0.0, record_tape=True)[0]
    u = s.macro()[1].cpu().numpy().reshape(-1, 3)
    assert rel(u[g["idx"]], g["u_eval"]) <= 1e-4
    s.adjoint()
    gr = s.grad()
    assert abs(loss - g["loss"]) <= 1e-4 * g["loss"]
    assert rel(gr["drho_in"], g["drho_in"].ravel()) <= 1e-3
    assert rel(gr["dtau"], [g["dtau"]]) <= 1e-3
    assert rel(gr["drho_out"], [g["drho_out"]]) <= 1e-3
    _release(s)


def test_sphere_box_128_velocity_at_8000_steps():
    from paper_2310_00810_amd import lbm
    g = golden("c3_128")
    n, T = int(g["n"]), int(g["T"])
    solid, prof = _box(n)
    s = lbm.Solver(19, [lbm.Instance(n, n, n, solid=solid)], bc=BOX, steps=T, inlet_mode="profile")
    s.forward(float(g["tau"]), prof.ravel(), 0.0, want_loss=False)
    u = s.macro()[1].cpu().numpy().reshape(-1, 3)
    assert rel(u[g["idx"]], g["u"]) <= 1e-4
    _release(s)


def test_batch_of_64_media_at_5000_steps():
    from paper_2310_00810_amd import lbm, run
    g = golden("c4")
    insts, taus, dins = run.c4_instances(64)
    dins = [float(np.float32(d)) for d in dins]
    s = lbm.Solver(9, insts, steps=int(g["T"]), ckpt_interval=int(g["K"]), tape=True, resident_segments=2)
    losses = s.forward(taus, dins, 0.0, record_tape=True)
    us = s.split(s.macro()[1].cpu().numpy())
    s.adjoint()
    gr = s.grad()
    for j, b in enumerate(g["media"]):
        k = int(g["n_idx"][j])
        idx = g["idx"][j][:k]
        assert rel(us[b][idx], g["u"][j][:k]) <= 1e-4, b
        assert abs(losses[b] - g["loss"][j]) <= 1e-4 * g["loss"][j], b
        for key in ("drho_in", "dtau", "drho_out"):
            assert abs(gr[key][b] - g[key][j]) <= 1e-3 * abs(g[key][j]), (b, key)
    _release(s)
