"""Drivers of the workloads: inverse runs, batched throughput, warm start.

    python -m paper_2310_00810_amd.run c1|c2|c3|c4|c5|e1|e7 [--quick]

Each prints one JSON line with its results.  The workloads are synthetic
stand-ins for the paper's experiments (Section 3): channel and granular
media with Zou-He pressure faces, inverse estimation of the inlet density
(constant head, Section 3.1.1; per-node profile, Section 3.1.2), of the
viscosity (Section 3.4) and the Darcy permeability along the optimisation
path (Section 3.2, Eq. 12).
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np
import torch

from . import geometry as G
from . import inverse
from ._lib import LBMError
from .lbm import Instance, Solver


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def c1(quick=False):
    """2D channel 64 x 32, tau = 0.8, 2000 steps: gradient of the mismatch to
    the rho_in = 1.003 velocity field at rho_in = 1.005, and a constant-head
    recovery from 1.0."""
    nx, ny, T = 64, 32, 2000
    s0 = Solver(9, [Instance(nx, ny)], steps=T)
    s0.forward(0.8, 0.003, 0.0, want_loss=False)
    _, ut = s0.macro()
    tgt = ut.cpu().numpy().reshape(1, ny, nx, 2)
    s = Solver(9, [Instance(nx, ny, target_u=tgt)], steps=T, tape=True)
    p, h = inverse.recover_constant_head(s, 0.8, 0.005, max_iter=15, rtol=1e-4, true_drho=0.003)
    return dict(config="C1", recovered_drho_in=p, true_drho_in=0.003, iterations=len(h.loss),
                loss=[float(x) for x in h.loss], grad_first=float(h.grads[0]))


def c2(quick=False):
    """D2Q9 512 x 256, RSA disks r ~ U[6, 14], porosity 0.70, seed 2,
    tau = 0.9, T = 10000, K = 500: recover rho_in (truth 1.004) from 1.0 by
    gradient descent with Armijo backtracking; Darcy permeability fitted over
    the iterates."""
    nx, ny, T, K, tau = 512, 256, 10000, 500, 0.9
    if quick:
        T, K = 2000, 100
    solid = G.rsa_disks(nx, ny, (6.0, 14.0), 0.70, seed=2)[None]
    s0 = Solver(9, [Instance(nx, ny, solid=solid)], steps=T)
    s0.forward(tau, 0.004, 0.0, want_loss=False)
    _, ut = s0.macro()
    tgt = ut.cpu().numpy().reshape(1, ny, nx, 2)
    s = Solver(9, [Instance(nx, ny, solid=solid, target_u=tgt)], steps=T, ckpt_interval=K, tape=True)
    t0 = time.time()
    p, h = inverse.recover_constant_head(s, tau, 0.0, max_iter=30, rtol=1e-3, true_drho=0.004)
    dt = time.time() - t0
    # Darcy: steady states of the medium at four pressure differences up to the recovered one
    k, pts = inverse.darcy_fit(s0, tau, [0.25 * p, 0.5 * p, 0.75 * p, p], solid)
    return dict(config="C2", recovered_drho_in=p, true_drho_in=0.004, iterations=len(h.loss),
                loss=[float(x) for x in h.loss], seconds=dt, darcy_k_lu2=k, porosity=G.porosity(solid),
                darcy_points=[dict(drho_in=d, q=q, grad_p=g, rho_mean=r, steps=n) for d, q, g, r, n in pts])


def c3(quick=False):
    """D3Q19 128^3 Boolean spheres r ~ U[6, 10], porosity 0.40, periodic y/z,
    inlet profile 1 + 0.004 phi (8 Fourier modes, seed 33), tau = 0.75,
    T = 8000, K = 400: joint Adam recovery of the 16384-node profile and tau
    from rho_in = 1.002, tau = 1.0 (MEAN_FLUID VEC loss)."""
    n, T, K = 128, 8000, 400
    iters = 20
    if quick:
        n, T, K, iters = 48, 1500, 100, 10
    solid = G.boolean_spheres((n, n, n), (6.0, 10.0) if n >= 96 else (3.0, 5.0), 0.40, seed=3)
    phi = G.fourier_profile(n, n, 8, seed=33)
    din_true = 0.004 * phi
    bc = ("pressure", "periodic", "periodic")
    s0 = Solver(19, [Instance(n, n, n, solid=solid)], bc=bc, steps=T, inlet_mode="profile")
    s0.forward(0.75, din_true.ravel(), 0.0, want_loss=False)
    _, ut = s0.macro()
    tgt = ut.cpu().numpy().reshape(n, n, n, 3)
    del s0
    s = Solver(19, [Instance(n, n, n, solid=solid, target_u=tgt)], bc=bc, steps=T, ckpt_interval=K, tape=True,
               loss_scale="mean", inlet_mode="profile")
    t0 = time.time()
    p, tau, h = inverse.recover_profile_and_tau(s, 1.0, np.full(n * n, 0.002), iters=iters, lr_in=2e-4,
                                                lr_tau=2e-2)
    dt = time.time() - t0
    rmse = float(np.sqrt(np.mean((p - din_true.ravel()) ** 2)))
    ratio = float(np.mean(p) / np.mean(din_true)) / (inverse.viscosity(tau) / inverse.viscosity(0.75))
    return dict(config="C3", size=n, T=T, iterations=iters, seconds=dt, loss=[float(x) for x in h.loss],
                recovered_tau=tau, true_tau=0.75, profile_rmse=rmse,
                profile_to_viscosity_ratio_rel=ratio)


def c4_instances(n_inst=64):
    """The batch of uneven D2Q9 media of ``geometry.c4_media`` as solver
    instances.  Returns (instances, taus, drho_ins)."""
    media = G.c4_media(n_inst)
    insts = [Instance(m["nx"], m["ny"], solid=m["solid"], target_u=m["target"][None]) for m in media]
    return insts, [m["tau"] for m in media], [m["drho_in"] for m in media]


def c4(quick=False, n_inst=64, T=5000):
    """64 D2Q9 instances (sizes from {128x64, 256x128, 512x256, 1024x512},
    seeds 4000 + b, porosity U[0.5, 0.8], tau U[0.6, 1.2], rho_in - 1
    U[0.001, 0.006]): forward + adjoint of all instances in one launch per
    step (graph-replayed) against a loop of single-instance launches."""
    if quick:
        n_inst, T = 8, 500
    insts, taus, dins = c4_instances(n_inst)
    nodes = sum(i.nodes for i in insts)
    K = int(np.ceil(np.sqrt(T)))
    log(f"[c4] {n_inst} instances, {nodes} nodes, T={T}, K={K}")
    bs = Solver(9, insts, steps=T, ckpt_interval=K, tape=True)

    def batched():
        bs.forward(taus, dins, 0.0, record_tape=True)
        bs.adjoint()
        return bs.grad()

    batched()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    gb = batched()
    torch.cuda.synchronize()
    tb = time.perf_counter() - t0
    # per-kernel averages (HIP events around the kernels, launched one by one)
    bs.set_timing(True, reset=True)
    batched()
    torch.cuda.synchronize()
    tm = bs.timing()
    bs.set_timing(False)
    n_fluid = sum(int((i.solid == 0).sum()) if i.solid is not None else i.nodes for i in insts)
    fwd_ms = tm["forward_ms"] / max(tm["forward_launches"], 1)
    adj_ms = tm["adjoint_ms"] / max(tm["adjoint_launches"], 1)
    kern = dict(fluid_nodes=n_fluid,
                k_step_avg_us=fwd_ms * 1e3, k_step_tbs=2 * 9 * 4 * n_fluid / (fwd_ms * 1e-3) / 1e12,
                k_adj_step_avg_us=adj_ms * 1e3, k_adj_step_tbs=3 * 9 * 4 * n_fluid / (adj_ms * 1e-3) / 1e12)
    kern["k_step_hbm_frac"] = kern["k_step_tbs"] / 8.0
    kern["k_adj_step_hbm_frac"] = kern["k_adj_step_tbs"] / 8.0
    del bs
    torch.cuda.empty_cache()
    singles = []
    for k, ins in enumerate(insts):
        s = Solver(9, [ins], steps=T, ckpt_interval=K, tape=True)
        s.set_graphs(False)
        singles.append(s)
    for k, s in enumerate(singles[:1]):
        s.forward(taus[k], dins[k], 0.0, record_tape=True)
        s.adjoint()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    gl = []
    for k, s in enumerate(singles):
        s.forward(taus[k], dins[k], 0.0, record_tape=True)
        s.adjoint()
        gl.append(s.grad())
    torch.cuda.synchronize()
    tl = time.perf_counter() - t0
    same = all(gl[k]["dtau"][0] == gb["dtau"][k] and gl[k]["drho_in"][0] == gb["drho_in"][k] for k in range(n_inst))
    return dict(config="C4", instances=n_inst, nodes=nodes, T=T, K=K,
                batched_seconds=tb, loop_seconds=tl,
                batched_fwd_adj_mlups=nodes * T / tb / 1e6, loop_fwd_adj_mlups=nodes * T / tl / 1e6,
                speedup=tl / tb, gradients_bitwise_equal=bool(same), kernels=kern)


def e1(quick=False):
    """Obstructed pipe with anti-bounce-back faces (Section 3.1.1): D2Q9
    300 x 50, walls in y, a 1 x 30 plate at x = 80, tau = 1, 40000 steps.
    The target is the velocity at the true pressure difference 0.05
    (drho = 0.15 with p = rho / 3), observed only at x >= 275 (NORM loss,
    Eq. 7 with f(x, y) = 1 there); the inlet density is recovered from the
    pressure difference 0.0025 (drho = 0.0075)."""
    nx, ny, T, tau = 300, 50, 40000, 1.0
    d_true, d0 = 0.15, 0.0075
    if quick:
        T = 4000
    solid = G.obstructed_pipe(nx, ny)
    bc = ("abb", "wall", "periodic")
    s0 = Solver(9, [Instance(nx, ny, solid=solid)], bc=bc, steps=T)
    s0.forward(tau, d_true, 0.0, want_loss=False)
    _, ut = s0.macro()
    tgt = ut.cpu().numpy().reshape(1, ny, nx, 2)
    roi = np.zeros((1, ny, nx), np.float32)
    roi[:, :, 275:] = 1.0
    s = Solver(9, [Instance(nx, ny, solid=solid, roi=roi, target_u=tgt)], bc=bc, steps=T, tape=True,
               loss_kind="norm")
    t0 = time.time()
    p, h = inverse.recover_constant_head(s, tau, d0, max_iter=20, rtol=1e-4, true_drho=d_true)
    dt = time.time() - t0
    # one timed gradient evaluation with per-kernel HIP events
    s.set_timing(True, reset=True)
    t1 = time.perf_counter()
    s.forward(tau, p, 0.0, record_tape=True)
    s.adjoint()
    s.grad()
    tg = time.perf_counter() - t1
    tm = s.timing()
    s.set_timing(False)
    n_fluid = int((solid == 0).sum())
    return dict(config="E1", T=T, iterations=len(h.loss), seconds=dt, recovered_drho_in=p, true_drho_in=d_true,
                recovered_pressure_difference=p / 3.0, loss=[float(x) for x in h.loss],
                gradient_seconds=tg, fwd_adj_mlups=nx * ny * T / tg / 1e6,
                k_step_avg_us=tm["forward_ms"] / max(tm["forward_launches"], 1) * 1e3,
                k_adj_step_avg_us=tm["adjoint_ms"] / max(tm["adjoint_launches"], 1) * 1e3,
                fluid_nodes=n_fluid)


def e7(quick=False, iters=50, nu0=0.06, scan=False, horizon=1200, frames=12, stride=100):
    """Viscosity from a cylinder wake (Section 3.4): D2Q9 MRT, Re = 100,
    nu = 0.02 (tau = 0.56), Zou-He velocity inlet, density outlet, periodic
    y.  At the paper's u = 0.2 lu/ts and D = 10 the density outlet does not
    survive the start-up waves, so the same Re and nu are run at half the
    Mach number: u = 0.1, D = 20, 800 x 320 nodes, cylinder 25 diameters
    before the outlet.  Uniform flow at t = 0; shedding is developed by
    20000 steps.  By default that developed flow is the start state and the
    target is the velocity in Raissi's window (1 to 8 diameters downstream,
    +-2 diameters across) over the next shedding period: 12 frames, 100
    steps apart, the last one 1200 steps later (the wake observed while it
    sheds).  With horizon 0 the target is the window at T = 20000
    from the uniform start, a final-time snapshot whose shedding phase makes
    the basin of the true viscosity very narrow.  frames > 1: the loss is
    summed over that many states, `stride` steps apart and ending at the
    target time (the wake observed over time; the shedding period is about
    1200 steps).  Adam on nu (learning rate 0.01) from nu = 0.06 by default;
    a step into a viscosity that the flow does not survive is halved back
    toward the last stable one."""
    nx, ny, D, U, T = 800, 320, 20, 0.1, 20000
    if quick:
        T, iters = 2000, 5
    nu_true = 0.02
    tau_of = lambda nu: 3.0 * nu + 0.5
    solid = G.cylinder_channel(nx, ny, D, 300, 160)
    bc = ("velocity", "periodic", "periodic")
    u0 = torch.zeros(nx * ny * 2, device="cuda")
    u0[0::2] = U
    zero = torch.zeros(nx * ny, device="cuda")
    s0 = Solver(9, [Instance(nx, ny, solid=solid)], bc=bc, steps=T, collision="mrt")
    s0.set_initial(zero, u0)
    s0.forward(tau_of(nu_true), U, 0.0, want_loss=False)
    developed = None
    if horizon:
        # observed from a developed wake: the start state is the shedding flow at T,
        # the target is the window `horizon` steps later
        developed = s0.get_populations()
        T = horizon
    # the target frames: the true run's velocity at T - (frames - 1 - m) stride
    times = [T - (frames - 1 - m) * stride for m in range(frames)]
    if times[0] < 1:
        raise ValueError("the loss frames must lie after the start")
    tgts = []
    for m, t in enumerate(times):
        st = Solver(9, [Instance(nx, ny, solid=solid)], bc=bc, steps=t - (times[m - 1] if m else 0),
                    collision="mrt")
        if m == 0:
            if developed is None:
                st.set_initial(zero, u0)
            else:
                st.set_populations(developed)
        else:
            st.set_populations(prev)
        st.forward(tau_of(nu_true), U, 0.0, want_loss=False)
        prev = st.get_populations()
        tgts.append(st.macro()[1].cpu().numpy().reshape(ny, nx, 2))
        del st
    tgt = np.stack(tgts)[:, None]
    del s0
    roi = np.zeros((1, ny, nx), np.float32)
    roi[:, 160 - 2 * D:160 + 2 * D, 300 + D:300 + 8 * D] = 1.0
    s = Solver(9, [Instance(nx, ny, solid=solid, roi=roi, target_u=tgt)], bc=bc, steps=T, tape=True,
               collision="mrt", loss_frames=frames, loss_stride=stride)
    if developed is None:
        s.set_initial(zero, u0)
    else:
        s.set_populations(developed)
    if scan:
        # the loss along nu: a final-time snapshot of a shedding wake depends on its phase
        pts = []
        for nu in np.linspace(0.016, 0.10, 43):
            try:
                L = float(s.forward(tau_of(float(nu)), U, 0.0, want_loss=True)[0])
            except LBMError:
                L = None  # this viscosity does not survive the start-up at this resolution
            pts.append({"nu": float(nu), "loss": L})
            log(f"[e7 scan] nu {nu:.4f} loss {L}")
        return dict(config="E7 scan", T=T, horizon=horizon, frames=frames, stride=stride, scan=pts)
    opt = inverse.Adam(0.01)
    nu = np.array([nu0])
    hist = []
    t0 = time.time()
    prev = nu.copy()
    for it in range(iters):
        try:
            L = s.forward(tau_of(float(nu[0])), U, 0.0, record_tape=True)[0]
        except LBMError:
            # too small a viscosity for this resolution: back off halfway to the last stable one
            log(f"[e7] it {it} nu {nu[0]:.5f} unstable")
            nu = 0.5 * (nu + prev)
            continue
        prev = nu.copy()
        s.adjoint()
        g = s.grad()
        dnu = 3.0 * g["dtau"][0]
        hist.append((float(nu[0]), float(L), float(dnu)))
        log(f"[e7] it {it} nu {nu[0]:.5f} loss {L:.4e} dL/dnu {dnu:.4e}")
        nu = np.maximum(opt.step(nu, np.array([dnu])), 0.002)
    dt = time.time() - t0
    best = min(hist, key=lambda h: h[1])
    return dict(config="E7", T=T, horizon=horizon, frames=frames, stride=stride, iterations=iters, seconds=dt, true_nu=nu_true, initial_nu=nu0,
                final_nu=float(nu[0]), best_nu=best[0], best_loss=best[1],
                trajectory=[{"nu": h[0], "loss": h[1], "dL_dnu": h[2]} for h in hist])


def e3(quick=False, iters=100, n_knots=8):
    """Variable inlet pressure drawn as a cubic spline (Section 3.2, the
    multi-parameter inversion): D2Q9 200 x 200 granular packing (Boolean
    disks r ~ U[5, 7] placed to porosity 0.49 and painted at the
    hydrodynamic radius 0.9 R, seed 7), walls in y, tau = 1, T = 5000.  The
    inlet density profile is the natural cubic spline through n_knots equally
    spaced knots (truth: seeded values in [0.003, 0.006]); the outlet density
    is 1.  The velocity is observed near the outlet only (x >= 180; the paper
    observes y > 180 with its flow along y).  Adam on the knot values (the
    profile gradient mapped through the spline, B^T g) from a uniform guess
    of 0.0045."""
    nx = ny = 200
    T, tau = 5000, 1.0
    if quick:
        T, iters = 500, 5
    solid = G.boolean_disks(nx, ny, (5.0, 7.0), 0.49, seed=7, hydro=0.9)[None]
    B = inverse.spline_basis(ny, n_knots)
    rng = np.random.default_rng(17)
    knots_true = rng.uniform(0.003, 0.006, n_knots)
    prof_true = B @ knots_true
    s0 = Solver(9, [Instance(nx, ny, solid=solid)], steps=T, inlet_mode="profile")
    s0.forward(tau, prof_true, 0.0, want_loss=False)
    _, ut = s0.macro()
    tgt = ut.cpu().numpy().reshape(1, ny, nx, 2)
    del s0
    roi = np.zeros((1, ny, nx), np.float32)
    roi[:, :, 180:] = 1.0
    s = Solver(9, [Instance(nx, ny, solid=solid, roi=roi, target_u=tgt)], steps=T, tape=True,
               inlet_mode="profile")
    opt = inverse.Adam(1e-4)
    knots = np.full(n_knots, 0.0045)
    hist = []
    t0 = time.time()
    for it in range(iters):
        L = s.forward(tau, B @ knots, 0.0, record_tape=True)[0]
        s.adjoint()
        gk = B.T @ s.grad()["drho_in"]
        rmse = float(np.sqrt(np.mean((B @ knots - prof_true) ** 2)))
        hist.append((float(L), rmse))
        if it % 10 == 0:
            log(f"[e3] it {it} loss {L:.4e} profile rmse {rmse:.3e}")
        knots = opt.step(knots, gk)
    dt = time.time() - t0
    prof = B @ knots
    rmse = float(np.sqrt(np.mean((prof - prof_true) ** 2)))
    return dict(config="E3", T=T, iterations=iters, seconds=dt, porosity=G.porosity(solid), knots=n_knots,
                true_knots=knots_true.tolist(), recovered_knots=knots.tolist(), profile_rmse=rmse,
                profile_rmse_pressure=rmse / 3.0, relative_rmse=rmse / float(np.sqrt(np.mean(prof_true ** 2))),
                loss_first=hist[0][0], loss_last=hist[-1][0])


def c5(quick=False):
    from . import warmstart
    sys.argv = [sys.argv[0], "--dims", "2", "--train", "64" if quick else "2000", "--val", "16" if quick else "200",
                "--test", "4" if quick else "30", "--epochs", "3" if quick else "30"]
    warmstart.main()
    return None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("config", choices=["c1", "c2", "c3", "c4", "c5", "e1", "e3", "e7"])
    ap.add_argument("--quick", action="store_true")
    ap.add_argument("--nu0", type=float, default=0.06, help="e7: initial viscosity")
    ap.add_argument("--scan", action="store_true", help="e7: loss along nu instead of the inversion")
    ap.add_argument("--horizon", type=int, default=1200,
                    help="e7: start from the developed wake and match the window this many steps later; 0: final-time snapshot from uniform flow")
    ap.add_argument("--frames", type=int, default=12, help="e7: loss frames (time-windowed loss)")
    ap.add_argument("--stride", type=int, default=100, help="e7: steps between loss frames")
    a = ap.parse_args()
    kw = dict(nu0=a.nu0, scan=a.scan, horizon=a.horizon, frames=a.frames, stride=a.stride) if a.config == "e7" else {}
    res = globals()[a.config](quick=a.quick, **kw)
    if res is not None:
        print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
