"""Learned warm start: data generation, training and warm-versus-cold runs.

The paper suggests a neural-network initial guess to speed up its inverse
runs (Section 3.1.2 end, Section 3.5).  Here a U-Net (unet.py) learns the
map (solid mask, drho_in, drho_out, tau) -> Stokes-scaled steady (rho, u)
from steady states that the batched GPU solver itself produces; its
prediction, with the velocity of every cross-section rescaled to the mean
predicted flux (a steady flow carries the same flux through every section),
initialises equilibrium populations (Eq. 5) and the plain LBM
then runs to the residual threshold, so the converged state is the
solver's whatever the network predicts, and a poor prediction only costs
steps.

Synthetic media (stand-ins for the paper's packings): 2D 256 x 256 channels
between walls with overlapping disks (radii U[6, 14]); 3D 64^3 boxes,
periodic in y and z, with overlapping spheres (radii U[4, 8]); porosity
U[0.4, 0.8]; tau U[0.6, 1.2]; rho_in - 1 U[0.001, 0.006]; rho_out = 1.
Seeds: train 500000 + i, validation 600000 + i, test 700000 + i.

    python -m paper_2310_00810_amd.warmstart --dims 2 --train 2000 --epochs 20
"""
from __future__ import annotations

import argparse
import ctypes
import json
import os
import sys
import time

import numpy as np
import torch

from . import _lib as C
from . import geometry as G
from .lbm import Instance, Solver
from .unet import UNet

SEED_TRAIN, SEED_VAL, SEED_TEST = 500_000, 600_000, 700_000


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def sample(dims, seed, n2d=256, n3d=64):
    """(solid (nz, ny, nx) uint8, drho_in, drho_out, tau) of one seeded case."""
    rng = np.random.default_rng(seed)
    phi = rng.uniform(0.4, 0.8)
    tau = rng.uniform(0.6, 1.2)
    din = rng.uniform(0.001, 0.006)
    if dims == 2:
        solid = G.boolean_disks(n2d, n2d, (6.0, 14.0), phi, seed=seed)[None]
    else:
        solid = G.boolean_spheres((n3d, n3d, n3d), (4.0, 8.0), phi, seed=seed, periodic=(False, True, True))
    return solid.astype(np.uint8), din, 0.0, tau


def bc_of(dims):
    return ("pressure", "wall", "periodic") if dims == 2 else ("pressure", "periodic", "periodic")


def periodic_axes(dims):
    """Axes of a (nz, ny, nx) mask that bc_of(dims) makes periodic."""
    _, by, bz = bc_of(dims)
    return tuple(a for a, b in ((1, by), (0, bz)) if b == "periodic")


class Dataset:
    """Network inputs and Stokes-scaled targets, resident on the GPU, with the
    per-sample fluid pixel counts on the host."""

    def __init__(self, dims, cases, features, targets, wpix, prm, steps, dropped=0):
        self.dims, self.cases = dims, cases
        self.features, self.targets, self.wpix, self.prm, self.steps = features, targets, wpix, prm, steps
        self.nfluid = wpix.reshape(wpix.shape[0], -1).sum(1).round().long().cpu().numpy()
        self.dropped = dropped

    def __len__(self):
        return self.features.shape[0]


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def features_of(solid_dev, prm_dev, n, d, h, w):
    out = torch.empty((n, d, h, w, 8), dtype=torch.bfloat16, device="cuda")
    C.check(C.nnlib().lbmnn_features(ctypes.c_void_p(solid_dev.data_ptr()), ctypes.c_void_p(prm_dev.data_ptr()),
                                     n, d, h, w, ctypes.c_void_p(out.data_ptr()), _stream()), "lbmnn_features")
    return out


def generate(dims, seeds, batch=32, tol=1e-6, max_steps=100_000, check_every=100, flowing_only=False):
    """Runs the batched solver to the residual threshold for every seed and
    returns a Dataset (features, targets and fluid weights on the GPU) of the
    cases that reached it; cases still above the threshold at max_steps are
    left out (counted in Dataset.dropped).  A batch runs until its slowest
    case converges, and the steps to converge scale with 1 / nu, so the cases
    are batched in order of tau.  flowing_only: closed pockets of the pore
    space (geometry.flowing) get weight 0, since their state is the initial
    one and not a response to the pressure drop."""
    D = dims
    feats, tgts, wps, prms, steps, cases = [], [], [], [], [], []
    dropped = 0
    t0 = time.time()
    drawn = sorted((sample(dims, s) for s in seeds), key=lambda c: c[3])
    for b0 in range(0, len(drawn), batch):
        chunk = drawn[b0:b0 + batch]
        insts = [Instance(c[0].shape[2], c[0].shape[1], c[0].shape[0], solid=c[0]) for c in chunk]
        s = Solver(9 if dims == 2 else 19, insts, bc=bc_of(dims), steps=1)
        taus = [c[3] for c in chunk]
        dins = [c[1] for c in chunk]
        nstep, r = s.run_to_residual(taus, dins, 0.0, tol=tol, max_steps=max_steps, check_every=check_every)
        keep = np.flatnonzero(s.residuals() <= tol)
        drho, u = s.macro(mean2=True)
        nz, ny, nx = chunk[0][0].shape
        nb = len(chunk)
        solid = torch.from_numpy(np.stack([c[0] for c in chunk])).cuda()
        prm = torch.tensor([[c[1], c[2], c[3]] for c in chunk], dtype=torch.float32, device="cuda")
        per = nz * ny * nx
        tg = torch.empty((nb * per, 1 + D), dtype=torch.float32, device="cuda")
        wp = torch.empty(nb * per, dtype=torch.float32, device="cuda")
        C.check(C.nnlib().lbmnn_normalize(ctypes.c_void_p(drho.data_ptr()), ctypes.c_void_p(u.data_ptr()),
                                          ctypes.c_void_p(solid.data_ptr()), ctypes.c_void_p(prm.data_ptr()),
                                          per, D, nb * per, ctypes.c_void_p(tg.data_ptr()),
                                          ctypes.c_void_p(wp.data_ptr()), _stream()), "lbmnn_normalize")
        if flowing_only:
            fm = np.stack([G.flowing(c[0], periodic=periodic_axes(dims)) for c in chunk])
            wp *= torch.from_numpy(fm.reshape(-1).astype(np.float32)).cuda()
        kd = torch.from_numpy(keep).cuda()
        feats.append(features_of(solid, prm, nb, nz, ny, nx).index_select(0, kd))
        tgts.append(tg.view(nb, nz, ny, nx, 1 + D).index_select(0, kd))
        wps.append(wp.view(nb, nz, ny, nx).index_select(0, kd))
        prms.append(prm.index_select(0, kd))
        steps += [nstep] * keep.size
        cases += [chunk[k] for k in keep]
        dropped += nb - keep.size
        log(f"[data] dims={dims} {b0 + nb}/{len(drawn)} samples, batch ran {nstep} steps (largest r={r:.2e}), "
            f"{nb - keep.size} above the threshold left out, {time.time() - t0:.1f} s")
        del s
    return Dataset(dims, cases, torch.cat(feats), torch.cat(tgts), torch.cat(wps), torch.cat(prms),
                   np.array(steps), dropped)


def channel_scale(ds):
    """Root mean square of each target channel over fluid nodes: the
    network trains on targets divided by it, so that the small velocity
    channels weigh as much as the density channel in the loss."""
    t = ds.targets.reshape(-1, ds.targets.shape[-1])
    w = ds.wpix.reshape(-1, 1)
    ms = (t * t * w).sum(0) / w.sum().clamp(min=1.0)
    return ms.sqrt().clamp(min=1e-12)


def standardized(ds, scale):
    return Dataset(ds.dims, ds.cases, ds.features, (ds.targets / scale).contiguous(), ds.wpix, ds.prm, ds.steps,
                   ds.dropped)


def mirrored(x, tg, wp, axis, dims):
    """A batch reflected across the mid-plane of a transverse axis (1 = z in
    3D, 2 = y): walls and periodic boundaries are symmetric under it, the
    inputs depend on the transverse position only through the mask, and the
    velocity component along that axis changes sign."""
    comp = 1 + (1 if axis == 2 else 2)
    sign = torch.ones(tg.shape[-1], device=tg.device)
    sign[comp] = -1.0
    return x.flip(axis).contiguous(), (tg.flip(axis) * sign).contiguous(), wp.flip(axis).contiguous()


def reversed_flow(x, tg, wp, s0):
    """A batch reflected across the mid-plane normal to the flow (x), with
    the pressure drop turned back to its usual direction.  The creeping-flow
    steady state is linear in the drop and the inlet and outlet closures
    mirror each other, so the reflected medium's normalised state is the
    reflection of this one with t0 -> 1 - t0, the streamwise velocity kept
    and the transverse velocities negated.  The positional input channel
    (x / (w - 1)) stays as it is.  s0: the density channel's standardisation
    scale (the targets are divided by it)."""
    xf = x.flip(3)
    xf[..., 1] = x[..., 1]
    sign = torch.full((tg.shape[-1],), -1.0, device=tg.device)
    sign[1] = 1.0
    tf = tg.flip(3) * sign
    wf = wp.flip(3).contiguous()
    tf[..., 0] += wf / s0
    return xf.contiguous(), tf.contiguous(), wf


def evaluate_loss(net, ds, batch):
    tot, n = 0.0, 0
    for b0 in range(0, len(ds), batch):
        x = ds.features[b0:b0 + batch]
        out = net.forward(x)
        wp = ds.wpix[b0:b0 + batch]
        nfl = max(float(wp.sum().item()), 1.0)
        net.loss_and_grad(out, ds.targets[b0:b0 + batch].contiguous(), wp.contiguous(), 1.0 / nfl)
        tot += float(net.loss_dev.item()) * x.shape[0]
        n += x.shape[0]
    return tot / max(n, 1)


def train(net, ds, val, epochs, batch, lr, seed=0, augment=True, reverse_s0=None):
    """Adam with a cosine learning-rate schedule.  augment: each batch is
    reflected across a transverse mid-plane with probability 1/2 per axis,
    and, given reverse_s0 (the density channel's scale), across the
    streamwise mid-plane with the drop reversed (reversed_flow) with
    probability 1/2.
    With a validation set the weights of the epoch with the lowest validation
    loss are kept."""
    g = torch.Generator(device="cpu").manual_seed(seed)
    hist = []
    t0 = time.time()
    best, best_w = float("inf"), None
    axes = (2,) if ds.dims == 2 else (1, 2)
    for ep in range(epochs):
        perm = torch.randperm(len(ds), generator=g)
        tot = torch.zeros((), dtype=torch.float64, device=net.device)
        nb = 0
        lr_ep = lr * 0.5 * (1 + np.cos(np.pi * ep / max(epochs, 1)))
        for b0 in range(0, len(ds) - batch + 1, batch):
            sel = perm[b0:b0 + batch]
            idx = sel.cuda()
            x = ds.features.index_select(0, idx)
            tg = ds.targets.index_select(0, idx)
            wp = ds.wpix.index_select(0, idx)
            if augment:
                for ax in axes:
                    if torch.rand((), generator=g).item() < 0.5:
                        x, tg, wp = mirrored(x, tg, wp, ax, ds.dims)
                if reverse_s0 is not None and torch.rand((), generator=g).item() < 0.5:
                    x, tg, wp = reversed_flow(x, tg, wp, reverse_s0)
            tot += net.train_step(x, tg, wp, lr_ep, n_fluid=int(ds.nfluid[sel.numpy()].sum()))[0]
            nb += 1
        vl = evaluate_loss(net, val, batch) if val is not None and len(val) else float("nan")
        tl = float(tot.item()) / max(nb, 1)
        hist.append((ep, tl, vl))
        if vl < best:
            best, best_w = vl, net.master.clone()
        log(f"[train] epoch {ep + 1}/{epochs} loss {tl:.4e} val {vl:.4e} lr {lr_ep:.2e} {time.time() - t0:.1f} s")
    if best_w is not None:
        net.master.copy_(best_w)
        net.sync_bf16()
    return hist


def predict_fields(net, solid, din, dout, tau, balance=True):
    """Network prediction for one case -> (drho (nodes,), u (nodes, D)) on the GPU.
    balance: rescale the velocity of each cross-section so that every section
    carries the mean predicted flux (lbmnn_flux_balance), as the steady state
    does."""
    nz, ny, nx = solid.shape
    D = net.dims
    sd = torch.from_numpy(solid[None]).cuda()
    prm = torch.tensor([[din, dout, tau]], dtype=torch.float32, device="cuda")
    x = features_of(sd, prm, 1, nz, ny, nx)
    out = net.forward(x)
    per = nz * ny * nx
    drho = torch.empty(per, dtype=torch.float32, device="cuda")
    u = torch.empty(per, D, dtype=torch.float32, device="cuda")
    C.check(C.nnlib().lbmnn_denormalize(ctypes.c_void_p(out.data_ptr()), net.cout, ctypes.c_void_p(sd.data_ptr()),
                                        ctypes.c_void_p(prm.data_ptr()), per, D, per,
                                        ctypes.c_void_p(drho.data_ptr()), ctypes.c_void_p(u.data_ptr()),
                                        _stream()), "lbmnn_denormalize")
    if balance:
        L = C.nnlib()
        nb = L.lbmnn_flux_balance_workspace_bytes(1, nz, ny, nx)
        ws = torch.empty(-(-nb // 8), dtype=torch.float64, device="cuda")
        C.check(L.lbmnn_flux_balance(ctypes.c_void_p(sd.data_ptr()), 1, nz, ny, nx, D, ctypes.c_void_p(u.data_ptr()),
                                     ctypes.c_void_p(ws.data_ptr()), nb, _stream()), "lbmnn_flux_balance")
    return drho, u


def warm_vs_cold(net, case, tol=1e-6, max_steps=100_000, check_every=100):
    """Cold start (rest) and warm start (network prediction) of the same
    case, both run to the residual threshold.  Seconds include the network
    inference for the warm start."""
    solid, din, dout, tau = case
    dims = net.dims
    nz, ny, nx = solid.shape
    s = Solver(9 if dims == 2 else 19, [Instance(nx, ny, nz, solid=solid)], bc=bc_of(dims), steps=1)
    # warm-up of both paths (graph capture, kernel loading)
    s.run_to_residual(tau, din, dout, tol=1.0, max_steps=2 * check_every, check_every=check_every)
    predict_fields(net, solid, din, dout, tau)
    torch.cuda.synchronize()
    s.set_initial(None, None)
    t0 = time.perf_counter()
    sc, rc = s.run_to_residual(tau, din, dout, tol=tol, max_steps=max_steps, check_every=check_every)
    torch.cuda.synchronize()
    tc = time.perf_counter() - t0
    _, uc = s.macro(mean2=True)
    uc = uc.clone()
    t0 = time.perf_counter()
    drho_p, u_p = predict_fields(net, solid, din, dout, tau)
    s.set_initial(drho_p, u_p)
    sw, rw = s.run_to_residual(tau, din, dout, tol=tol, max_steps=max_steps, check_every=check_every)
    torch.cuda.synchronize()
    tw = time.perf_counter() - t0
    _, uw = s.macro(mean2=True)
    fl = torch.from_numpy(solid.reshape(-1) == 0).cuda()
    err_net = float(((u_p - uc)[fl].norm() / uc[fl].norm()).item())
    same = float(((uw - uc)[fl].norm() / uc[fl].norm()).item())
    return dict(cold_steps=sc, cold_s=tc, warm_steps=sw, warm_s=tw, net_rel_l2_u=err_net,
                warm_cold_rel_l2=same, cold_r=rc, warm_r=rw)


def summarize(res, tol):
    """Held-out figures on equal terms: how many cases each start brings to
    the threshold, and the step and time comparison over the cases where
    both do (medians; speed-up = cold seconds / warm seconds, inference
    included)."""
    both = [r for r in res if r["cold_r"] <= tol and r["warm_r"] <= tol]
    med = lambda k, rs: float(np.median([r[k] for r in rs])) if rs else None
    sp = [r["cold_s"] / r["warm_s"] for r in both]
    return {
        "cold_converged": int(sum(r["cold_r"] <= tol for r in res)),
        "warm_converged": int(sum(r["warm_r"] <= tol for r in res)),
        "both_converged": len(both),
        "cold_steps_median": med("cold_steps", both), "warm_steps_median": med("warm_steps", both),
        "cold_s_median": med("cold_s", both), "warm_s_median": med("warm_s", both),
        "speedup_median": float(np.median(sp)) if sp else None,
        "speedup_mean": float(np.mean(sp)) if sp else None,
        "warm_faster_fraction": float(np.mean([r["warm_s"] < r["cold_s"] for r in both])) if both else None,
        "net_rel_l2_u_median": med("net_rel_l2_u", res),
        "net_rel_l2_u_mean": float(np.mean([r["net_rel_l2_u"] for r in res])) if res else None,
        "warm_cold_rel_l2_max": float(np.max([r["warm_cold_rel_l2"] for r in both])) if both else None,
    }


def held_out(net, n, max_steps):
    res = []
    for i in range(n):
        case = sample(net.dims, SEED_TEST + i)
        r = warm_vs_cold(net, case, max_steps=max_steps)
        res.append(r)
        log(f"[test] {i}: cold {r['cold_steps']} steps {r['cold_s']:.3f} s, warm {r['warm_steps']} steps "
            f"{r['warm_s']:.3f} s, net err {r['net_rel_l2_u']:.3f}, warm/cold fixed point {r['warm_cold_rel_l2']:.1e}")
    return res


def evaluate_saved(args):
    """The held-out evaluation of saved weights with the current warm start;
    the training figures of their metadata are kept, the evaluation figures
    replaced (the previous ones kept under summary_before_reevaluation)."""
    net = UNet.load(args.eval_weights)
    res = held_out(net, args.test, args.max_steps)
    path = args.eval_weights[:-4] + ".json"
    meta = json.load(open(path))
    new = summarize(res, 1e-6)
    old = meta["summary"]
    meta["summary_before_reevaluation"] = {k: old[k] for k in new if k in old}
    old.update(new)
    old["test"] = args.test
    meta["tests"] = res
    meta["evaluation_command"] = "python -m paper_2310_00810_amd.warmstart " + " ".join(sys.argv[1:])
    print(json.dumps(old), flush=True)
    out = args.out or path
    os.makedirs(os.path.dirname(out) or ".", exist_ok=True)
    with open(out, "w") as f:
        json.dump(meta, f)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--dims", type=int, default=2)
    ap.add_argument("--train", type=int, default=2000)
    ap.add_argument("--val", type=int, default=200)
    ap.add_argument("--test", type=int, default=100)
    ap.add_argument("--epochs", type=int, default=30)
    ap.add_argument("--batch", type=int, default=0)
    ap.add_argument("--gen-batch", type=int, default=0)
    ap.add_argument("--lr", type=float, default=0.0, help="Adam learning rate (default 2e-3 in 2D, 5e-4 in 3D)")
    ap.add_argument("--out", default="")
    ap.add_argument("--max-steps", type=int, default=100_000)
    ap.add_argument("--levels", type=int, default=4, help="U-Net levels (the deepest runs at 1 / 2^(levels-1) size)")
    ap.add_argument("--eval-weights", default="",
                    help="only re-run the held-out evaluation of saved weights (.npz) and rewrite the summary of "
                         "their .json (to --out if given)")
    ap.add_argument("--reverse-flow", action="store_true",
                    help="also augment with the streamwise reflection and reversed drop (reversed_flow); "
                         "closed pockets of the pore space then carry no weight in the loss")
    args = ap.parse_args()
    if args.eval_weights:
        evaluate_saved(args)
        return
    dims = args.dims
    # 3D: batch 4 at lr 5e-4; at batch 2 and lr 2e-3 the 1000 Adam steps of an epoch over 2000
    # samples drove the network into a constant prediction
    batch = args.batch or (16 if dims == 2 else 4)
    lr = args.lr or (2e-3 if dims == 2 else 5e-4)
    gb = args.gen_batch or 64
    t0 = time.time()
    fo = args.reverse_flow
    tr = generate(dims, [SEED_TRAIN + i for i in range(args.train)], batch=gb, max_steps=args.max_steps,
                  flowing_only=fo)
    va = generate(dims, [SEED_VAL + i for i in range(args.val)], batch=gb, max_steps=args.max_steps,
                  flowing_only=fo) if args.val else None
    gen_s = time.time() - t0
    scale = channel_scale(tr)
    log(f"[data] target channel RMS {scale.cpu().numpy()}; steps to converge: median "
        f"{int(np.median(tr.steps))}, max {int(tr.steps.max())}")
    net = UNet(dims, levels=args.levels, seed=0)
    hist = train(net, standardized(tr, scale), standardized(va, scale) if va is not None else None, args.epochs,
                 batch, lr, reverse_s0=float(scale[0]) if args.reverse_flow else None)
    net.fold_output_scale(scale)
    train_s = time.time() - t0 - gen_s
    res = held_out(net, args.test, args.max_steps)
    summ = {"dims": dims, "levels": args.levels, "train": len(tr), "train_dropped": tr.dropped, "val": len(va) if va is not None else 0,
            "test": args.test, "epochs": args.epochs, "max_steps": args.max_steps, "gen_seconds": gen_s,
            "train_seconds": train_s, "final_train_loss": hist[-1][1] if hist else None,
            "best_val_loss": min(h[2] for h in hist) if hist and va is not None else None}
    summ.update(summarize(res, 1e-6))
    print(json.dumps(summ), flush=True)
    if args.out:
        os.makedirs(os.path.dirname(args.out) or ".", exist_ok=True)
        net.save(args.out)
        with open(args.out + ".json", "w") as f:
            json.dump({"command": "python -m paper_2310_00810_amd.warmstart " + " ".join(sys.argv[1:]),
                       "summary": summ, "history": hist, "tests": res,
                       "target_scale": scale.cpu().numpy().tolist()}, f)


if __name__ == "__main__":
    main()
