"""Benchmark of the differentiable LBM hot path on one MI355X.

One benchmark step is one full gradient evaluation of the 3D inverse
problem (inlet pressure profile + viscosity in a packed-sphere box):
taped forward over T steps with checkpoints every K, loss, reverse sweep
(segment recompute + adjoint steps), gradient reductions.

Workload (synthetic stand-in for the paper's 3D granular media): D3Q19,
128^3 nodes, overlapping spheres with radii U[6, 10] to porosity 0.40
(seed 3), periodic y and z, Zou-He inlet profile rho_in = 1 + 0.004 phi
(phi: 8 Fourier modes, seed 33), rho_out = 1, tau = 0.75, T = 8000, K = 400,
VEC loss against the velocity of a second run at tau = 0.9, mean over
fluid nodes.

The taped forward keeps the states of as many trailing K-step segments as fit
in device memory (288 GB on MI355X: 11 of the 20 segments here), so the
reverse sweep recomputes only the others; `--resident 1` keeps only the last
one.  The gradient is bit for bit the same either way.

Prints ONE JSON line.  value = forward+adjoint MLUPS (all lattice nodes x T
per second of the whole gradient evaluation).  roofline = the dominant kernel
of that evaluation, k_step (forward pass and segment recomputes: about 57 % of
the GPU time), averaged over all its launches; adj_roofline = k_adj_step.
Both use algorithmic bytes (152 B and 228 B per fluid node) over HIP-event
kernel times on the library stream.  The 128^3 box's working set (63.6 MB per
state) is partly served by the 256 MB Infinity Cache, so hbm_resident_roofline
repeats the two kernel figures on a 256^3 plane channel (1.27 GB per state).
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLUPS fwd & fwd+adjoint (D3Q19 grains) vs HBM roofline; warm vs cold solve sec"
HBM_PEAK_GBS = 8000.0
Q = 19
BYTES_FWD = 2 * Q * 4        # read + write one population set per fluid node
BYTES_ADJ = 3 * Q * 4        # gather F^{k-1}, gather nu^{k+1}, write nu^k
PROFILES = os.path.join(ROOT, "profiles")
# kernel names as the profiler reports them (template arguments: Q, x boundary kind = pressure,
# adjoint: no loss frame on the step, then the cache policy: the 128^3 states fit the Infinity
# Cache, so steps into the ping-pong pair and the adjoint keep the default policy and steps into
# the tape store non-temporal)
ADJ_KERNEL = "k_adj_step<19, 0, false, false>"
FWD_KERNEL = "k_step<19, 0, *>"
FWD_VARIANTS = ("k_step<19, 0, 0>", "k_step<19, 0, 1>")      # into the ping-pong pair, into the tape


def workload(n=128, T=8000, K=400, kind="spheres"):
    from paper_2310_00810_amd import geometry as G
    phi = G.fourier_profile(n, n, n_modes=8, seed=33)
    if kind == "channel":
        # plane channel: walls in y, periodic z, no grains (kernel efficiency on a working set
        # far larger than the 256 MB last-level cache)
        return dict(n=n, T=T, K=K, solid=np.zeros((n, n, n), np.uint8), din=(0.004 * phi).astype(np.float32),
                    tau=0.75, tau_target=0.9, bc=("pressure", "wall", "periodic"), kind=kind)
    solid = G.boolean_spheres((n, n, n), (6.0, 10.0), 0.40, seed=3, periodic=(False, True, True), x_margin=4)
    return dict(n=n, T=T, K=K, solid=solid, din=(0.004 * phi).astype(np.float32), tau=0.75, tau_target=0.9,
                bc=("pressure", "periodic", "periodic"), kind=kind)


def channel_roofline(torch, n=256, T=40, K=20):
    """k_step and k_adj_step against the HBM peak on a working set far larger
    than the 256 MB Infinity Cache: a D3Q19 n^3 plane channel (1.27 GB per
    state at n = 256), one timed gradient evaluation after one untimed."""
    from paper_2310_00810_amd import lbm
    w = workload(n, T, K, "channel")
    ins = lbm.Instance(n, n, n, solid=w["solid"], target_u=np.zeros((n, n, n, 3), np.float32))
    s = lbm.Solver(19, [ins], bc=w["bc"], steps=T, ckpt_interval=K, tape=True, loss_scale="mean",
                   inlet_mode="profile")
    for timed in (False, True):
        s.set_timing(timed, reset=True)
        s.forward(w["tau"], w["din"].ravel(), 0.0, record_tape=True)
        s.adjoint()
        s.grad()
    torch.cuda.synchronize()
    tm = s.timing()
    del s
    torch.cuda.empty_cache()
    nodes = n ** 3
    step_ms = (tm["forward_ms"] + tm["recompute_ms"]) / max(tm["forward_launches"] + tm["recompute_launches"], 1)
    adj_ms = tm["adjoint_ms"] / max(tm["adjoint_launches"], 1)
    f = lambda b, ms: round(b * nodes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
    return {"workload": f"D3Q19 {n}^3 plane channel, walls y, periodic z, T={T}, K={K}",
            "k_step_frac": f(BYTES_FWD, step_ms), "k_step_avg_launch_ms": round(step_ms, 5),
            "k_adj_step_frac": f(BYTES_ADJ, adj_ms), "k_adj_step_avg_launch_ms": round(adj_ms, 5)}


def d2q9_batch(torch, T=5000):
    """The D2Q9 grain-media batch: 64 uneven RSA-disk media (11.0 M nodes) in
    one launch per step, T = 5000, K = ceil(sqrt(T)).  Forward-only and
    forward+adjoint MLUPS of graph-replayed passes (one untimed pass of each
    first), and k_step / k_adj_step against the HBM peak from HIP events
    around launches one by one."""
    from paper_2310_00810_amd import lbm, run
    insts, taus, dins = run.c4_instances(64)
    nodes = sum(i.nodes for i in insts)
    fluid = sum(int((i.solid == 0).sum()) for i in insts)
    K = int(np.ceil(np.sqrt(T)))
    s = lbm.Solver(9, insts, steps=T, ckpt_interval=K, tape=True, resident_segments="max")

    def fwd():
        s.forward(taus, dins, 0.0, want_loss=False)

    def grad():
        s.forward(taus, dins, 0.0, record_tape=True)
        s.adjoint()
        s.grad()

    secs = {}
    for name, fn in (("fwd", fwd), ("grad", grad)):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        secs[name] = time.perf_counter() - t0
    s.set_timing(True, reset=True)
    grad()
    torch.cuda.synchronize()
    tm = s.timing()
    s.set_timing(False)
    resident = s.resident_segments
    del s
    torch.cuda.empty_cache()
    step_ms = (tm["forward_ms"] + tm["recompute_ms"]) / max(tm["forward_launches"] + tm["recompute_launches"], 1)
    adj_ms = tm["adjoint_ms"] / max(tm["adjoint_launches"], 1)
    f = lambda b, ms: round(b * fluid / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
    return {"workload": f"D2Q9 batch of 64 RSA-disk media (128x64 .. 1024x512, porosity U[0.5,0.8]), "
                        f"one launch per step, T={T}, K={K}",
            "nodes": nodes, "fluid_nodes": fluid, "resident_segments": resident,
            "recomputed_steps": tm["recompute_launches"],
            "fwd_mlups": round(nodes * T / secs["fwd"] / 1e6, 1),
            "fwd_adj_mlups": round(nodes * T / secs["grad"] / 1e6, 1),
            "fwd_s": round(secs["fwd"], 4), "fwd_adj_s": round(secs["grad"], 4),
            "k_step_frac": f(2 * 9 * 4, step_ms), "k_step_avg_launch_ms": round(step_ms, 5),
            "k_adj_step_frac": f(3 * 9 * 4, adj_ms), "k_adj_step_avg_launch_ms": round(adj_ms, 5)}


def load_traffic(kernel, weights=None):
    """HBM bytes per launch from the committed rocprofv3 --pmc summary of this
    kernel, if it was taken on the current kernel source; else None.  With
    weights {variant name: launches}, the launch-weighted mean over the
    variants (all of them must have been measured)."""
    p = os.path.join(PROFILES, "pmc_traffic.json")
    if not os.path.exists(p):
        return None
    try:
        d = json.load(open(p))
    except Exception:
        return None
    from paper_2310_00810_amd.profiling import kernel_source_hash
    h = kernel_source_hash()
    parts = weights or {kernel: 1}
    tot = n = 0
    for name, w in parts.items():
        e = d.get(name)
        if not e or e.get("source_hash") != h:
            return None
        tot += w * e["bytes_per_launch"]
        n += w
    return tot / n if n else None


def copy_peak_gbs(torch, nbytes=4 << 30, reps=10):
    """Measured device-to-device copy bandwidth (read + write bytes / s): the
    library's 16-byte-per-lane copy (the fastest plain stream measured on the
    chip) and torch's copy."""
    import ctypes
    from paper_2310_00810_amd import _lib as C
    x = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    x.fill_(1.0)
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    out = {}
    for name, fn in (("copy16", lambda: C.check(C.lib().lbm_stream_copy(ctypes.c_void_p(y.data_ptr()),
                                                                        ctypes.c_void_p(x.data_ptr()), nbytes,
                                                                        stream), "lbm_stream_copy")),
                     ("torch", lambda: y.copy_(x))):
        fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            fn()
        b.record()
        torch.cuda.synchronize()
        out[name] = 2 * nbytes * reps / (a.elapsed_time(b) * 1e-3) / 1e9
    del x, y
    torch.cuda.empty_cache()
    return out


def warm_vs_cold(torch, n2d=8, n3d=4):
    """Warm start (committed trained U-Nets) against cold start on held-out
    media (test seeds 700000+): seconds to the 1e-6 residual, inference
    included, compared over the cases where both starts reach it; plus the
    training run's own evaluation over its 100 held-out media."""
    from paper_2310_00810_amd import warmstart as W
    from paper_2310_00810_amd.unet import UNet
    out = {}
    for dims, cases in ((2, n2d), (3, n3d)):
        path = os.path.join(ROOT, "paper_2310_00810_amd", "weights", f"unet{dims}d.npz")
        if not os.path.exists(path):
            continue
        net = UNet.load(path)
        res = [W.warm_vs_cold(net, W.sample(dims, W.SEED_TEST + i), tol=1e-6, max_steps=100_000)
               for i in range(cases)]
        entry = {"cases": cases, "workload": ("D2Q9 256^2 Boolean disks" if dims == 2 else
                                              "D3Q19 64^3 Boolean spheres") + ", porosity U[0.4,0.8], test seeds 700000+"}
        entry.update({k: (round(v, 5) if isinstance(v, float) else v) for k, v in W.summarize(res, 1e-6).items()})
        try:
            entry["training_run_evaluation"] = json.load(open(path[:-4] + ".json"))["summary"]
        except (OSError, ValueError, KeyError):
            pass
        out[f"{dims}d"] = entry
        del net
    return out


def cpu_baseline(w, cold_steps_2d=None):
    """The FP64 oracle on the host cores, built with -O3 -march=native for
    this host, timed on bounded samples of the workloads: all host threads
    (OMP_NUM_THREADS, else the CPU count) and, for the benchmark's own
    workload, one thread.  value: forward + reverse gradient MLUPS of the
    benchmark's 128^3 problem (a few steps)."""
    import tempfile
    import oracle as O
    from oracle import build as ob
    from paper_2310_00810_amd import geometry as G
    from paper_2310_00810_amd import warmstart as W
    tmp = tempfile.mkdtemp()
    O.load(ob.build(out=os.path.join(tmp, "liblbm_oracle_native.so"), native=True))
    cores = int(os.environ.get("OMP_NUM_THREADS") or os.cpu_count() or 1)
    O.set_threads(cores)
    model = "unknown CPU"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass

    def timed(fn):
        t0 = time.perf_counter()
        fn()
        return time.perf_counter() - t0

    def pair(lat, tau, rin, steps_f, steps_g, K=0, scale=1.0):
        f0 = O.init_eq(lat, 1.0, 0.0)
        tgt = np.zeros(lat.shape + (3,))
        nodes = lat.nx * lat.ny * lat.nz
        tf = timed(lambda: O.run(lat, tau, rin, 1.0, f0, steps_f))
        tg = timed(lambda: O.grad(lat, tau, rin, 1.0, f0, steps_g, tgt, scale=scale, K=K or steps_g))
        return nodes * steps_f / tf / 1e6, nodes * steps_g / tg / 1e6, tf + tg

    walls = (O.BC_PRESSURE, O.BC_WALL, O.BC_PERIODIC)
    n = w["n"]
    lat3 = O.Lattice(19, n, n, n, (O.BC_PRESSURE, O.BC_PERIODIC, O.BC_PERIODIC), w["solid"])
    nfl = int(lat3.fluid().sum())
    rin3 = 1.0 + w["din"].astype(np.float64)
    c3f, c3g, c3t = pair(lat3, w["tau"], rin3, 12, 4, scale=1.0 / nfl)
    O.set_threads(1)
    f0 = O.init_eq(lat3, 1.0, 0.0)
    t1 = timed(lambda: O.grad(lat3, w["tau"], rin3, 1.0, f0, 1, np.zeros(lat3.shape + (3,)), scale=1.0 / nfl, K=1))
    O.set_threads(cores)
    configs = {"c3_128_spheres": {"fwd_mlups": round(c3f, 3), "fwd_adj_mlups": round(c3g, 3),
                                  "fwd_adj_mlups_1_thread": round(n ** 3 / t1 / 1e6, 3),
                                  "sample": "128^3 spheres: 12 forward steps; 4-step gradient; 1-step gradient on "
                                            "one thread"}}
    lat1 = O.Lattice(9, 64, 32, 1, walls)
    f, g, _ = pair(lat1, 0.8, 1.005, 2000, 2000, K=45)
    configs["c1_64x32_channel"] = {"fwd_mlups": round(f, 3), "fwd_adj_mlups": round(g, 3),
                                   "sample": "full T = 2000 (K = 45)"}
    lat2 = O.Lattice(9, 512, 256, 1, walls, G.rsa_disks(512, 256, (6.0, 14.0), 0.70, seed=2)[None])
    f, g, _ = pair(lat2, 0.9, 1.004, 200, 200, K=20)
    configs["c2_512x256_grains"] = {"fwd_mlups": round(f, 3), "fwd_adj_mlups": round(g, 3),
                                    "sample": "200 of the 10 000 steps (K = 20)"}
    media = G.c4_media(8)
    fsum = gsum = work = 0.0
    for m in media:
        lat = O.Lattice(9, m["nx"], m["ny"], 1, walls, m["solid"])
        f, g, _ = pair(lat, m["tau"], 1.0 + m["drho_in"], 100, 100, K=10)
        nodes = m["nx"] * m["ny"] * 100
        fsum += nodes / f
        gsum += nodes / g
        work += nodes
    configs["c4_batch"] = {"fwd_mlups": round(work / fsum, 3), "fwd_adj_mlups": round(work / gsum, 3),
                           "sample": "the first 8 of the 64 media, 100 steps each, one after another"}
    solid, din, dout, tau = W.sample(2, W.SEED_TEST)
    lat5 = O.Lattice(9, 256, 256, 1, walls, solid)
    f0 = O.init_eq(lat5, 1.0, 0.0)
    t5 = timed(lambda: O.run(lat5, tau, 1.0 + din, 1.0 + dout, f0, 500))
    c5 = {"fwd_mlups": round(256 * 256 * 500 / t5 / 1e6, 3), "s_per_step": t5 / 500,
          "sample": "held-out 2D medium (seed 700000), 500 forward steps"}
    if cold_steps_2d:
        c5["cold_start_s_extrapolated"] = round(t5 / 500 * cold_steps_2d, 2)
        c5["cold_steps"] = int(cold_steps_2d)
    configs["c5_2d_cold_start"] = c5
    return {"value": round(c3g, 3), "unit": "MLUPS", "cores": cores, "kind": "oracle",
            "sample": f"FP64 oracle (-O3 -march=native) forward + reverse gradient of the benchmark's 128^3 "
                      f"D3Q19 problem over 4 steps (K = 4), OpenMP on {cores} threads of {model}; per-workload "
                      f"samples in configs",
            "configs": configs}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--size", type=int, default=128)
    ap.add_argument("--workload", choices=["spheres", "channel"], default="spheres")
    ap.add_argument("--T", type=int, default=8000)
    ap.add_argument("--K", type=int, default=400)
    ap.add_argument("--resident", default="max",
                    help="tape segments kept resident by the taped forward (an integer, or 'max': as many as "
                         "fit in device memory); the others are recomputed in the reverse sweep")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-copy", action="store_true", help="skip the copy-bandwidth calibration")
    ap.add_argument("--no-warm", action="store_true", help="skip the warm-versus-cold start comparison")
    ap.add_argument("--no-channel", action="store_true", help="skip the 256^3 channel roofline")
    ap.add_argument("--no-d2q9", action="store_true", help="skip the D2Q9 grain-media batch")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU (the several-GPU slab decomposition is design only); --gpus must be 1"}))
        sys.exit(2)

    import torch
    from paper_2310_00810_amd import lbm

    w = workload(args.size, args.T, args.K, args.workload)
    n, T, K = w["n"], w["T"], w["K"]
    fluid_frac = float((w["solid"] == 0).mean())
    n_fluid = int((w["solid"] == 0).sum())
    print(f"[bench] workload D3Q19 {n}^3 porosity {fluid_frac:.3f} T={T} K={K}", file=sys.stderr, flush=True)

    # target velocity from a run at another tau (the inverse problem recovers tau and the profile)
    ins0 = lbm.Instance(n, n, n, solid=w["solid"])
    s0 = lbm.Solver(19, [ins0], bc=w["bc"], steps=T, inlet_mode="profile")
    s0.forward(w["tau_target"], w["din"].ravel(), 0.0, want_loss=False)
    _, ut = s0.macro()
    target = ut.cpu().numpy().reshape(n, n, n, 3)
    del s0, ut
    torch.cuda.empty_cache()

    ins = lbm.Instance(n, n, n, solid=w["solid"], target_u=target)
    s = lbm.Solver(19, [ins], bc=w["bc"], steps=T, ckpt_interval=K, tape=True,
                   loss_scale="mean", inlet_mode="profile",
                   resident_segments=args.resident if args.resident == "max" else int(args.resident))
    print(f"[bench] workspace {s.workspace_bytes / 2**30:.1f} GiB, {s.resident_segments} resident tape segments",
          file=sys.stderr, flush=True)

    def one():
        s.forward(w["tau"], w["din"].ravel(), 0.0, record_tape=True)
        s.adjoint()
        return s.grad()

    for i in range(args.warmup):
        one()
        print(f"[bench] warmup {i + 1}/{args.warmup} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        g = one()
        print(f"[bench] step {i + 1}/{args.steps} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    # one more evaluation with per-phase HIP events (kernels launched one by one
    # between events on the library stream) for the per-kernel averages
    s.set_timing(True, reset=True)
    one()
    torch.cuda.synchronize()
    tm = s.timing()
    s.set_timing(False)

    ms_step = dt / args.steps * 1e3
    value = n ** 3 * T / (ms_step * 1e-3) / 1e6
    fwd_ms = tm["forward_ms"] / max(tm["forward_launches"], 1)
    adj_ms = tm["adjoint_ms"] / max(tm["adjoint_launches"], 1)
    rec_ms = tm["recompute_ms"] / max(tm["recompute_launches"], 1)
    # k_step runs the forward pass and the segment recomputes: its average over
    # all launches of one gradient evaluation is the dominant kernel's figure
    step_launches = tm["forward_launches"] + tm["recompute_launches"]
    step_ms = (tm["forward_ms"] + tm["recompute_ms"]) / max(step_launches, 1)
    # launches into the ping-pong pair: the steps of the segments that are not kept (their first
    # step writes a checkpoint) and the last step; every other launch writes the tape
    pp_launches = max(-(-T // K) - s.resident_segments, 0) * (K - 1) + 1
    adj_bytes = BYTES_ADJ * n_fluid
    fwd_bytes = BYTES_FWD * n_fluid
    adj_gbs = adj_bytes / (adj_ms * 1e-3) / 1e9
    step_gbs = fwd_bytes / (step_ms * 1e-3) / 1e9
    fwd_mlups = n ** 3 / (fwd_ms * 1e-3) / 1e6

    out = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": (f"D3Q19 {n}^3 packed spheres r~U[6,10] porosity 0.40, periodic y/z, "
                                if w["kind"] == "spheres" else f"D3Q19 {n}^3 plane channel, walls y, periodic z, ")
                               + f"Zou-He profile inlet (8 Fourier modes) + tau gradient, T={T}, K={K}, "
                               f"one step = taped forward + reverse sweep",
                   "lattice": "D3Q19", "nodes": n ** 3, "fluid_nodes": n_fluid, "T": T, "K": K,
                   "resident_segments": s.resident_segments, "recomputed_steps": tm["recompute_launches"],
                   "workspace_gib": round(s.workspace_bytes / 2 ** 30, 1)},
        "roofline": {"bound": "hbm", "achieved": round(step_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(step_gbs / HBM_PEAK_GBS, 4),
                     "traffic": load_traffic(FWD_KERNEL, {FWD_VARIANTS[0]: pp_launches,
                                                          FWD_VARIANTS[1]: step_launches - pp_launches}),
                     "kernel": FWD_KERNEL, "bytes_per_launch": fwd_bytes, "avg_launch_ms": round(step_ms, 5),
                     "launches": "forward + segment recompute, one gradient evaluation"},
        "adj_roofline": {"kernel": ADJ_KERNEL, "achieved": round(adj_gbs, 1), "unit": "GB/s",
                         "frac": round(adj_gbs / HBM_PEAK_GBS, 4), "avg_launch_ms": round(adj_ms, 5),
                         "bytes_per_launch": adj_bytes, "traffic": load_traffic(ADJ_KERNEL)},
        "value_fluid_mlups": round(n_fluid * T / (ms_step * 1e-3) / 1e6, 1),
        "fwd_mlups": round(fwd_mlups, 1),
        "fwd_fluid_mlups": round(n_fluid / (fwd_ms * 1e-3) / 1e6, 1),
        "k_step_phases": {"forward_avg_launch_ms": round(fwd_ms, 5), "recompute_avg_launch_ms": round(rec_ms, 5),
                          "forward_frac": round(fwd_bytes / (fwd_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                          "recompute_frac": round(fwd_bytes / (rec_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)},
        "gradient_norms": {"drho_in": float(np.linalg.norm(g["drho_in"])), "dtau": float(g["dtau"][0])},
        "warm_vs_cold": None,
    }
    del s
    torch.cuda.empty_cache()
    if args.workload == "spheres" and not args.no_channel:
        print("[bench] 256^3 channel roofline ...", file=sys.stderr, flush=True)
        out["hbm_resident_roofline"] = channel_roofline(torch)
    if args.workload == "spheres" and not args.no_d2q9:
        print("[bench] D2Q9 grain-media batch ...", file=sys.stderr, flush=True)
        out["d2q9_batch"] = d2q9_batch(torch)
    if not args.no_copy:
        cp = copy_peak_gbs(torch)
        out["copy_peak_gbs"] = round(cp["copy16"], 1)
        out["copy_torch_gbs"] = round(cp["torch"], 1)
    if not args.no_warm:
        print("[bench] warm vs cold start ...", file=sys.stderr, flush=True)
        out["warm_vs_cold"] = warm_vs_cold(torch)
        # the warm start's network kernels (BF16 MFMA convolutions) against their roofline
        from paper_2310_00810_amd.unet import measure
        out["unet_mfma"] = []
        for m in (measure(2, 16, 256), measure(3, 2, 64)):
            m["ops_shown"] = f"the 8 longest of {len(m['ops'])} operations of a training step"
            m["ops"] = m["ops"][:8]
            out["unet_mfma"].append(m)
    if not args.no_cpu:
        print("[bench] cpu baseline (oracle) ...", file=sys.stderr, flush=True)
        cold = None
        try:
            cold = out["warm_vs_cold"]["2d"]["training_run_evaluation"]["cold_steps_median"]
        except (TypeError, KeyError):
            pass
        out["cpu_baseline"] = cpu_baseline(w, cold)
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
