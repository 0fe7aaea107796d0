"""Writes the FP64 oracle's results for the workloads at their stated step
counts, for the GPU parity tests (``tests/test_gpu_goldens.py``).

CPU only.  It imports the oracle and the seeded input recipes
(``paper_2310_00810_amd.geometry``, which holds no lattice Boltzmann
arithmetic) and nothing of the GPU path.  Every stored input is FP32 (the
precision the GPU side receives it in) and is handed to the oracle as that
FP32 value widened to FP64.

    python tests/golden/make_goldens.py c2 c4 c3_64 c3_128     # one .npz per case

Cases (the oracle's gradient is the same for every checkpoint interval, so it
uses whichever interval fits the host's memory):

* ``c2``: the 512 x 256 granular channel (RSA disks r ~ U[6, 14], porosity
  0.70, seed 2, walls in y), tau 0.9, T = 10 000.  Target = the velocity after
  T steps at rho_in - 1 = 0.004 (the inverse problem's truth); the loss
  (VEC, SUM), its three gradients and the velocity at the half-way guess
  rho_in - 1 = 0.002.
* ``c3_64``: the 3D sphere box recipe (Boolean spheres r ~ U[6, 10], porosity
  0.40, seed 3, periodic y and z, 4-node sphere-free buffers) on a 64^3
  lattice, inlet profile 0.004 phi (8 Fourier modes, seed 33), tau 0.75,
  T = 8000.  Target = the velocity after T steps at the truth; the loss
  (VEC, MEAN_FLUID), dL/drho_in at every inlet node, dL/dtau, dL/drho_out
  and the velocity at 20 000 sampled fluid nodes, at the initial guess
  rho_in - 1 = 0.002, tau = 1.0.
* ``c3_128``: the same recipe on the full 128^3 lattice at the truth,
  T = 8000: the velocity at 20 000 sampled fluid nodes.
* ``c4``: the batch of 64 uneven channels (``geometry.c4_media``) from rest,
  T = 5000: for every 128 x 64 and 256 x 128 medium and the first two of
  each larger size, the loss (VEC, SUM, N(0, 1e-4) targets), its three
  gradients and the velocity at up to 4096 sampled fluid nodes.
"""
import hashlib
import os
import sys
import tempfile
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
from oracle import build as oracle_build  # noqa: E402
from paper_2310_00810_amd import geometry as G  # noqa: E402

WALLS = (O.BC_PRESSURE, O.BC_WALL, O.BC_PERIODIC)
BOX = (O.BC_PRESSURE, O.BC_PERIODIC, O.BC_PERIODIC)
SAMPLE_SEED = 12345


def f32(x):
    return np.asarray(x, np.float32).astype(np.float64)


def oracle_hash():
    h = hashlib.sha256()
    for name in ("lbm_oracle.c", "lbm_oracle_core.h"):
        with open(os.path.join(ROOT, "oracle", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def log(msg):
    print(f"[{time.strftime('%H:%M:%S')}] {msg}", flush=True)


def velocity(lat, f):
    return O.macro(lat, f)[1][..., :lat_dims(lat)]


def lat_dims(lat):
    return 2 if lat.q == 9 else 3


def sample(lat, k, seed=SAMPLE_SEED):
    """Sorted flat indices of min(k, fluid) fluid nodes, drawn without replacement."""
    fl = np.flatnonzero(lat.fluid().ravel())
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(fl, size=min(k, fl.size), replace=False))


def pad3(u):
    out = np.zeros(u.shape[:-1] + (3,))
    out[..., :u.shape[-1]] = u
    return out


def save(name, **arrays):
    path = os.path.join(HERE, name + ".npz")
    np.savez_compressed(path, oracle_sha=np.array(oracle_hash()), **arrays)
    log(f"wrote {path} ({os.path.getsize(path) / 1e6:.2f} MB)")


def case_c2():
    nx, ny, tau, T = 512, 256, 0.9, 10000
    d_true, d_eval = f32(0.004), f32(0.002)
    solid = G.rsa_disks(nx, ny, (6.0, 14.0), 0.70, seed=2)[None]
    lat = O.Lattice(9, nx, ny, 1, WALLS, solid)
    f0 = O.init_eq(lat, 1.0, 0.0)
    log("c2: target run")
    target = velocity(lat, O.run(lat, tau, 1.0 + d_true, 1.0, f0, T)).astype(np.float32)
    log("c2: velocity at the guess")
    u_eval = velocity(lat, O.run(lat, tau, 1.0 + d_eval, 1.0, f0, T))
    log("c2: gradient at the guess")
    g = O.grad(lat, tau, 1.0 + d_eval, 1.0, f0, T, pad3(target.astype(np.float64)), K=100)
    save("c2", T=T, tau=tau, drho_true=d_true, drho_eval=d_eval, target=target,
         u_eval=u_eval.astype(np.float32), loss=g["loss"], drho_in=g["drho_in"].sum(), dtau=g["dtau"],
         drho_out=g["drho_out"].sum())


def c3_lattice(n):
    solid = G.boolean_spheres((n, n, n), (6.0, 10.0), 0.40, seed=3, periodic=(False, True, True), x_margin=4)
    prof = f32(0.004 * G.fourier_profile(n, n, n_modes=8, seed=33))
    return solid, prof, O.Lattice(19, n, n, n, BOX, solid)


def case_c3_64():
    n, T, tau_true, tau_eval = 64, 8000, 0.75, 1.0
    d_eval = f32(0.002)
    solid, prof, lat = c3_lattice(n)
    f0 = O.init_eq(lat, 1.0, 0.0)
    nfl = int(lat.fluid().sum())
    log(f"c3_64: {nfl} fluid nodes; target run")
    target = velocity(lat, O.run(lat, tau_true, 1.0 + prof, 1.0, f0, T)).astype(np.float32)
    idx = sample(lat, 20000)
    log("c3_64: velocity at the guess")
    u_eval = velocity(lat, O.run(lat, tau_eval, 1.0 + d_eval, 1.0, f0, T)).reshape(-1, 3)[idx]
    log("c3_64: gradient at the guess")
    g = O.grad(lat, tau_eval, 1.0 + d_eval, 1.0, f0, T, pad3(target.astype(np.float64)), scale=1.0 / nfl, K=100)
    save("c3_64", n=n, T=T, tau_true=tau_true, tau_eval=tau_eval, drho_eval=d_eval, profile=prof.astype(np.float32),
         target=target, idx=idx, u_eval=u_eval, loss=g["loss"], drho_in=g["drho_in"], dtau=g["dtau"],
         drho_out=g["drho_out"].sum())


def case_c3_128():
    n, T, tau = 128, 8000, 0.75
    solid, prof, lat = c3_lattice(n)
    f0 = O.init_eq(lat, 1.0, 0.0)
    log(f"c3_128: {int(lat.fluid().sum())} fluid nodes; run at the truth")
    idx = sample(lat, 20000)
    u = velocity(lat, O.run(lat, tau, 1.0 + prof, 1.0, f0, T)).reshape(-1, 3)[idx]
    save("c3_128", n=n, T=T, tau=tau, idx=idx, u=u)


def c4_selection(media):
    """Every 128 x 64 and 256 x 128 medium and the first two of each larger size."""
    pick, seen = [], {}
    for b, m in enumerate(media):
        size = (m["nx"], m["ny"])
        seen[size] = seen.get(size, 0) + 1
        if size in ((128, 64), (256, 128)) or seen[size] <= 2:
            pick.append(b)
    return pick


def case_c4():
    T, K = 5000, 71
    media = G.c4_media(64)
    pick = c4_selection(media)
    log(f"c4: {len(pick)} media of 64: {pick}")
    res = dict(loss=[], drho_in=[], dtau=[], drho_out=[], idx=[], u=[], n_idx=[])
    for b in pick:
        m = media[b]
        lat = O.Lattice(9, m["nx"], m["ny"], 1, WALLS, m["solid"])
        f0 = O.init_eq(lat, 1.0, 0.0)
        rin = 1.0 + f32(m["drho_in"])
        tau = float(m["tau"])
        idx = sample(lat, 4096, seed=SAMPLE_SEED + b)
        u = velocity(lat, O.run(lat, tau, rin, 1.0, f0, T)).reshape(-1, 2)[idx]
        g = O.grad(lat, tau, rin, 1.0, f0, T, pad3(m["target"][None].astype(np.float64)), K=K)
        for k, v in (("loss", g["loss"]), ("drho_in", g["drho_in"].sum()), ("dtau", g["dtau"]),
                     ("drho_out", g["drho_out"].sum())):
            res[k].append(v)
        res["idx"].append(np.pad(idx, (0, 4096 - idx.size), constant_values=-1))
        res["u"].append(np.pad(u, ((0, 4096 - idx.size), (0, 0))))
        res["n_idx"].append(idx.size)
        log(f"c4: medium {b} ({m['nx']}x{m['ny']}) loss {g['loss']:.6e}")
    save("c4", T=T, K=K, media=np.array(pick), **{k: np.array(v) for k, v in res.items()})


CASES = {"c2": case_c2, "c3_64": case_c3_64, "c3_128": case_c3_128, "c4": case_c4}


def main(argv):
    names = argv or list(CASES)
    with tempfile.TemporaryDirectory() as tmp:
        O.load(oracle_build.build(out=os.path.join(tmp, "liblbm_oracle_native.so"), native=True))
        for name in names:
            t0 = time.perf_counter()
            CASES[name]()
            log(f"{name}: {time.perf_counter() - t0:.0f} s")


if __name__ == "__main__":
    main(sys.argv[1:])
