"""Seeded synthetic inputs: grain packings, inlet profiles, test states.

This module holds input generation only -- none of the lattice Boltzmann
arithmetic.  Both the GPU path and the CPU oracle consume what it produces,
as plain arrays.

Stand-ins for the paper's data: the paper's 2D packings and its CT scan of
Hamburg sand (Section 3.3) are not available, so packings of the same kind
are drawn here from explicit, seeded recipes:

* ``rsa_disks``: non-overlapping circular grains by random sequential
  addition, a throat of at least ``gap`` nodes between grains, kept clear of
  ``x_margin`` nodes at the inlet and outlet faces (2D media, Section 3.1.1);
* ``boolean_spheres``: overlapping spheres (Boolean model), periodic on the
  chosen axes, for porosities below the jamming limit of hard spheres (3D
  media, Section 3.3);
* ``fourier_profile``: a smooth per-node inlet field built from a handful of
  Fourier modes (a smooth non-uniform inlet pressure, Section 3.1.2);
* ``c4_media``: the batch of 64 uneven granular channels (sizes, packings,
  relaxation times, inlet densities and target velocities, all seeded).

A node is solid iff its squared distance to a grain centre is at most r^2.
"""
from __future__ import annotations

import numpy as np

try:
    from scipy import ndimage as _ndi
except Exception:  # pragma: no cover - scipy is present in this image
    _ndi = None


def porosity(solid: np.ndarray) -> float:
    return float(1.0 - np.count_nonzero(solid) / solid.size)


def percolates(solid: np.ndarray) -> bool:
    """True if fluid nodes of the x = 0 face connect to fluid nodes of the
    x = nx-1 face through face-adjacent fluid nodes (x is the last axis)."""
    fluid = solid == 0
    if _ndi is not None:
        lab, _ = _ndi.label(fluid)
        a = set(np.unique(lab[..., 0])) - {0}
        b = set(np.unique(lab[..., -1])) - {0}
        return bool(a & b)
    # plain BFS fallback
    from collections import deque
    seen = np.zeros_like(fluid)
    dq = deque()
    for idx in zip(*np.nonzero(fluid[..., 0])):
        full = tuple(idx) + (0,)
        seen[full] = True
        dq.append(full)
    nd = fluid.ndim
    while dq:
        p = dq.popleft()
        if p[-1] == fluid.shape[-1] - 1:
            return True
        for a in range(nd):
            for d in (-1, 1):
                q = list(p)
                q[a] += d
                if 0 <= q[a] < fluid.shape[a]:
                    q = tuple(q)
                    if fluid[q] and not seen[q]:
                        seen[q] = True
                        dq.append(q)
    return False


def flowing(solid: np.ndarray, periodic=()) -> np.ndarray:
    """Fluid nodes joined to both the x = 0 and the x = nx-1 face through
    lattice links (x is the last axis): face and diagonal neighbours in 2D
    (D2Q9), face and edge neighbours in 3D (D3Q19), also across the axes
    listed in `periodic` (axis numbers of `solid`).  The rest of the pore
    space is closed pockets, which no pressure drop moves.  A leading axis of
    length 1 is taken as 2D."""
    from scipy.sparse import coo_matrix
    from scipy.sparse.csgraph import connected_components
    solid = np.asarray(solid)
    squeeze = solid.ndim == 3 and solid.shape[0] == 1
    s2 = solid[0] if squeeze else solid
    per = {a - 1 for a in periodic if a >= 1} if squeeze else set(periodic)
    nd = s2.ndim
    fluid = s2 == 0
    struct = _ndi.generate_binary_structure(nd, nd if nd == 2 else 2)
    lab, n = _ndi.label(fluid, structure=struct)
    edges = []
    offs = [np.array(o) - 1 for o in np.argwhere(struct)]
    for a in per:
        src = np.take(lab, -1, axis=a)
        dst = np.take(lab, 0, axis=a)
        rest = [b for b in range(nd) if b != a]
        for o in offs:
            if o[a] != 1:
                continue
            sh, ok = dst, np.ones(src.shape, bool)
            for i, b in enumerate(rest):
                if o[b] == 0:
                    continue
                sh = np.roll(sh, -o[b], axis=i)
                if b not in per:
                    idx = [slice(None)] * len(rest)
                    idx[i] = slice(-1, None) if o[b] > 0 else slice(0, 1)
                    ok[tuple(idx)] = False
            m = ok & (src > 0) & (sh > 0)
            edges.append(np.stack([src[m], sh[m]]))
    e = np.concatenate(edges, axis=1) if edges else np.zeros((2, 0), int)
    g = coo_matrix((np.ones(e.shape[1]), (e[0], e[1])), shape=(n + 1, n + 1))
    ncomp, comp = connected_components(g, directed=False)
    comp = comp.copy()
    comp[0] = -1                                       # label 0: solid
    cl = comp[lab]
    ends = (set(np.unique(cl[..., 0])) & set(np.unique(cl[..., -1]))) - {-1}
    keep = np.zeros(ncomp + 1, bool)                   # index -1: the solid entry
    keep[list(ends)] = True
    out = keep[cl] & fluid
    return out[None] if squeeze else out


def _paint_disk(solid, cx, cy, r):
    ny, nx = solid.shape
    x0, x1 = max(int(np.floor(cx - r)), 0), min(int(np.ceil(cx + r)), nx - 1)
    y0, y1 = max(int(np.floor(cy - r)), 0), min(int(np.ceil(cy + r)), ny - 1)
    if x1 < x0 or y1 < y0:
        return
    yy, xx = np.mgrid[y0:y1 + 1, x0:x1 + 1]
    m = (xx - cx) ** 2 + (yy - cy) ** 2 <= r * r
    solid[y0:y1 + 1, x0:x1 + 1] |= m.astype(np.uint8)


def rsa_disks(nx: int, ny: int, r_range=(6.0, 14.0), target_porosity=0.7, seed=0,
              x_margin=4, gap=2.0, max_reject=100_000, max_reseed=20, batch=512, hydro=1.0):
    """2D solid mask (ny, nx) uint8 of non-overlapping disks.

    Disks are drawn with radius ~ U[r_range] and a real-valued centre such
    that the disk lies inside y in [0, ny-1] and x in [x_margin,
    nx-1-x_margin]; a candidate is rejected if its centre distance to any
    placed disk is below r1 + r2 + gap.  Disks are added until the porosity
    is at most target_porosity.  After max_reject consecutive rejections the
    non-overlap rule is dropped (overlapping placement).  Candidates are drawn
    in batches and the first acceptable one of a batch is placed (the others
    are discarded), which is random sequential addition with a different use
    of the random stream.  The mask must let fluid percolate from inlet to
    outlet; otherwise the next seed of the stream is used.

    hydro < 1: the grains are placed (and the porosity target is met) with
    their radius R, but the returned mask paints them with the hydrodynamic
    radius hydro * R (Section 3.1.2 uses 0.9 R), which opens the contacts
    that would close the 2D pore space."""
    rng = np.random.default_rng(seed)
    for _ in range(max_reseed):
        solid = np.zeros((ny, nx), np.uint8)
        hsolid = solid if hydro == 1.0 else np.zeros((ny, nx), np.uint8)
        placed = np.zeros((0, 3))
        rejects = 0
        overlap_ok = False
        while porosity(solid) > target_porosity:
            r = rng.uniform(r_range[0], r_range[1], batch)
            lo_x, hi_x = x_margin + r, nx - 1 - x_margin - r
            lo_y, hi_y = r, ny - 1 - r
            if np.any(hi_x < lo_x) or np.any(hi_y < lo_y):
                raise ValueError("lattice too small for the grain radius")
            cx = lo_x + (hi_x - lo_x) * rng.uniform(size=batch)
            cy = lo_y + (hi_y - lo_y) * rng.uniform(size=batch)
            if overlap_ok or placed.shape[0] == 0:
                j = 0
            else:
                d2 = (placed[:, 0, None] - cx[None]) ** 2 + (placed[:, 1, None] - cy[None]) ** 2
                ok = ~np.any(d2 < (placed[:, 2, None] + r[None] + gap) ** 2, axis=0)
                if not ok.any():
                    rejects += batch
                    if rejects >= max_reject:
                        overlap_ok = True
                    continue
                j = int(np.argmax(ok))
                rejects = 0 if j == 0 else rejects + j
            placed = np.vstack([placed, [cx[j], cy[j], r[j]]])
            _paint_disk(solid, cx[j], cy[j], r[j])
            if hsolid is not solid:
                _paint_disk(hsolid, cx[j], cy[j], hydro * r[j])
        if percolates(hsolid):
            return hsolid
    raise RuntimeError("no percolating packing found")


def boolean_spheres(n, r_range=(6.0, 10.0), target_porosity=0.4, seed=0,
                    periodic=(False, True, True), x_margin=4, max_reseed=20):
    """3D solid mask (nz, ny, nx) uint8 of overlapping spheres.

    n = (nx, ny, nz).  Centres are uniform with x in [x_margin + r,
    nx-1-x_margin-r] (sphere-free inlet/outlet buffers) and uniform over the
    whole extent of periodic axes (spheres wrap around).  Spheres are added
    until the porosity is at most target_porosity; the pore space must
    percolate from inlet to outlet."""
    nx, ny, nz = n
    rng = np.random.default_rng(seed)
    ext = (nx, ny, nz)
    for _ in range(max_reseed):
        solid = np.zeros((nz, ny, nx), np.uint8)
        while porosity(solid) > target_porosity:
            r = rng.uniform(*r_range)
            c = [rng.uniform(x_margin + r, nx - 1 - x_margin - r)]
            for a in (1, 2):
                c.append(rng.uniform(0, ext[a]) if periodic[a] else rng.uniform(r, ext[a] - 1 - r))
            _paint_sphere(solid, c, r, periodic)
        if percolates(solid):
            return solid
    raise RuntimeError("no percolating packing found")


def _paint_sphere(solid, c, r, periodic):
    nz, ny, nx = solid.shape
    ext = (nx, ny, nz)
    rng_ax = []
    for a in range(3):
        lo, hi = int(np.floor(c[a] - r)), int(np.ceil(c[a] + r))
        idx = np.arange(lo, hi + 1)
        d = idx - c[a]
        if periodic[a]:
            idx = np.mod(idx, ext[a])
        else:
            keep = (idx >= 0) & (idx < ext[a])
            idx, d = idx[keep], d[keep]
        rng_ax.append((idx, d))
    (ix, dx), (iy, dy), (iz, dz) = rng_ax
    d2 = dz[:, None, None] ** 2 + dy[None, :, None] ** 2 + dx[None, None, :] ** 2
    m = (d2 <= r * r).astype(np.uint8)
    solid[np.ix_(iz, iy, ix)] |= m


def boolean_disks(nx, ny, r_range=(6.0, 14.0), target_porosity=0.6, seed=0, periodic_y=False, x_margin=4,
                  max_reseed=20, hydro=1.0):
    """2D solid mask (ny, nx) uint8 of overlapping disks (Boolean model), for
    porosities below what non-overlapping placement reaches.  Centres have
    x in [x_margin + r, nx-1-x_margin-r] and y uniform (periodic_y) or inside
    [r, ny-1-r]; the pore space must percolate from inlet to outlet.
    hydro: as in rsa_disks (placement with R, mask painted with hydro * R)."""
    rng = np.random.default_rng(seed)
    for _ in range(max_reseed):
        solid = np.zeros((ny, nx), np.uint8)
        hsolid = solid if hydro == 1.0 else np.zeros((ny, nx), np.uint8)
        while porosity(solid) > target_porosity:
            r = rng.uniform(*r_range)
            cx = rng.uniform(x_margin + r, nx - 1 - x_margin - r)
            cy = rng.uniform(0, ny) if periodic_y else rng.uniform(r, ny - 1 - r)
            for sh in ((-ny, 0, ny) if periodic_y else (0,)):
                _paint_disk(solid, cx, cy + sh, r)
                if hsolid is not solid:
                    _paint_disk(hsolid, cx, cy + sh, hydro * r)
        if percolates(hsolid):
            return hsolid
    raise RuntimeError("no percolating packing found")


def fourier_profile(ny: int, nz: int, n_modes=8, seed=0, kmax=3):
    """Smooth field phi(z, y) in [0, 1] from n_modes Fourier modes:
    psi = sum_k a_k cos(2 pi (m_k y / ny + n_k z / nz) + theta_k) with
    (m_k, n_k) integers in [-kmax, kmax]^2 minus the origin, a_k ~ N(0, 1),
    theta_k ~ U[0, 2 pi); phi = (psi - min) / (max - min)."""
    rng = np.random.default_rng(seed)
    yy, zz = np.meshgrid(np.arange(ny), np.arange(nz), indexing="xy")
    psi = np.zeros((nz, ny))
    for _ in range(n_modes):
        while True:
            m, nn = rng.integers(-kmax, kmax + 1, size=2)
            if m != 0 or nn != 0:
                break
        a = rng.normal()
        th = rng.uniform(0, 2 * np.pi)
        psi += a * np.cos(2 * np.pi * (m * yy / ny + nn * zz / nz) + th)
    lo, hi = psi.min(), psi.max()
    return (psi - lo) / (hi - lo) if hi > lo else np.zeros_like(psi)


def random_perturbation(shape, q, amplitude, seed=0):
    """Seeded uniform perturbation in [-amplitude, amplitude] of shape
    shape + (q,) -- used as non-equilibrium test states (added to the
    lattice weights by the caller)."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-amplitude, amplitude, size=tuple(shape) + (q,))


def random_field(shape, scale, seed=0):
    rng = np.random.default_rng(seed)
    return rng.normal(0.0, scale, size=shape)


def obstructed_pipe(nx=300, ny=50, x_plate=80, plate_len=30):
    """2D pipe (walls in y) with a thin plate normal to the flow: one node
    wide at x = x_plate, plate_len nodes long, centred in y (Section 3.1.1's
    obstructed pipe; the plate's position in y is not stated there).
    Returns a (1, ny, nx) uint8 solid mask."""
    solid = np.zeros((1, ny, nx), np.uint8)
    y0 = (ny - plate_len) // 2
    solid[0, y0:y0 + plate_len, x_plate] = 1
    return solid


def cylinder_channel(nx=800, ny=320, diameter=20, xc=300, yc=160):
    """2D domain with one circular cylinder (Section 3.4's wake): a node is
    solid iff its distance to (xc, yc) is at most diameter / 2.  Returns a
    (1, ny, nx) uint8 solid mask."""
    yy, xx = np.mgrid[0:ny, 0:nx]
    return (((xx - xc) ** 2 + (yy - yc) ** 2) <= (diameter / 2) ** 2).astype(np.uint8)[None]


C4_SIZES = ((128, 64), (256, 128), (512, 256), (1024, 512))


def c4_media(n_inst=64):
    """The batch of uneven D2Q9 granular channels.  Medium b draws, from seed
    4000 + b, its size from C4_SIZES, a porosity U[0.5, 0.8] of RSA disks
    r ~ U[6, 14], tau U[0.6, 1.2] and rho_in - 1 U[0.001, 0.006]; its target
    velocity (ny, nx, 2) float32 is N(0, 1e-4), drawn in medium order from one
    generator seeded 4000.  Returns a list of dicts (nx, ny, solid (1, ny, nx),
    tau, drho_in, target)."""
    out = []
    rng = np.random.default_rng(4000)
    for b in range(n_inst):
        r = np.random.default_rng(4000 + b)
        nx, ny = C4_SIZES[r.integers(0, 4)]
        phi = r.uniform(0.5, 0.8)
        solid = rsa_disks(nx, ny, (6.0, 14.0), phi, seed=4000 + b, max_reject=20000)[None]
        tgt = (1e-4 * rng.standard_normal((ny, nx, 2))).astype(np.float32)
        out.append(dict(nx=nx, ny=ny, solid=solid, tau=r.uniform(0.6, 1.2), drho_in=r.uniform(0.001, 0.006),
                        target=tgt))
    return out
