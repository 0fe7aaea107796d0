import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long-running check")


def pytest_collection_modifyitems(config, items):
    try:
        import torch
        have_gpu = torch.cuda.is_available()
    except Exception:
        have_gpu = False
    if have_gpu:
        return
    skip = pytest.mark.skip(reason="no GPU in this environment")
    for it in items:
        if "gpu" in it.keywords:
            it.add_marker(skip)


@pytest.fixture(scope="session")
def oracle_mod():
    import oracle
    oracle.lib()
    return oracle


def tiny_lattices():
    """Small lattices that exercise every boundary kind: Zou-He faces, walls,
    periodic axes, grain nodes next to the faces and in the interior."""
    import oracle as O
    out = []
    s2 = np.zeros((1, 6, 8), np.uint8)
    s2[0, 2, 3] = 1
    s2[0, 3, 4] = 1
    s2[0, 0, 1] = 1           # grain node touching the wall, next to the inlet
    out.append(("d2q9_wall_grains", O.Lattice(9, 8, 6, 1, (O.BC_PRESSURE, O.BC_WALL, O.BC_PERIODIC), s2)))
    s2p = np.zeros((1, 5, 7), np.uint8)
    s2p[0, 1, 2] = 1
    s2p[0, 4, 0] = 1          # solid node on the inlet face
    out.append(("d2q9_periodic_y", O.Lattice(9, 7, 5, 1, (O.BC_PRESSURE, O.BC_PERIODIC, O.BC_PERIODIC), s2p)))
    s3 = np.zeros((4, 5, 6), np.uint8)
    s3[1, 2, 2] = 1
    s3[2, 2, 3] = 1
    s3[0, 4, 5] = 1           # solid node on the outlet face
    out.append(("d3q19_periodic_yz", O.Lattice(19, 6, 5, 4, (O.BC_PRESSURE, O.BC_PERIODIC, O.BC_PERIODIC), s3)))
    s3w = np.zeros((4, 5, 6), np.uint8)
    s3w[2, 1, 3] = 1
    out.append(("d3q19_wall_y", O.Lattice(19, 6, 5, 4, (O.BC_PRESSURE, O.BC_WALL, O.BC_PERIODIC), s3w)))
    s3ww = np.zeros((3, 4, 5), np.uint8)
    s3ww[1, 1, 2] = 1
    out.append(("d3q19_wall_yz", O.Lattice(19, 5, 4, 3, (O.BC_PRESSURE, O.BC_WALL, O.BC_WALL), s3ww)))
    return out


def multi_tile_lattices():
    """Lattices of many 256-node fluid tiles: random solids (isolated fluid
    nodes, grains on the faces), rows wider than a block's staged
    neighbourhood (D2Q9 16384 wide), very sparse boxes whose tiles span many
    rows (both read their neighbours' row words from global memory), x and y
    wrap-around, and a one-plane periodic D3Q19 box."""
    import oracle as O
    rng = np.random.default_rng(77)
    out = []

    def rand(shape, frac, clear_inlet=False):
        s = (rng.random(shape) < frac).astype(np.uint8)
        if clear_inlet:
            s[:, :, 0] = 0
        return s

    out.append(("d2q9_wide_rows", O.Lattice(9, 16384, 4, 1, (O.BC_PRESSURE, O.BC_PERIODIC, O.BC_PERIODIC),
                                            rand((1, 4, 16384), 0.4))))
    out.append(("d2q9_periodic_x", O.Lattice(9, 300, 40, 1, (O.BC_PERIODIC, O.BC_WALL, O.BC_PERIODIC),
                                             rand((1, 40, 300), 0.4))))
    out.append(("d3q19_sparse", O.Lattice(19, 200, 16, 16, (O.BC_PRESSURE, O.BC_PERIODIC, O.BC_PERIODIC),
                                          rand((16, 16, 200), 0.9))))
    out.append(("d3q19_wide_rows", O.Lattice(19, 4096, 4, 3, (O.BC_PRESSURE, O.BC_PERIODIC, O.BC_PERIODIC),
                                             rand((3, 4, 4096), 0.5))))
    out.append(("d3q19_walls", O.Lattice(19, 40, 24, 20, (O.BC_PRESSURE, O.BC_WALL, O.BC_PERIODIC),
                                         rand((20, 24, 40), 0.5))))
    out.append(("d3q19_one_plane", O.Lattice(19, 70, 30, 1, (O.BC_PRESSURE, O.BC_PERIODIC, O.BC_PERIODIC),
                                             rand((1, 30, 70), 0.3))))
    return out


def abb_lattices():
    """The tiny lattices with anti-bounce-back density faces on x."""
    import oracle as O
    out = []
    for name, lat in tiny_lattices():
        bc = (O.BC_ABB,) + tuple(lat.bc_tuple[1:])
        out.append((name.replace("d2q9", "abb_d2q9").replace("d3q19", "abb_d3q19"),
                    O.Lattice(lat.q, lat.nx, lat.ny, lat.nz, bc, lat.solid.copy())))
    return out


def mrt_velocity_lattices():
    """D2Q9 lattices with the multiple-relaxation-time collision and / or the
    Zou-He velocity inlet (grains at the faces, walls, periodic y), and a
    many-tile MRT lattice."""
    import oracle as O
    out = []
    tiny = [(n, l) for n, l in tiny_lattices() if l.q == 9]
    for name, lat in tiny:
        for bcx, mrt, tag in ((O.BC_PRESSURE, O.MRT_RATES, "mrt"), (O.BC_VELOCITY, None, "vel"),
                              (O.BC_VELOCITY, O.MRT_RATES, "mrt_vel")):
            out.append((f"{tag}_{name}", O.Lattice(9, lat.nx, lat.ny, 1, (bcx,) + tuple(lat.bc_tuple[1:]),
                                                   lat.solid.copy(), mrt=mrt)))
    rng = np.random.default_rng(78)
    s = (rng.random((1, 40, 300)) < 0.4).astype(np.uint8)
    s[:, :, 0] = 0
    out.append(("mrt_vel_multi_tile", O.Lattice(9, 300, 40, 1, (O.BC_VELOCITY, O.BC_WALL, O.BC_PERIODIC), s,
                                                mrt=O.MRT_RATES)))
    return out
