"""Porous-media post-processing and parameterisation helpers, pinned to the
numbers the paper prints and to library routines (no GPU)."""
import numpy as np
import pytest

from paper_2310_00810_amd import geometry as G
from paper_2310_00810_amd import inverse as I


def test_carman_kozeny_on_the_2d_packing():
    # Eq. 8 with the 2D packing of Section 3.2: D_p = 1.18 mm, porosity 0.489,
    # Phi_CK = 180, sphericity 1.  Table 1 lists 3.47e-9 m^2 (the text's
    # 3.164e-9 does not follow from these inputs).
    k = I.carman_kozeny(0.489, 1.18e-3)
    assert k == pytest.approx(3.464e-9, rel=2e-4)
    assert k == pytest.approx(3.47e-9, rel=3e-3)
    # sphericity enters squared, the Kozeny factor inversely
    assert I.carman_kozeny(0.489, 1.18e-3, phi_s=0.5) == pytest.approx(k / 4)
    assert I.carman_kozeny(0.489, 1.18e-3, phi_ck=90.0) == pytest.approx(2 * k)


def test_kozeny_factor_from_tortuosity():
    # Section 3.3: Phi = 90 for spheres and L_e / L = 1.44 give Phi_CK = 186.63 (printed, rounded)
    assert I.kozeny_factor(1.44) == pytest.approx(186.63, abs=0.01)
    assert I.kozeny_factor(1.0) == 90.0


def test_reynolds_number_worked_example():
    # Eq. 11: U = 3.88e-3 lu/ts, D = 200 lu, nu = 0.167 lu^2/ts gives 2.33 (printed to two
    # decimals); the same flow in physical units: 2.33e-4 m/s, 0.02 m, 1e-6 m^2/s
    assert I.reynolds(3.88e-3, 200.0, 0.167) == pytest.approx(2.33, abs=0.01)
    assert I.reynolds(2.33e-4, 0.02, 1e-6) == pytest.approx(2.33, rel=1e-12)


def test_unit_conversions():
    # Section 3.2: k_LBM = 0.317 lu^2 at 1e-4 m per lu is 3.17e-9 m^2
    assert I.physical_permeability(0.317, 1e-4) == pytest.approx(3.17e-9, rel=1e-12)
    # matching nu_LBM = 0.167 to water (1e-6 m^2/s) at 1e-4 m per lu: 1 ts = 1.67e-3 s
    assert I.lattice_time_step(0.167, 1e-4) == pytest.approx(1.67e-3, rel=1e-12)
    assert I.viscosity(I.tau_from_viscosity(0.02)) == pytest.approx(0.02)


@pytest.mark.parametrize("n_nodes,n_knots", [(200, 8), (37, 2), (64, 5), (256, 16)])
def test_spline_basis_is_the_natural_cubic_spline(n_nodes, n_knots):
    from scipy.interpolate import CubicSpline
    B = I.spline_basis(n_nodes, n_knots)
    xk = np.linspace(0, n_nodes - 1, n_knots)
    rng = np.random.default_rng(n_nodes + n_knots)
    v = rng.standard_normal(n_knots)
    ref = CubicSpline(xk, v, bc_type="natural")(np.arange(n_nodes))
    assert np.allclose(B @ v, ref, rtol=0, atol=1e-12 * max(1.0, np.abs(v).max()))


def test_spline_basis_properties():
    B = I.spline_basis(200, 8)
    xk = np.linspace(0, 199, 8)
    # interpolates the knots; reproduces constants and straight lines exactly
    on = np.isclose(np.arange(200)[:, None], xk[None]).any(axis=1)
    v = np.random.default_rng(3).standard_normal(8)
    assert np.allclose((B @ v)[on], v[np.isin(np.round(xk), np.arange(200)[on])], atol=1e-12)
    assert np.allclose(B.sum(axis=1), 1.0, atol=1e-12)
    assert np.allclose(B @ (2.0 + 0.5 * xk), 2.0 + 0.5 * np.arange(200), atol=1e-10)
    # the knot gradient is the transpose: <B v, g> = <v, B^T g>
    g = np.random.default_rng(4).standard_normal(200)
    assert np.dot(B @ v, g) == pytest.approx(np.dot(v, B.T @ g), rel=1e-12)


def test_hydrodynamic_radius_opens_the_packing():
    # same placements (the porosity target is met with the full radius R); the mask painted
    # at 0.9 R is a strict subset of the one painted at R
    full = G.boolean_disks(200, 200, (5.0, 7.0), 0.49, seed=7)
    hydro = G.boolean_disks(200, 200, (5.0, 7.0), 0.49, seed=7, hydro=0.9)
    assert G.porosity(full) <= 0.49
    assert np.all(hydro <= full) and G.porosity(hydro) > G.porosity(full) + 0.03
    assert G.percolates(hydro)
    a = G.rsa_disks(128, 64, (4.0, 6.0), 0.7, seed=5)
    b = G.rsa_disks(128, 64, (4.0, 6.0), 0.7, seed=5, hydro=0.9)
    assert np.all(b <= a) and G.porosity(b) > G.porosity(a)


def test_hydrodynamic_disk_is_the_smaller_disk():
    # one grain: painting at hydro * R is painting a disk of radius hydro * R
    m = np.zeros((40, 40), np.uint8)
    G._paint_disk(m, 19.3, 20.1, 0.9 * 8.0)
    yy, xx = np.mgrid[0:40, 0:40]
    assert np.array_equal(m, ((xx - 19.3) ** 2 + (yy - 20.1) ** 2 <= (0.9 * 8.0) ** 2).astype(np.uint8))


def _bfs_flowing(solid, links, periodic):
    """Brute force: breadth-first search over the lattice links from every
    fluid node of the x = 0 face, and again from the x = nx-1 face."""
    from collections import deque
    fluid = solid == 0
    shape = fluid.shape

    def reach(face):
        seen = np.zeros(shape, bool)
        dq = deque()
        for idx in zip(*np.nonzero(fluid)):
            if idx[-1] == face:
                seen[idx] = True
                dq.append(idx)
        while dq:
            p = dq.popleft()
            for c in links:
                q = []
                for a, (pa, ca) in enumerate(zip(p, c)):
                    v = pa + ca
                    if a in periodic:
                        v %= shape[a]
                    elif not 0 <= v < shape[a]:
                        break
                    q.append(v)
                else:
                    q = tuple(q)
                    if fluid[q] and not seen[q]:
                        seen[q] = True
                        dq.append(q)
        return seen

    return reach(0) & reach(shape[-1] - 1)


D2Q9_LINKS = [(a, b) for a in (-1, 0, 1) for b in (-1, 0, 1) if (a, b) != (0, 0)]
D3Q19_LINKS = [(a, b, c) for a in (-1, 0, 1) for b in (-1, 0, 1) for c in (-1, 0, 1)
               if 0 < abs(a) + abs(b) + abs(c) <= 2]


def test_flowing_takes_diagonal_links_in_2d_and_edge_links_only_in_3d():
    s = np.ones((4, 6), np.uint8)
    s[1, 0:3] = 0
    s[2, 3:6] = 0               # joined to row 1 only through the diagonal (1,2)-(2,3)
    s[3, 0] = 0                 # a pocket on the inlet face
    f = G.flowing(s)
    assert f[1, 0:3].all() and f[2, 3:6].all() and not f[3, 0] and f.sum() == 6
    v = np.ones((3, 3, 6), np.uint8)
    v[0, 0, 0:3] = 0
    v[1, 1, 3:6] = 0            # a vertex contact only: no D3Q19 link
    assert not G.flowing(v).any()
    v[1, 0, 3] = 0              # an edge contact (0,0,2)-(1,0,3)
    assert G.flowing(v)[1, 1, 3:6].all()


def test_flowing_crosses_periodic_axes():
    v = np.ones((3, 4, 6), np.uint8)
    v[0, 0, 0:3] = 0
    v[0, 3, 3:6] = 0            # joined to the first run only across y = 3 -> 0
    v[0, 3, 2] = 1
    assert not G.flowing(v).any()
    f = G.flowing(v, periodic=(1,))
    assert f[0, 0, 0:3].all() and f[0, 3, 3:6].all()


@pytest.mark.parametrize("dims", [2, 3])
def test_flowing_matches_a_breadth_first_search(dims):
    rng = np.random.default_rng(5)
    for trial in range(12):
        if dims == 2:
            s = (rng.random((9, 13)) < 0.45).astype(np.uint8)
            per = {0} if trial % 2 else set()
            links = D2Q9_LINKS
        else:
            s = (rng.random((5, 6, 9)) < 0.72).astype(np.uint8)
            per = [set(), {0}, {1}, {0, 1}][trial % 4]
            links = D3Q19_LINKS
        got = G.flowing(s, periodic=tuple(per))
        assert np.array_equal(got, _bfs_flowing(s, links, per)), (dims, trial)
    s2 = (rng.random((1, 9, 13)) < 0.45).astype(np.uint8)
    assert np.array_equal(G.flowing(s2)[0], _bfs_flowing(s2[0], D2Q9_LINKS, set()))
