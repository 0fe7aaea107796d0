"""Host logic of the warm start's data augmentation (CPU)."""
import pytest

torch = pytest.importorskip("torch")


def _batch(dims, seed=0):
    g = torch.Generator().manual_seed(seed)
    n, d, h, w = 2, (1 if dims == 2 else 3), 5, 6
    x = torch.rand((n, d, h, w, 8), generator=g).to(torch.bfloat16)
    x[..., 1] = torch.linspace(0, 1, w).to(torch.bfloat16)
    wp = (torch.rand((n, d, h, w), generator=g) > 0.3).float()
    tg = torch.randn((n, d, h, w, 1 + dims), generator=g) * wp[..., None]
    return x, tg, wp


@pytest.mark.parametrize("dims", [2, 3])
def test_reversed_flow_is_an_involution_and_keeps_the_position_channel(dims):
    from paper_2310_00810_amd.warmstart import reversed_flow
    x, tg, wp = _batch(dims)
    s0 = 0.7
    x1, t1, w1 = reversed_flow(x, tg, wp, s0)
    assert torch.equal(x1[..., 1], x[..., 1])
    assert torch.equal(x1[..., 0], x[..., 0].flip(3))
    x2, t2, w2 = reversed_flow(x1, t1, w1, s0)
    assert torch.equal(x2, x) and torch.equal(w2, wp)
    assert torch.allclose(t2, tg, atol=1e-6)


@pytest.mark.parametrize("dims", [2, 3])
def test_reversed_flow_maps_each_channel(dims):
    """Density: 1 - t0 (in standardised units 1/s0 - t0) at fluid pixels and
    0 at solid ones; streamwise velocity kept; transverse velocities negated;
    all reflected in x."""
    from paper_2310_00810_amd.warmstart import reversed_flow
    x, tg, wp = _batch(dims, seed=3)
    s0 = 0.5
    _, t1, w1 = reversed_flow(x, tg, wp, s0)
    rf = lambda a: a.flip(3)
    assert torch.allclose(t1[..., 0], rf(wp) / s0 - rf(tg[..., 0]), atol=1e-6)
    assert torch.all(t1[..., 0][rf(wp) == 0] == 0)
    assert torch.equal(t1[..., 1], rf(tg[..., 1]))
    for a in range(2, 1 + dims):
        assert torch.equal(t1[..., a], -rf(tg[..., a]))
    assert torch.equal(w1, rf(wp))


def test_summary_compares_only_cases_where_both_starts_converge():
    """Speed-ups, medians and the faster fraction are taken over the cases
    where both starts reach the threshold; the converged counts cover all."""
    from paper_2310_00810_amd.warmstart import summarize
    res = [dict(cold_steps=1000, cold_s=1.0, warm_steps=500, warm_s=0.5, net_rel_l2_u=0.2, warm_cold_rel_l2=1e-3,
                cold_r=5e-7, warm_r=8e-7),
           dict(cold_steps=3000, cold_s=3.0, warm_steps=3000, warm_s=3.5, net_rel_l2_u=0.6, warm_cold_rel_l2=2e-3,
                cold_r=9e-7, warm_r=9e-7),
           dict(cold_steps=100000, cold_s=90.0, warm_steps=800, warm_s=0.8, net_rel_l2_u=1.0, warm_cold_rel_l2=5e-2,
                cold_r=3e-6, warm_r=9e-7)]                     # cold start stopped at the cap: left out
    s = summarize(res, 1e-6)
    assert (s["cold_converged"], s["warm_converged"], s["both_converged"]) == (2, 3, 2)
    assert s["speedup_median"] == pytest.approx((2.0 + 3.0 / 3.5) / 2)
    assert s["speedup_mean"] == pytest.approx((2.0 + 3.0 / 3.5) / 2)
    assert s["warm_faster_fraction"] == 0.5
    assert (s["cold_steps_median"], s["warm_steps_median"]) == (2000.0, 1750.0)
    assert s["net_rel_l2_u_median"] == pytest.approx(0.6) and s["net_rel_l2_u_mean"] == pytest.approx(0.6)
    assert s["warm_cold_rel_l2_max"] == pytest.approx(2e-3)


def test_periodic_axes_follow_the_boundary_kinds():
    from paper_2310_00810_amd.warmstart import bc_of, periodic_axes
    assert bc_of(2)[1] == "wall" and periodic_axes(2) == (0,)       # 2D: z (length 1) only
    assert periodic_axes(3) == (1, 0)                                # 3D: y and z
