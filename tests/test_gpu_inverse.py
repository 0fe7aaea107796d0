"""End-to-end inverse runs on the GPU: the optimiser driven by the adjoint
recovers the inlet density that generated the target flow."""
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def test_constant_head_recovery_channel():
    from paper_2310_00810_amd import run
    r = run.c1()
    assert abs(r["recovered_drho_in"] - 0.003) <= 1e-6
    assert r["loss"][-1] <= 1e-8 * r["loss"][0]


def test_constant_head_recovery_granular_media_and_darcy():
    from paper_2310_00810_amd import run
    r = run.c2(quick=True)
    assert abs(r["recovered_drho_in"] - 0.004) <= 4e-6
    assert r["darcy_k_lu2"] > 0


def test_batched_launch_matches_single_launches():
    from paper_2310_00810_amd import run
    r = run.c4(quick=True)
    assert r["gradients_bitwise_equal"]
