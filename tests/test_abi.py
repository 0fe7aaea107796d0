"""The C-ABI library loads, exports every symbol include/lbm.h declares, and
its host-side planning and validation behave (no GPU needed)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2310_00810_amd import _lib as C

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared(header):
    text = open(os.path.join(ROOT, "include", header)).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b((?:lbm|lbmnn)_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(C.LIBPATH):
        from paper_2310_00810_amd import build
        build.build()
    return C.lib()


def test_every_declared_symbol_is_exported(L):
    names = declared("lbm.h")
    assert len(names) >= 15
    for n in names:
        assert hasattr(L, n), n
    assert sorted(C.EXPORTS) == sorted(n for n in names if n.startswith("lbm_"))


def test_every_declared_network_symbol_is_exported(L):
    names = declared("lbmnn.h")
    assert sorted(C.NN_EXPORTS) == names
    C.nnlib()
    for n in names:
        assert hasattr(L, n), n


def test_conv_workspace_only_for_layers_with_few_output_tiles(L):
    """Host-side split choice of lbmnn_conv_ws (no GPU call): a 3x3x3 layer on
    2 x 8^3 pixels, 256 -> 256 channels, has 16 x 4 output tiles and a K loop of
    108 steps of 64: 16 splits of 7 steps, 16 x 1024 x 256 FP32 partials.  A
    2D layer on 16 x 256^2 pixels has 16 384 tiles and needs none; an invalid
    descriptor reports 0."""
    C.nnlib()
    fake_in, fake_out = 1 << 20, 1 << 21          # aligned stand-ins, never dereferenced on the host
    deep = C.lbmnn_conv_desc(2, 8, 8, 8, 3, 3, 256, 256, 0, fake_in, 256, 0, fake_out, None, 256, 0)
    assert L.lbmnn_conv_workspace_bytes(ctypes.byref(deep)) == 16 * 1024 * 256 * 4
    top = C.lbmnn_conv_desc(16, 1, 256, 256, 2, 3, 32, 32, 0, fake_in, 32, 0, fake_out, None, 32, 0)
    assert L.lbmnn_conv_workspace_bytes(ctypes.byref(top)) == 0
    bad = C.lbmnn_conv_desc(2, 8, 8, 8, 4, 3, 256, 256, 0, fake_in, 256, 0, fake_out, None, 256, 0)
    assert L.lbmnn_conv_workspace_bytes(ctypes.byref(bad)) == 0


def _problem(nx=64, ny=32, nz=1, q=9, steps=100, K=0, tape=0, solid=None, n=1, **kw):
    arr = (C.lbm_instance * n)()
    keep = []
    for k in range(n):
        arr[k].nx, arr[k].ny, arr[k].nz = nx, ny, nz
        if solid is not None:
            s = np.ascontiguousarray(solid, np.uint8)
            keep.append(s)
            arr[k].solid = s.ctypes.data_as(ctypes.c_void_p)
    p = C.lbm_problem(q, n, arr, kw.get("bcx", 0), kw.get("bcy", 2), kw.get("bcz", 1), steps, K, tape,
                      kw.get("loss_kind", 0), kw.get("loss_scale", 0), kw.get("inlet_mode", 0))
    p.resident_segments = kw.get("resident", 0)
    p.loss_frames, p.loss_stride = kw.get("frames", 0), kw.get("stride", 0)
    p._keep = (arr, keep)
    return p


def _bytes(L, p):
    b = ctypes.c_size_t(0)
    rc = L.lbm_workspace_bytes(ctypes.byref(p), ctypes.byref(b))
    return rc, b.value


def test_workspace_size_matches_the_plan(L):
    rc, b0 = _bytes(L, _problem(steps=2000))
    assert rc == 0
    state = 9 * 32 * 64 * 4
    assert 3 * state <= b0 < 3 * state + 200_000
    # tape: (n_seg - 1) checkpoints + (K - 1) segment states + 2 adjoint buffers
    rc, b1 = _bytes(L, _problem(steps=2000, K=45, tape=1))
    n_seg = -(-2000 // 45)
    assert b1 - b0 == (n_seg - 1 + 45 - 1 + 2) * state
    # 128^3 D3Q19 with K = 400 over 8000 steps: 423 states of 159.4 MB
    rc, b3 = _bytes(L, _problem(128, 128, 128, q=19, steps=8000, K=400, tape=1, bcy=1))
    assert rc == 0 and abs(b3 / (423 * 19 * 128 ** 3 * 4) - 1) < 3e-3


def test_resident_segments_cost_k_minus_one_states_each(L):
    state = 9 * 32 * 64 * 4
    n_seg = -(-2000 // 45)
    _, b1 = _bytes(L, _problem(steps=2000, K=45, tape=1))
    for R in (0, 1):
        assert _bytes(L, _problem(steps=2000, K=45, tape=1, resident=R))[1] == b1
    for R in (2, 7, n_seg):
        assert _bytes(L, _problem(steps=2000, K=45, tape=1, resident=R))[1] - b1 == (R - 1) * 44 * state
    # more than the number of segments is clamped; without a tape nothing is reserved
    assert _bytes(L, _problem(steps=2000, K=45, tape=1, resident=n_seg + 5))[1] == \
        _bytes(L, _problem(steps=2000, K=45, tape=1, resident=n_seg))[1]
    assert _bytes(L, _problem(steps=2000, resident=9))[1] == _bytes(L, _problem(steps=2000))[1]


@pytest.mark.parametrize("kw,code", [
    (dict(q=7), C.LBM_EINVAL),
    (dict(resident=-1), C.LBM_EINVAL),
    (dict(frames=-1), C.LBM_EINVAL),
    (dict(frames=3, stride=0), C.LBM_EINVAL),
    (dict(frames=3, stride=50, steps=100), C.LBM_EINVAL),   # the first frame would be step 0
    (dict(nx=1 << 20, ny=2), C.LBM_EINVAL),     # x positions are packed into 20 bits
    (dict(nz=2), C.LBM_EINVAL),                 # D2Q9 with nz != 1
    (dict(nx=1), C.LBM_EINVAL),                 # pressure axis needs nx >= 2
    (dict(steps=0), C.LBM_EINVAL),
    (dict(K=-1), C.LBM_EINVAL),
    (dict(bcy=0), C.LBM_EINVAL),                # pressure only on x
    (dict(loss_kind=5), C.LBM_EINVAL),
    (dict(nx=0), C.LBM_EINVAL),
])
def test_invalid_problems_are_rejected(L, kw, code):
    rc, _ = _bytes(L, _problem(**kw))
    assert rc == code
    assert len(L.lbm_last_error()) > 0


def test_loss_frames_hold_one_target_each(L):
    _, b1 = _bytes(L, _problem(steps=100))
    rc, b3 = _bytes(L, _problem(steps=100, frames=3, stride=49))
    assert rc == 0
    # two more target frames of D planes over the fluid nodes (64 x 32, all fluid)
    assert b3 - b1 == 2 * 2 * 64 * 32 * 4


def test_largest_row_length_is_accepted(L):
    rc, b = _bytes(L, _problem(nx=(1 << 20) - 1, ny=2))
    assert rc == 0 and b >= 3 * 9 * 2 * ((1 << 20) - 1) * 4


def test_instance_state_must_stay_below_4_gib(L):
    """One instance's Q planes of fluid nodes (padded to 64) are addressed with
    32-bit byte offsets: 19 x 56 512 704 x 4 B is the largest D3Q19 state
    below 4 GiB; one fluid node more pads the plane past it.  The limit counts
    fluid nodes, so a larger box of grains is accepted."""
    n = 400
    biggest = ((1 << 32) - 1) // (19 * 4) // 64 * 64
    assert biggest == 56_512_704
    solid = np.ones(n ** 3, np.uint8)
    for fluid, ok in ((biggest, True), (biggest + 1, False), (n ** 3, False)):
        solid[:] = 1
        solid[:fluid] = 0
        rc, b = _bytes(L, _problem(n, n, n, q=19, bcy=1, solid=solid.reshape(n, n, n)))
        assert (rc == 0) == ok, fluid
        if ok:
            assert b >= 3 * 19 * biggest * 4
        else:
            assert rc == C.LBM_EINVAL and "4 GiB" in L.lbm_last_error().decode()


def test_solid_inlet_rejected_in_profile_mode(L):
    s = np.zeros((1, 8, 16), np.uint8)
    s[0, 3, 0] = 1
    rc, _ = _bytes(L, _problem(16, 8, solid=s, inlet_mode=1))
    assert rc == C.LBM_EINVAL
    rc, _ = _bytes(L, _problem(16, 8, solid=s, inlet_mode=0))
    assert rc == C.LBM_OK


def test_init_rejects_small_or_misaligned_workspace(L):
    p = _problem(steps=10)
    rc, b = _bytes(L, p)
    h = ctypes.c_void_p()
    # validation happens before any device call: fake, never dereferenced pointers
    assert L.lbm_init(ctypes.byref(h), ctypes.byref(p), ctypes.c_void_p(1 << 20), b - 1, None) == C.LBM_ENOMEM
    assert L.lbm_init(ctypes.byref(h), ctypes.byref(p), ctypes.c_void_p((1 << 20) + 8), b, None) == C.LBM_EINVAL
    assert L.lbm_init(ctypes.byref(h), ctypes.byref(p), None, b, None) == C.LBM_EINVAL


def test_error_strings(L):
    for code in (0, -1, -2, -3, -4, -5, -6):
        assert len(L.lbm_strerror(code)) > 0
    assert L.lbm_strerror(-99) == b"unknown error"


def test_calls_without_handle_fail_cleanly(L):
    assert L.lbm_forward(None, None, 0, None) == C.LBM_EINVAL
    assert L.lbm_adjoint(None, None) == C.LBM_EINVAL
    assert L.lbm_grad(None, None, None, None) == C.LBM_EINVAL
    assert L.lbm_destroy(None) == C.LBM_OK


def test_flux_balance_workspace_bytes(L):
    """Per sample and section: one FP64 partial per chunk of at least 16 node
    rows (at most 64 chunks) and one FP32 factor; 0 for invalid sizes."""
    C.nnlib()
    f = L.lbmnn_flux_balance_workspace_bytes
    assert f(1, 1, 256, 256) == 256 * (16 * 8 + 4)          # 256 rows: 16 chunks
    assert f(2, 64, 64, 64) == 2 * 64 * (64 * 8 + 4)        # 4096 rows: capped at 64 chunks
    assert f(3, 1, 5, 300) == 3 * 300 * (1 * 8 + 4)         # 5 rows: one chunk
    assert f(1, 1, 4, 2049) == 0 and f(0, 1, 1, 1) == 0
