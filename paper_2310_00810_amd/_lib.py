"""ctypes binding of liblbm.so (declared in include/lbm.h).

Argument marshalling only: every step of the method runs in the library's
HIP kernels.  Loading fails loudly when the library has not been built.
"""
import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(PKG, "liblbm.so")

LBM_OK, LBM_EINVAL, LBM_ENOMEM, LBM_ESTATE, LBM_EUNSTABLE, LBM_ECORRUPT, LBM_EDEVICE = 0, -1, -2, -3, -4, -5, -6
LBM_D2Q9, LBM_D3Q19 = 9, 19
BC_PRESSURE, BC_PERIODIC, BC_WALL, BC_ABB, BC_VELOCITY = 0, 1, 2, 3, 4
COLL_BGK, COLL_MRT = 0, 1
LOSS_VEC, LOSS_NORM = 0, 1
SCALE_SUM, SCALE_MEAN_FLUID = 0, 1
INLET_CONST, INLET_PROFILE = 0, 1
POP_STATE, POP_ADJOINT = 0, 1

# Every symbol include/lbm.h declares.
EXPORTS = [
    "lbm_workspace_bytes", "lbm_init", "lbm_destroy", "lbm_set_initial", "lbm_set_populations",
    "lbm_get_populations", "lbm_forward", "lbm_adjoint", "lbm_grad", "lbm_run_to_residual",
    "lbm_get_macro", "lbm_set_graphs", "lbm_set_timing", "lbm_get_timing", "lbm_checkpoint", "lbm_get_residuals", "lbm_stream_copy",
    "lbm_strerror",
    "lbm_last_error",
]


class LBMError(RuntimeError):
    def __init__(self, code, where, detail):
        super().__init__(f"{where}: {detail} (code {code})")
        self.code = code


class lbm_instance(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
                ("solid", ctypes.c_void_p), ("roi", ctypes.c_void_p), ("target_u", ctypes.c_void_p)]


class lbm_problem(ctypes.Structure):
    _fields_ = [("lattice", ctypes.c_int), ("n_inst", ctypes.c_int),
                ("inst", ctypes.POINTER(lbm_instance)),
                ("bc_x", ctypes.c_int), ("bc_y", ctypes.c_int), ("bc_z", ctypes.c_int),
                ("steps", ctypes.c_int), ("ckpt_interval", ctypes.c_int), ("tape", ctypes.c_int),
                ("loss_kind", ctypes.c_int), ("loss_scale", ctypes.c_int), ("inlet_mode", ctypes.c_int),
                ("collision", ctypes.c_int), ("mrt_rates", ctypes.c_double * 9),
                ("resident_segments", ctypes.c_int), ("loss_frames", ctypes.c_int),
                ("loss_stride", ctypes.c_int)]


class lbm_params(ctypes.Structure):
    _fields_ = [("tau", ctypes.POINTER(ctypes.c_double)), ("drho_in", ctypes.POINTER(ctypes.c_double)),
                ("drho_out", ctypes.POINTER(ctypes.c_double))]


class lbm_timing(ctypes.Structure):
    _fields_ = [("forward_ms", ctypes.c_double), ("forward_launches", ctypes.c_long),
                ("recompute_ms", ctypes.c_double), ("recompute_launches", ctypes.c_long),
                ("adjoint_ms", ctypes.c_double), ("adjoint_launches", ctypes.c_long)]


_lib = None


def lib():
    """The loaded liblbm.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIBPATH):
            raise RuntimeError(f"{LIBPATH} is missing: build it with `python -m paper_2310_00810_amd.build` "
                               "(the HIP library is required; there is no fallback)")
        L = ctypes.CDLL(LIBPATH)
        vp, ip, dp = ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_double)
        L.lbm_workspace_bytes.argtypes = [ctypes.POINTER(lbm_problem), ctypes.POINTER(ctypes.c_size_t)]
        L.lbm_init.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(lbm_problem), vp, ctypes.c_size_t, vp]
        L.lbm_destroy.argtypes = [vp]
        L.lbm_set_initial.argtypes = [vp, vp, vp]
        L.lbm_set_populations.argtypes = [vp, vp]
        L.lbm_get_populations.argtypes = [vp, ip, vp]
        L.lbm_forward.argtypes = [vp, ctypes.POINTER(lbm_params), ip, dp]
        L.lbm_adjoint.argtypes = [vp, vp]
        L.lbm_grad.argtypes = [vp, dp, dp, dp]
        L.lbm_run_to_residual.argtypes = [vp, ctypes.POINTER(lbm_params), ctypes.c_double, ip, ip,
                                          ctypes.POINTER(ctypes.c_int), dp]
        L.lbm_get_macro.argtypes = [vp, vp, vp, ip]
        L.lbm_set_graphs.argtypes = [vp, ip]
        L.lbm_set_timing.argtypes = [vp, ip, ip]
        L.lbm_get_timing.argtypes = [vp, ctypes.POINTER(lbm_timing)]
        L.lbm_get_residuals.argtypes = [vp, dp]
        L.lbm_stream_copy.argtypes = [vp, vp, ctypes.c_size_t, vp]
        L.lbm_checkpoint.argtypes = [vp, ip, ctypes.POINTER(vp), ctypes.POINTER(ctypes.c_size_t)]
        L.lbm_strerror.restype = ctypes.c_char_p
        L.lbm_strerror.argtypes = [ip]
        L.lbm_last_error.restype = ctypes.c_char_p
        for name in EXPORTS:
            if name not in ("lbm_strerror", "lbm_last_error"):
                getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def check(rc, where):
    if rc != LBM_OK:
        L = lib()
        raise LBMError(rc, where, f"{L.lbm_strerror(rc).decode()}: {L.lbm_last_error().decode()}")
    return rc


# ------------------------------------------------------------ lbmnn.h ABI --
NN_EXPORTS = [
    "lbmnn_conv", "lbmnn_conv_workspace_bytes", "lbmnn_conv_ws", "lbmnn_wgrad_workspace_bytes", "lbmnn_conv_wgrad",
    "lbmnn_conv_wgrad_noalloc",
    "lbmnn_weight_transpose",
    "lbmnn_bias_grad", "lbmnn_relu_bwd", "lbmnn_relu_bwd_bias_grad", "lbmnn_pool_fwd", "lbmnn_pool_bwd",
    "lbmnn_mse", "lbmnn_adam", "lbmnn_to_bf16", "lbmnn_features", "lbmnn_normalize", "lbmnn_denormalize",
    "lbmnn_flux_balance_workspace_bytes", "lbmnn_flux_balance",
]
NN_RELU, NN_ACCUMULATE, NN_S2D, NN_D2S, NN_S2D_G = 1, 2, 4, 8, 16
LBMNN_NOALLOC_SCRATCH_BYTES = 32 << 20


class lbmnn_conv_desc(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("d", ctypes.c_int), ("h", ctypes.c_int), ("w", ctypes.c_int),
                ("dims", ctypes.c_int), ("ks", ctypes.c_int), ("cin", ctypes.c_int), ("cout", ctypes.c_int),
                ("flags", ctypes.c_int), ("in_", ctypes.c_void_p), ("in_cstride", ctypes.c_int),
                ("in_coff", ctypes.c_int), ("out", ctypes.c_void_p), ("out_f32", ctypes.c_void_p),
                ("out_cstride", ctypes.c_int), ("out_coff", ctypes.c_int)]


_nn_ready = False


def nnlib():
    """liblbm.so with the lbmnn_* signatures declared."""
    global _nn_ready
    L = lib()
    if not _nn_ready:
        vp, ip, ll, fl = ctypes.c_void_p, ctypes.c_int, ctypes.c_longlong, ctypes.c_float
        dp = ctypes.POINTER(lbmnn_conv_desc)
        L.lbmnn_conv.argtypes = [dp, vp, vp, vp]
        L.lbmnn_conv_workspace_bytes.argtypes = [dp]
        L.lbmnn_conv_workspace_bytes.restype = ctypes.c_size_t
        L.lbmnn_conv_ws.argtypes = [dp, vp, vp, vp, ctypes.c_size_t, vp]
        L.lbmnn_wgrad_workspace_bytes.argtypes = [ll, ip, ip, ip]
        L.lbmnn_wgrad_workspace_bytes.restype = ctypes.c_size_t
        L.lbmnn_conv_wgrad.argtypes = [dp, vp, ip, ip, ip, vp, ip, vp, ctypes.c_size_t, ip, vp]
        L.lbmnn_conv_wgrad_noalloc.argtypes = [dp, vp, ip, ip, ip, vp, ip, ip, vp]
        L.lbmnn_weight_transpose.argtypes = [vp, vp, ip, ip, ip, ip, vp]
        L.lbmnn_bias_grad.argtypes = [vp, ip, ip, ll, ip, vp, ip, vp, ip, vp]
        L.lbmnn_relu_bwd.argtypes = [vp, vp, ip, ip, ll, ip, vp]
        L.lbmnn_relu_bwd_bias_grad.argtypes = [vp, vp, ip, ip, ll, ip, vp, ip, vp, ip, vp]
        L.lbmnn_pool_fwd.argtypes = [vp, ip, ip, vp, ip, ip, ip, ip, ip, ip, ip, ip, vp]
        L.lbmnn_pool_bwd.argtypes = [vp, ip, ip, vp, ip, ip, vp, ip, ip, ip, ip, ip, ip, ip, ip, ip, vp]
        L.lbmnn_mse.argtypes = [vp, ip, vp, vp, ip, ll, fl, vp, vp, vp, vp]
        L.lbmnn_adam.argtypes = [vp, vp, vp, vp, vp, ll, fl, fl, fl, fl, ip, vp]
        L.lbmnn_to_bf16.argtypes = [vp, vp, ll, vp]
        L.lbmnn_features.argtypes = [vp, vp, ip, ip, ip, ip, vp, vp]
        L.lbmnn_normalize.argtypes = [vp, vp, vp, vp, ll, ip, ll, vp, vp, vp]
        L.lbmnn_denormalize.argtypes = [vp, ip, vp, vp, ll, ip, ll, vp, vp, vp]
        L.lbmnn_flux_balance_workspace_bytes.argtypes = [ip, ip, ip, ip]
        L.lbmnn_flux_balance_workspace_bytes.restype = ll
        L.lbmnn_flux_balance.argtypes = [vp, ip, ip, ip, ip, ip, vp, vp, ll, vp]
        for n in NN_EXPORTS:
            if n not in ("lbmnn_wgrad_workspace_bytes", "lbmnn_conv_workspace_bytes"):
                getattr(L, n).restype = ctypes.c_int
        _nn_ready = True
    return L
