"""ctypes declarations of the libgx C ABI (include/gx.h).

Loading fails loudly when libgx.so has not been built: there is no fallback
path of any kind.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgx.so")

P = C.c_void_p
I32 = C.c_int
I64 = C.c_int64
D = C.c_double

GX_OK, GX_EINVAL, GX_ENOMEM, GX_EHIP, GX_ENOTBUILT, GX_ESTALE, GX_ENOCONV = 0, -1, -2, -3, -4, -5, -6
GX_TREE_ALL, GX_TREE_GAS = 0, 1
GX_QUAD, GX_DIRECT, GX_PREC_FP64 = 1, 2, 4
GX_NOALLOC_MAX_REGIONS = 16384

STATUS_NAMES = {0: "GX_OK", -1: "GX_EINVAL", -2: "GX_ENOMEM", -3: "GX_EHIP", -4: "GX_ENOTBUILT",
                -5: "GX_ESTALE", -6: "GX_ENOCONV"}


class GxStats(C.Structure):
    _fields_ = [("n_pp", I64), ("n_pc", I64), ("n_sph_list", I64), ("n_sph_ngb", I64),
                ("n_groups", I64), ("n_nodes", I64), ("n_iter_max", I64), ("n_noconv", I64),
                ("n_rewalk", I64), ("ms", D), ("ms_kernel", D)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class GxParticles(C.Structure):
    _fields_ = [("x", P), ("y", P), ("z", P), ("vx", P), ("vy", P), ("vz", P), ("m", P),
                ("eps2", P), ("id", P), ("type", P), ("n", I64)]


class GxGas(C.Structure):
    _fields_ = [("u", P), ("dudt", P), ("H64", P), ("H", P), ("rho", P), ("P", P), ("cs", P),
                ("vsig", P), ("n", I64)]


class GxUNet(C.Structure):
    _fields_ = [("levels", I32), ("base", I32), ("cin", I32), ("cout", I32), ("w_bf16", P),
                ("w_f32", P)]


# name -> (restype, argtypes), mirroring include/gx.h
SIGNATURES = {
    "gx_create": (I32, [C.POINTER(P), I32, P]),
    "gx_destroy": (I32, [P]),
    "gx_set_stream": (I32, [P, P]),
    "gx_last_error": (C.c_char_p, [P]),
    "gx_version": (C.c_char_p, []),
    "gx_set_walk_stack_limit": (I32, [P, I32]),
    "gx_tree_build": (I32, [P, C.POINTER(GxParticles), I32, I32, I32, P, C.POINTER(GxStats)]),
    "gx_gravity_forces": (I32, [P, C.POINTER(GxParticles), D, D, I32, P, P, P, P,
                                C.POINTER(GxStats)]),
    "gx_sph_density": (I32, [P, C.POINTER(GxParticles), C.POINTER(GxGas), D, D, D, I32,
                             C.POINTER(GxStats)]),
    "gx_sph_forces": (I32, [P, C.POINTER(GxParticles), C.POINTER(GxGas), D, D, P, P, P,
                            C.POINTER(GxStats)]),
    "gx_kick_drift": (I32, [P, I64, D, D, P, P, P, P, P, P, P, P, P, I64, P, P, D, P, P]),
    "gx_add_accel": (I32, [P, I64, P, P, P, P, P, P]),
    "gx_kick_drift_cubes": (I32, [P, I64, P, P, D, D, P, P, P, P, P, P, P, P, P, P, P, D, P, P]),
    "gx_energy": (I32, [P, C.POINTER(GxParticles), P, I64, P, P, P]),
    "gx_sph_timestep": (I32, [P, C.POINTER(GxGas), D, P, I32, P]),
    "gx_tree_counts": (I32, [P, I32, C.POINTER(I64), C.POINTER(I64)]),
    "gx_tree_export": (I32, [P, I32] + [P] * 15),
    "gx_gravity_list_sizes": (I32, [P, C.POINTER(I64), C.POINTER(I64), C.POINTER(I64)]),
    "gx_gravity_list_export": (I32, [P, P, P, P, P, P]),
    "gx_sn_extract": (I32, [P, C.POINTER(GxParticles), P, I32, D, P, P, I64, C.POINTER(I64)]),
    "gx_sn_inject": (I32, [P, C.POINTER(GxParticles), P, P, P, I32, I32, D, P]),
    "gx_sn_ambient": (I32, [P, C.POINTER(GxParticles), P, P, P, I32, D, D, P]),
    "gx_sn_gather": (I32, [P, C.POINTER(GxParticles), P, P, P, P, I32, I64, P, P, D, P, P, P, P, P,
                           P, P, P, P]),
    "gx_sn_unframe": (I32, [P, P, I32, I64, P, P, P, D, D, P, P, P]),
    "gx_sn_voxelize": (I32, [P, C.POINTER(GxParticles), P, P, P, I32, D, I32, D, P, P, P, P,
                             I32, P]),
    "gx_sn_resample": (I32, [P, P, I32, I32, D, P, P, I64, P, D, P, P, P, P, P, P, P]),
    "gx_sn_resample_gibbs": (I32, [P, P, I32, I32, D, P, P, I64, P, P, P, I32, P, D,
                                   P, P, P, P, P, P, P]),
    "gx_sn_encode8": (I32, [P, I64, P, I32, D, P]),
    "gx_sn_decode8": (I32, [P, I64, P, I32, P]),
    "gx_sn_check": (I32, [P, P, I32, I32, P, P, P]),
    "gx_sn_check_noalloc": (I32, [P, P, I32, I32, P, P, P]),
    "gx_sn_replace": (I32, [P, I64, P, I64, P, P, P, P, P, P, P, I64, P, I64, P, P, P, P, P, P, P,
                            P, C.POINTER(I64)]),
    "gx_conv3d_fwd": (I32, [P, P, I32, I32, I32, P, P, I32, I32, I32, P, P]),
    "gx_conv3d_fwd_fused": (I32, [P, P, I32, P, I32, I32, I32, I32, P, P, I32, I32, P, P]),
    "gx_conv3d_fwd_pool": (I32, [P, P, I32, I32, I32, P, P, I32, I32, P, P]),
    "gx_conv_head": (I32, [P, P, I32, I32, I32, P, P, I32, I32, P, P, P, I32]),
    "gx_conv3d_bwd_data": (I32, [P, P, I32, I32, I32, P, I32, I32, P, P]),
    "gx_conv3d_bwd_weight": (I32, [P, P, P, I32, I32, I32, I32, I32, P, P]),
    "gx_conv3d_bwd_weight_fused": (I32, [P, P, I32, P, I32, P, I32, I32, I32, I32, I32, P, P]),
    "gx_avgpool2": (I32, [P, P, I32, I32, I32, P, I32]),
    "gx_upsample2": (I32, [P, P, I32, I32, I32, P, I32]),
    "gx_concat": (I32, [P, P, I32, P, I32, I64, P, I32]),
    "gx_mse": (I32, [P, P, I32, P, I32, I64, P, C.POINTER(D)]),
    "gx_adam_step": (I32, [P, I64, P, P, P, P, D, D, D, D, I64, P]),
    "gx_f32_to_bf16": (I32, [P, P, I64, P]),
    "gx_chan_stats": (I32, [P, I64, P, I32, I32, P]),
    "gx_cube_sym": (I32, [P, P, I32, I32, I32, I32, P, P]),
    "gx_chan_affine": (I32, [P, I64, P, I32, I32, P, P, P, I32, P, I32]),
    "gx_grad_combine": (I32, [P, I64, P, P, P, P]),
    "gx_unet_sizes": (I32, [I32, I32, I32, I32, C.POINTER(I64), C.POINTER(I64)]),
    "gx_unet_layer": (I32, [I32, I32, I32, I32, I32, C.c_char_p, I32, C.POINTER(I32),
                            C.POINTER(I32), C.POINTER(I32), C.POINTER(I64), C.POINTER(I64)]),
    "gx_unet_forward": (I32, [P, C.POINTER(GxUNet), P, I32, I32, I32, P, I32, P, P, P]),
    "gx_unet_backward": (I32, [P, C.POINTER(GxUNet), P, I32, I32, P, P]),
    "gx_unet_saved": (I32, [P, C.c_char_p, I32, P, I64, C.POINTER(I64)]),
    "gx_chan_moments": (I32, [P, P, I32, D, D, P, P, P, P]),
}

_lib = None


def load():
    """Load libgx.so and declare every entry point; raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libgx.so not found at {LIB_PATH}: build it first "
                          f"(python -m paper_2510_23330_amd.build)")
    lib = C.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib
