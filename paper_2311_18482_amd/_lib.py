"""ctypes view of liblegs.so (include/legs.h). Argument marshalling only.

The library is built in-tree by paper_2311_18482_amd/build.py; importing this
module never builds or falls back to anything: a missing library raises.
"""
from __future__ import annotations

import ctypes as ct
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblegs.so")

LEGS_OK = 0
LEGS_ERR_ARG = -1
LEGS_ERR_CAPACITY = -2
LEGS_ERR_HIP = -3
LEGS_ERR_UNSUPPORTED = -4
LEGS_MAX_CHANNELS = 64
LEGS_FLAG_PERSISTENT = 1
LEGS_FLAG_FULL_SORT = 2
LEGS_FLAG_FULL_BOX = 4
LEGS_FLAG_IDS_ONLY = 8
LEGS_MLP_NORMALIZE_INPUT = 1


class LegsError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"legs error {code}: {msg}")
        self.code = code


class Camera(ct.Structure):
    _fields_ = [("width", ct.c_int32), ("height", ct.c_int32), ("fx", ct.c_double),
                ("fy", ct.c_double), ("cx", ct.c_double), ("cy", ct.c_double),
                ("R", ct.c_double * 9), ("t", ct.c_double * 3)]


class View(ct.Structure):
    _fields_ = [("cam", Camera), ("tiles_x", ct.c_int32), ("tiles_y", ct.c_int32),
                ("tile_offset", ct.c_int64), ("pixel_offset", ct.c_int64)]


class Opts(ct.Structure):
    _fields_ = [("tile", ct.c_int32), ("lds_batch", ct.c_int32), ("alpha_max", ct.c_float),
                ("alpha_min", ct.c_float), ("t_min", ct.c_float), ("flags", ct.c_int32),
                ("lowpass", ct.c_double), ("z_near", ct.c_double), ("guard", ct.c_double)]


class Projected(ct.Structure):
    _fields_ = [("mean2d", ct.c_void_p), ("conic", ct.c_void_p), ("box", ct.c_void_p),
                ("depth", ct.c_void_p), ("ntiles", ct.c_void_p), ("block_offsets", ct.c_void_p),
                ("order", ct.c_void_p)]


class AdamGroup(ct.Structure):
    _fields_ = [("param", ct.c_void_p), ("grad", ct.c_void_p), ("m", ct.c_void_p),
                ("v", ct.c_void_p), ("n", ct.c_int64), ("clamp_every", ct.c_int32),
                ("clamp_offset", ct.c_int32), ("clamp_lo", ct.c_float), ("clamp_hi", ct.c_float)]


class Bins(ct.Structure):
    _fields_ = [("keys", ct.c_void_p), ("keys_alt", ct.c_void_p), ("ids", ct.c_void_p),
                ("ids_alt", ct.c_void_p), ("ranges", ct.c_void_p), ("scratch", ct.c_void_p),
                ("count", ct.c_void_p), ("capacity", ct.c_int64)]


_lib = None

# name -> (restype, argtypes)
P = ct.c_void_p
I32, I64 = ct.c_int32, ct.c_int64
_SIGS = {
    "legs_version": (I32, []),
    "legs_opts_default": (None, [ct.POINTER(Opts)]),
    "legs_create": (I32, [I32, ct.POINTER(P)]),
    "legs_destroy": (I32, [P]),
    "legs_last_error": (ct.c_char_p, [P]),
    "legs_views_build": (I32, [ct.POINTER(Camera), I32, ct.POINTER(Opts), ct.POINTER(View),
                               ct.POINTER(I64), ct.POINTER(I64)]),
    "legs_projected_blocks": (I64, [I64, I32]),
    "legs_sort_scratch_bytes": (I64, [I64, I64]),
    "legs_order_scratch_bytes": (I64, [I64, I32]),
    "legs_sort_passes": (I32, [I64]),
    "legs_project": (I32, [P, P, P, P, P, I64, P, I32, ct.POINTER(Opts), ct.POINTER(Projected), P]),
    "legs_bin_sort": (I32, [P, ct.POINTER(Projected), I64, P, I32, I64, ct.POINTER(Opts),
                            ct.POINTER(Bins), ct.POINTER(I64), P]),
    "legs_render_forward": (I32, [P, ct.POINTER(Projected), I64, ct.POINTER(Bins), P, I32, I64, P,
                                  I32, ct.POINTER(Opts), P, P, P, P]),
    "legs_render_forward_zero": (I32, [P, ct.POINTER(Projected), I64, ct.POINTER(Bins), P, I32, I64, P,
                                       I32, ct.POINTER(Opts), P, P, P, P, I64, P]),
    "legs_render_backward": (I32, [P, ct.POINTER(Projected), I64, ct.POINTER(Bins), P, I32, I64,
                                   P, I32, ct.POINTER(Opts), P, P, P, P, P, P]),
    "legs_render_counts": (I32, [P, ct.POINTER(Projected), I64, ct.POINTER(Bins), P, I32, I64,
                                 ct.POINTER(Opts), P, P]),
    "legs_project_backward": (I32, [P, P, P, P, P, I64, P, I32, ct.POINTER(Opts),
                                    ct.POINTER(Projected), P, P, P, P, P, P]),
    "legs_decode_plain": (I32, [P, P, I64, I64, I64, P, I32, P, I32, P, P, P]),
    "legs_decode_fold": (I32, [P, P, I32, P, I32, P, P]),
    "legs_decode_folded": (I32, [P, P, I64, I64, I64, P, I32, P, P, P]),
    "legs_mlp_param_count": (I64, [I32]),
    "legs_decode_mlp": (I32, [P, P, I64, I64, I64, P, I32, I32, P, P, P]),
    "legs_mlp_workspace_bytes": (I64, [I64, I32]),
    "legs_dmlp_param_count": (I64, [I32]),
    "legs_smooth_param_count": (I64, []),
    "legs_smooth_workspace_bytes": (I64, [I64]),
    "legs_smooth_loss_grad": (I32, [P, P, P, I32, I32, I32, I64, P, ct.c_float, ct.c_float, P, P, P, P, P]),
    "legs_quantize_workspace_bytes": (I64, [I64, I32, I32]),
    "legs_quantize": (I32, [P, P, I64, I32, I32, P, I32, ct.c_float, ct.c_float, ct.c_float, P, P, P, P, P,
                            P, P]),
    "legs_decode_dmlp": (I32, [P, P, I64, I64, I64, P, I32, I32, P, P, P, P]),
    "legs_language_features": (I32, [P, P, I64, I32, P, I32, I32, P, P]),
    "legs_mlp_grad": (I32, [P, P, I64, I64, I64, P, I32, I32, P, P, P, P, P]),
    "legs_semantic_loss_grad": (I32, [P, P, P, I64, I64, I64, P, I32, I32, P, ct.c_float, ct.c_float,
                                      ct.c_float, P, P, P, I64, I64, P, P, P]),
    "legs_semantic_loss_grad_noalloc": (I32, [P, P, P, I64, I64, I64, P, I32, I32, P, ct.c_float,
                                              ct.c_float, ct.c_float, P, P, I64, I64, P, P, P]),
    "legs_adam": (I32, [P, ct.POINTER(AdamGroup), I32, I32, ct.c_float, ct.c_double, ct.c_double,
                        ct.c_float, P]),
    "legs_mlp_train_step": (I32, [P, P, I64, I64, I64, P, I32, I32, P, P, P, P, I32, ct.c_float,
                                  ct.c_double, ct.c_double, ct.c_float, P, P, P]),
    "legs_l1_loss_grad": (I32, [P, P, P, P, I32, I64, I32, I32, ct.c_float, P, P, P]),
    "legs_clear": (I32, [P, P, I64, P]),
    "legs_capture_begin": (I32, [P, P]),
    "legs_capture_end": (I32, [P, P, ct.POINTER(P)]),
    "legs_graph_launch": (I32, [P, P, P]),
    "legs_graph_destroy": (I32, [P]),
    "legs_autotune": (I32, [P, P, P, P, P, P, I64, I32, ct.POINTER(Camera), I32, ct.POINTER(Opts),
                            P, I32, ct.POINTER(Opts), P, P]),
}


def exported_names():
    return sorted(_SIGS)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -c 'import __graft_entry__ as g; g.build()'`")
        L = ct.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def check(ctx, code):
    if code != LEGS_OK:
        msg = lib().legs_last_error(ctx) if ctx else b""
        raise LegsError(code, (msg or b"").decode(errors="replace"))
    return code
