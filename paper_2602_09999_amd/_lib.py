"""ctypes view of libfastergs.so (include/fastergs.h).  Argument marshalling only."""
from __future__ import annotations

import ctypes
import os
import threading

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfastergs.so")

c_int32, c_int64, c_uint32, c_float, c_size_t, c_void_p, c_double = (
    ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_float, ctypes.c_size_t,
    ctypes.c_void_p, ctypes.c_double)

FGS_OK, FGS_ERR_INVALID_ARGUMENT, FGS_ERR_CAPACITY, FGS_ERR_HIP, FGS_ERR_UNSUPPORTED = range(5)
FGS_F32, FGS_BF16 = 0, 1
FGS_MAX_VIEWS = 16
FGS_FORWARD_NO_SYNC = 1


def FGS_FORWARD_DEPTH_BITS(b: int) -> int:
    """Mode bits: with FGS_FORWARD_NO_SYNC, sort the depth keys' low b bits only."""
    return int(b) << 8
FGS_FLAG_FP64_CONIC, FGS_FLAG_LOOKBACK_FALLBACK, FGS_FLAG_BLEND_QUEUE, FGS_FLAG_SORT_LARGE_BLOCKS = 1, 2, 4, 8
FGS_FLAG_KEEP_ACCUM_ZERO = 16
FGS_SORT_NOALLOC_MAX_PAIRS = 1 << 20
FGS_SORT_NOALLOC_SCRATCH_BYTES = 17 << 19


class Gaussians(ctypes.Structure):
    _fields_ = [("n", c_int64), ("means", c_void_p), ("log_scales", c_void_p), ("quats", c_void_p),
                ("opacity_logits", c_void_p), ("sh_dc", c_void_p), ("sh_rest", c_void_p),
                ("sh_dtype", c_int32), ("sh_degree", c_int32), ("velocity", c_void_p), ("accel", c_void_p),
                ("mean_t", c_void_p), ("log_scale_t", c_void_p), ("quats_r", c_void_p)]


class GaussianGrads(ctypes.Structure):
    _fields_ = [("means", c_void_p), ("log_scales", c_void_p), ("quats", c_void_p),
                ("opacity_logits", c_void_p), ("sh_dc", c_void_p), ("sh_rest", c_void_p),
                ("velocity", c_void_p), ("accel", c_void_p), ("mean_t", c_void_p), ("log_scale_t", c_void_p),
                ("quats_r", c_void_p)]


class Camera(ctypes.Structure):
    _fields_ = [("world_to_cam", c_float * 16), ("fx", c_float), ("fy", c_float), ("cx", c_float),
                ("cy", c_float), ("width", c_int32), ("height", c_int32), ("near_z", c_float),
                ("bg", c_float * 3)]


class Settings(ctypes.Structure):
    _fields_ = [("tile", c_int32), ("alpha_min", c_float), ("alpha_max", c_float), ("t_min", c_float),
                ("dilation", c_float), ("quat_min", c_float), ("det_min", c_float), ("flags", c_uint32)]


class ForwardStats(ctypes.Structure):
    _fields_ = [("n_visible", c_int64), ("n_instances", c_int64), ("tiles_x", c_int64), ("tiles_y", c_int64),
                ("depth_key_bits", c_int64)]


class Layout(ctypes.Structure):
    _fields_ = [("rec", c_size_t), ("n_tiles", c_size_t), ("depth_key", c_size_t),
                ("counters", c_size_t), ("vis_keys", c_size_t * 2), ("vis_ids", c_size_t * 2),
                ("dup_scan", c_size_t), ("inst_keys", c_size_t * 2), ("inst_vals", c_size_t * 2),
                ("ranges", c_size_t), ("accum", c_size_t), ("marks", c_size_t), ("touched", c_size_t),
                ("touched_list", c_size_t), ("slot_of", c_size_t), ("sparse_grads", c_size_t), ("queues", c_size_t),
                ("scratch", c_size_t),
                ("total", c_size_t),
                ("inst_final", c_int32), ("inst_key_bytes", c_int32), ("tiles_x", c_int32), ("tiles_y", c_int32),
                ("instance_capacity", c_int64), ("n_views", c_int64), ("total_tiles", c_int64)]


class AdamGroup(ctypes.Structure):
    _fields_ = [("param", c_void_p), ("grad", c_void_p), ("exp_avg", c_void_p), ("exp_avg_sq", c_void_p),
                ("numel", c_int64), ("lr", c_float), ("dtype", c_int32)]


class AdamMoments(ctypes.Structure):
    _fields_ = [("exp_avg", c_void_p * 6), ("exp_avg_sq", c_void_p * 6), ("lr", c_float * 6)]


# name -> (restype, argtypes); every symbol the header declares
SIGNATURES = {
    "fgs_abi_version": (c_int32, []),
    "fgs_status_string": (ctypes.c_char_p, [c_int32]),
    "fgs_last_error": (ctypes.c_char_p, []),
    "fgs_default_settings": (c_int32, [ctypes.POINTER(Settings)]),
    "fgs_workspace_size": (c_int32, [c_int64, ctypes.POINTER(Camera), ctypes.POINTER(Settings), c_int64,
                                     ctypes.POINTER(c_size_t)]),
    "fgs_workspace_layout": (c_int32, [c_int64, ctypes.POINTER(Camera), ctypes.POINTER(Settings), c_int64,
                                       ctypes.POINTER(Layout)]),
    "fgs_rasterize_forward": (c_int32, [ctypes.POINTER(Gaussians), ctypes.POINTER(Camera), ctypes.POINTER(Settings),
                                        c_void_p, c_size_t, c_int64, c_void_p, c_void_p, c_void_p,
                                        ctypes.POINTER(ForwardStats), c_void_p]),
    "fgs_rasterize_backward": (c_int32, [ctypes.POINTER(Gaussians), ctypes.POINTER(Camera), ctypes.POINTER(Settings),
                                         c_void_p, c_size_t, c_int64, c_void_p, c_void_p, c_void_p,
                                         ctypes.POINTER(GaussianGrads), c_void_p]),
    "fgs_rasterize_backward_adam": (c_int32, [ctypes.POINTER(Gaussians), ctypes.POINTER(Camera),
                                              ctypes.POINTER(Settings), c_void_p, c_size_t, c_int64, c_void_p,
                                              c_void_p, c_void_p, ctypes.POINTER(AdamMoments), c_int64, c_double,
                                              c_double, c_double, c_void_p]),
    "fgs_batch_workspace_size": (c_int32, [c_int64, ctypes.POINTER(Camera), c_int32, ctypes.POINTER(Settings),
                                           c_int64, ctypes.POINTER(c_size_t)]),
    "fgs_batch_workspace_layout": (c_int32, [c_int64, ctypes.POINTER(Camera), c_int32, ctypes.POINTER(Settings),
                                             c_int64, ctypes.POINTER(Layout)]),
    "fgs_rasterize_forward_batch": (c_int32, [ctypes.POINTER(Gaussians), ctypes.POINTER(Camera),
                                              ctypes.POINTER(c_float), c_int32, ctypes.POINTER(Settings), c_void_p,
                                              c_size_t, c_int64, c_void_p, c_void_p, c_void_p, c_uint32,
                                              ctypes.POINTER(ForwardStats), c_void_p]),
    "fgs_rasterize_backward_batch": (c_int32, [ctypes.POINTER(Gaussians), ctypes.POINTER(Camera),
                                               ctypes.POINTER(c_float), c_int32, ctypes.POINTER(Settings), c_void_p,
                                               c_size_t, c_int64, c_void_p, c_void_p, c_void_p,
                                               ctypes.POINTER(GaussianGrads), c_void_p]),
    "fgs_adam_step": (c_int32, [ctypes.POINTER(AdamGroup), c_int32, c_int64, c_double, c_double, c_double,
                                c_void_p]),
    "fgs_adam_step_device": (c_int32, [ctypes.POINTER(AdamGroup), c_int32, c_void_p, c_double, c_double, c_double,
                                       c_void_p]),
    "fgs_l1_loss_backward": (c_int32, [c_void_p, c_void_p, c_int64, c_void_p, c_void_p, c_void_p]),
    "fgs_time_next_launch": (c_int32, [ctypes.c_char_p, c_void_p, c_void_p]),
    "fgs_zorder_workspace_size": (c_int32, [c_int64, ctypes.POINTER(c_size_t)]),
    "fgs_zorder_permutation": (c_int32, [c_void_p, c_int64, c_void_p, c_size_t, c_void_p, c_void_p]),
    "fgs_sort_workspace_size": (c_int32, [c_int64, c_int32, ctypes.POINTER(c_size_t)]),
    "fgs_sort_pairs": (c_int32, [c_void_p, c_void_p, c_int64, c_int32, c_int32, c_void_p, c_size_t, c_void_p]),
    "fgs_sort_pairs_noalloc": (c_int32, [c_void_p, c_void_p, c_int64, c_int32, c_int32, c_void_p]),
    "fgs_permute_planes": (c_int32, [c_void_p, c_void_p, c_int64, c_int32, c_int32, c_void_p, c_void_p]),
}

_lib = None
_lock = threading.Lock()


class FasterGSError(RuntimeError):
    def __init__(self, status: int, fn: str, message: str):
        super().__init__(f"{fn} failed with status {status}: {message}")
        self.status = status


# the structures above mirror include/fastergs.h at this ABI version
ABI_VERSION = 13


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load the HIP library; raises if it has not been built (there is no fallback)."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(path):
                raise FileNotFoundError(
                    f"{path} is missing: build it with `python -m paper_2602_09999_amd.build` "
                    "(the rasterizer has no CPU fallback)")
            lib = ctypes.CDLL(path)
            for name, (res, args) in SIGNATURES.items():
                fn = getattr(lib, name)
                fn.restype = res
                fn.argtypes = args
            if lib.fgs_abi_version() != ABI_VERSION:
                raise RuntimeError(f"{path} has ABI version {lib.fgs_abi_version()}, this binding expects "
                                   f"{ABI_VERSION}: rebuild it with `python -m paper_2602_09999_amd.build`")
            _lib = lib
        return _lib


def check(status: int, fn: str) -> None:
    if status != FGS_OK:
        msg = load().fgs_last_error().decode(errors="replace")
        raise FasterGSError(status, fn, msg)
