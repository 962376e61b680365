"""ctypes view of the msplat C ABI (include/msplat.h).

Loading fails loudly if the HIP library has not been built: there is no
fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmsplat.so")

MSPLAT_OK = 0
MSPLAT_E_INVALID = 1
MSPLAT_E_CAPACITY = 2
MSPLAT_E_UNSUPPORTED = 3
MSPLAT_E_HIP = 4
MSPLAT_E_STATE = 5

MSPLAT_CHORD = 0
MSPLAT_CONTACT = 1

MSPLAT_FP32 = 0
MSPLAT_BF16 = 1
MSPLAT_BF16X3 = 2

c_f32p = ctypes.POINTER(ctypes.c_float)
c_f64p = ctypes.POINTER(ctypes.c_double)


class Model(ctypes.Structure):
    _fields_ = [("num_prims", ctypes.c_int32), ("pe_freqs", ctypes.c_int32),
                ("hidden_width", ctypes.c_int32), ("hidden_layers", ctypes.c_int32),
                ("out_dim", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("primitive", ctypes.c_int32)]


class Opts(ctypes.Structure):
    _fields_ = [("samples_fixed", ctypes.c_int32), ("samples_min", ctypes.c_int32),
                ("samples_max", ctypes.c_int32), ("samples_per_unit", ctypes.c_float),
                ("t_stop", ctypes.c_float), ("jitter", ctypes.c_int32),
                ("jitter_seed", ctypes.c_uint32), ("background", ctypes.c_float * 3),
                ("order", ctypes.c_int32), ("hits_per_item", ctypes.c_int32),
                ("items_per_group", ctypes.c_int32), ("tile_rays", ctypes.c_void_p)]


class Stats(ctypes.Structure):
    _fields_ = [("num_rays", ctypes.c_int64), ("num_hits", ctypes.c_int64),
                ("num_samples", ctypes.c_int64), ("num_work_items", ctypes.c_int64),
                ("num_terminated", ctypes.c_int64), ("num_fallbacks", ctypes.c_int64),
                ("min_abs_g", ctypes.c_float), ("hits_per_item", ctypes.c_int32),
                ("items_per_group", ctypes.c_int32)]


EXPORTS = {
    "msplat_create": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(ctypes.c_void_p)]),
    "msplat_destroy": (None, [ctypes.c_void_p]),
    "msplat_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "msplat_num_params": (ctypes.c_int64, [ctypes.POINTER(Model)]),
    "msplat_workspace_size": (ctypes.c_int, [ctypes.POINTER(Model), ctypes.c_int64, ctypes.c_int64,
                                             ctypes.POINTER(ctypes.c_uint64)]),
    "msplat_render_forward": (ctypes.c_int, [
        ctypes.c_void_p, ctypes.POINTER(Model), ctypes.POINTER(Opts),
        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
        ctypes.c_void_p, ctypes.c_uint64, ctypes.POINTER(ctypes.c_uint64), ctypes.c_void_p]),
    "msplat_render_forward_noalloc": (ctypes.c_int, [
        ctypes.c_void_p, ctypes.POINTER(Model), ctypes.POINTER(Opts),
        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
        ctypes.POINTER(ctypes.c_uint64), ctypes.c_void_p]),
    "msplat_render_backward": (ctypes.c_int, [
        ctypes.c_void_p, ctypes.POINTER(Model), ctypes.POINTER(Opts),
        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64,
        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "msplat_slot_forward": (ctypes.c_int, [
        ctypes.c_void_p, ctypes.POINTER(Model), ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64,
        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p]),
    "msplat_render_backward_slots": (ctypes.c_int, [
        ctypes.c_void_p, ctypes.POINTER(Model), ctypes.POINTER(Opts),
        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
        ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64,
        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
        ctypes.c_void_p]),
    "msplat_autotune": (ctypes.c_int, [
        ctypes.c_void_p, ctypes.POINTER(Model), ctypes.POINTER(Opts),
        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
        ctypes.c_void_p, ctypes.c_uint64,
        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
        ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32), ctypes.c_void_p]),
    "msplat_profile_enable": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    "msplat_profile_read": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int,
                                           ctypes.POINTER(ctypes.c_char_p),
                                           ctypes.POINTER(ctypes.c_double),
                                           ctypes.POINTER(ctypes.c_int64),
                                           ctypes.POINTER(ctypes.c_int)]),
    "msplat_get_stats": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64,
                                        ctypes.POINTER(Stats), ctypes.c_void_p]),
    "msplat_debug_hits": (ctypes.c_int, [
        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int64,
        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
        ctypes.c_void_p]),
    "msplat_render_forward_f64": (ctypes.c_int, [
        ctypes.c_void_p, ctypes.POINTER(Model), ctypes.POINTER(Opts),
        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
        ctypes.c_void_p, ctypes.c_uint64, ctypes.POINTER(ctypes.c_uint64), ctypes.c_void_p]),
}

_lib = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libmsplat.so and declare every exported entry point."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"msplat HIP library not built: {path} is missing "
                          "(run `python -m paper_2606_03877_amd.build`)")
    lib = ctypes.CDLL(path)
    for name, (res, args) in EXPORTS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class MsplatError(RuntimeError):
    def __init__(self, status: int, where: str):
        lib = load()
        super().__init__(f"{where}: {lib.msplat_status_string(status).decode()} (status {status})")
        self.status = status
