"""ctypes declarations of libmg.so (the C ABI in include/mg.h).

Argument marshalling only: every step of the query and propagation path runs
in the library's HIP kernels. Importing this module fails loudly if the
library has not been built; there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmg.so")

MG_OK = 0
ERRORS = {
    -1: "MG_EINVAL", -2: "MG_ENOMEM", -3: "MG_EDEVICE", -4: "MG_ESTATE",
    -5: "MG_EDEPTH", -6: "MG_EIO", -7: "MG_EFORMAT", -8: "MG_ELIMIT",
}
MAX_LEVELS = 24


class MGError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("%s (%d): %s" % (ERRORS.get(code, "MG_E?"), code, msg))
        self.code = code


class BuildOpts(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_uint32), ("ny", ctypes.c_uint32), ("nz", ctypes.c_uint32),
                ("defer", ctypes.c_uint32), ("max_depth", ctypes.c_uint32), ("threads", ctypes.c_uint32),
                ("factorizer", ctypes.c_uint32), ("tau", ctypes.c_uint32), ("reserved", ctypes.c_uint32 * 2)]


class Info(ctypes.Structure):
    _fields_ = [("nseg", ctypes.c_uint32), ("n_nodes", ctypes.c_uint32), ("depth", ctypes.c_uint32),
                ("n_levels", ctypes.c_uint32), ("dims", (ctypes.c_uint32 * 3) * MAX_LEVELS),
                ("map_voxels", ctypes.c_uint64), ("device_bytes", ctypes.c_uint64), ("device", ctypes.c_int32),
                ("max_mixture", ctypes.c_uint32), ("quant_bits", ctypes.c_uint32), ("runs_mask", ctypes.c_uint32)]


class LaunchCfg(ctypes.Structure):
    _fields_ = [("unroll_big", ctypes.c_uint32), ("unroll_small", ctypes.c_uint32),
                ("unroll_naive", ctypes.c_uint32), ("tf_block", ctypes.c_uint32), ("table_big", ctypes.c_uint32),
                ("table_small", ctypes.c_uint32), ("table_retry", ctypes.c_uint32), ("block_small", ctypes.c_uint32),
                ("block_big", ctypes.c_uint32), ("chunk_small", ctypes.c_uint32),
                ("tf_planes", ctypes.c_uint32), ("tf_schedule", ctypes.c_uint32),
                ("run_min_row", ctypes.c_uint32)]


_lib = None

SYMBOLS = [
    "mg_build", "mg_info", "mg_quantize", "mg_export_codebook", "mg_export_dag", "mg_export_map", "mg_segment_ids", "mg_upload",
    "mg_device_bytes", "mg_bind_device", "mg_query_nnz_bound",
    "mg_workspace_bytes", "mg_workspace_init", "mg_query_boxes", "mg_query_boxes_plain", "mg_query_boxes_stats",
    "mg_query_boxes_sparse", "mg_query_boxes_noalloc",
    "mg_naive_boxes",
    "mg_check_load_addresses", "mg_footprint", "mg_propagate_tf", "mg_palette_fetch", "mg_box_colour", "mg_lut_build", "mg_export_lut", "mg_query_boxes_lut", "mg_query_boxes_err",
    "mg_get_launch", "mg_set_launch", "mg_autotune",
    "mg_save", "mg_load", "mg_pack", "mg_unpack", "mg_unpack_device", "mg_timing_enable", "mg_timing_read",
    "mg_last_error", "mg_free",
]


def load() -> ctypes.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    # torch first: libmg then binds to the HIP runtime torch loaded; a HIP runtime loaded
    # before torch's leaves torch without devices in the same process
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(LIB_PATH):
        raise ImportError("libmg.so is not built (%s); run `python -m paper_2009_02702_amd.build_ext` "
                          "or __graft_entry__.build()" % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    vp, u32, u64, i32 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int
    G = ctypes.c_void_p
    sig = {
        "mg_build": ([vp, ctypes.POINTER(BuildOpts), ctypes.POINTER(G)], i32),
        "mg_info": ([G, ctypes.POINTER(Info)], i32),
        "mg_quantize": ([G, u32, u32, ctypes.POINTER(G)], i32),
        "mg_export_codebook": ([G, vp, vp, vp, vp], i32),
        "mg_export_dag": ([G, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp], i32),
        "mg_export_map": ([G, u32, vp], i32),
        "mg_segment_ids": ([G, vp], i32),
        "mg_upload": ([G, i32], i32),
        "mg_device_bytes": ([G, ctypes.POINTER(u64)], i32),
        "mg_bind_device": ([G, i32, vp, u64, vp], i32),
        "mg_query_nnz_bound": ([G, vp, u32, vp, vp], i32),
        "mg_workspace_bytes": ([G, u32, ctypes.POINTER(u64)], i32),
        "mg_workspace_init": ([G, vp, u64, vp], i32),
        "mg_query_boxes": ([G, vp, u32, vp, vp, u64, vp], i32),
        "mg_query_boxes_plain": ([G, vp, u32, vp, vp, u64, vp], i32),
        "mg_query_boxes_stats": ([G, vp, u32, vp, vp, vp, u64, vp], i32),
        "mg_query_boxes_sparse": ([G, vp, u32, vp, vp, vp, u32, vp, vp, u64, vp], i32),
        "mg_query_boxes_noalloc": ([G, vp, u32, vp, vp], i32),
        "mg_naive_boxes": ([G, vp, u32, vp, vp, u64, vp], i32),
        "mg_check_load_addresses": ([u32, u32, u32, u32, vp, u32, u32, vp], i32),
        "mg_footprint": ([G, vp, u32, vp, vp, u32, vp, vp], i32),
        "mg_propagate_tf": ([G, vp, u32, vp, vp], i32),
        "mg_palette_fetch": ([G, vp, u32, u32, vp, u32, vp, vp], i32),
        "mg_box_colour": ([G, vp, u32, vp, u32, vp, vp, vp], i32),
        "mg_lut_build": ([G, u32, ctypes.POINTER(u64)], i32),
        "mg_export_lut": ([G, vp, vp, vp, vp], i32),
        "mg_query_boxes_lut": ([G, vp, u32, vp, vp, u64, vp], i32),
        "mg_query_boxes_err": ([G, vp, u32, vp, vp, vp, u64, vp], i32),
        "mg_get_launch": ([G, ctypes.POINTER(LaunchCfg)], i32),
        "mg_set_launch": ([G, ctypes.POINTER(LaunchCfg)], i32),
        "mg_autotune": ([G, vp, u32, vp, vp, u64, u32, vp, ctypes.POINTER(LaunchCfg)], i32),
        "mg_save": ([G, ctypes.c_char_p], i32),
        "mg_load": ([ctypes.c_char_p, ctypes.POINTER(G)], i32),
        "mg_pack": ([G, vp, u64, ctypes.POINTER(u64)], i32),
        "mg_unpack": ([vp, u64, u32, ctypes.POINTER(G)], i32),
        "mg_unpack_device": ([vp, u64, u32, i32, ctypes.POINTER(G)], i32),
        "mg_timing_enable": ([G, i32], i32),
        "mg_timing_read": ([G, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(u32)], i32),
        "mg_last_error": ([], ctypes.c_char_p),
        "mg_free": ([G], None),
    }
    for name in SYMBOLS:
        f = getattr(lib, name)
        f.argtypes, f.restype = sig[name]
    _lib = lib
    return lib


def check(rc: int) -> None:
    if rc != MG_OK:
        msg = load().mg_last_error()
        raise MGError(rc, msg.decode() if msg else "")
