"""ctypes declarations of include/pic.h (argument marshalling only)."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# PIC_LIBPIC names another build of the same library (the sanitized one of
# the CPU test run)
LIB_PATH = os.environ.get("PIC_LIBPIC") or os.path.join(HERE, "libpic.so")

PIC_OK, PIC_E_ARG, PIC_E_SCRATCH, PIC_E_CAPACITY, PIC_E_NONFINITE, PIC_E_TREE, PIC_E_HIP, PIC_E_RANGE, \
    PIC_E_STATE, PIC_E_MEMORY = range(10)
PIT, PIDT = 0, 1
F64, F32_OFFSET = 0, 1

EXPORTS = [
    "pic_tree_create", "pic_tree_destroy", "pic_tree_get_info", "pic_tree_get_instance",
    "pic_tree_leaf_table", "pic_tree_vertex_table", "pic_tree_pidt_table", "pic_tree_upload",
    "pic_status_sync", "pic_status_string", "pic_locate", "pic_gather_push", "pic_scratch_bytes",
    "pic_rebin", "pic_deposit", "pic_stream_push", "pic_profile_enable", "pic_profile_read",
    "pic_tune_set", "pic_tune_get", "pic_step", "pic_profile_only", "pic_convert",
    "pic_tree_tune_set", "pic_tree_tune_get", "pic_deposit_noalloc",
    "pic_free_stream", "pic_leaf_counts", "pic_tree_adapt", "pic_vmax", "pic_stream_step",
]
PERIODIC, REFLECTING = 0, 1   # PIC_PERIODIC, PIC_REFLECTING
NOALLOC_SCRATCH_BYTES = 64 << 20   # PIC_NOALLOC_SCRATCH_BYTES

STATS_LEVELS = 20          # PIC_STATS_LEVELS
STATS_WORDS = 4 + STATS_LEVELS   # pic_rebin_stats: particles, movers, lifts, max_tunnel, lift_hist[]


class TreeInfo(C.Structure):
    _fields_ = [("dim", C.c_int32), ("n_inst", C.c_int32), ("regular", C.c_int32), ("max_level", C.c_int32),
                ("n_leaves", C.c_int64), ("n_vertices", C.c_int64), ("n_pidt", C.c_int64),
                ("n_nodes", C.c_int64), ("device_bytes", C.c_int64)]


class InstanceInfo(C.Structure):
    _fields_ = [("max_level", C.c_int32), ("regular", C.c_int32),
                ("leaf_offset", C.c_int64), ("n_leaves", C.c_int64),
                ("vertex_offset", C.c_int64), ("n_vertices", C.c_int64),
                ("pidt_offset", C.c_int64), ("n_pidt", C.c_int64)]


class Particles(C.Structure):
    _fields_ = [("n", C.c_int64), ("x", C.c_void_p * 3), ("v", C.c_void_p * 3),
                ("off", C.c_void_p * 3), ("u", C.c_void_p * 3), ("inst_start_dev", C.c_void_p)]


class PushParams(C.Structure):
    _fields_ = [("qmdt_dev", C.c_void_p), ("dt_dev", C.c_void_p)]


class KernelTime(C.Structure):
    _fields_ = [("name", C.c_char * 48), ("launches", C.c_int64), ("total_ms", C.c_double)]


class PicError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what}: {status_string(code)} (status {code})")
        self.code = code


_lib = None


def lib():
    """Load libpic.so; fails loudly when the HIP library has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1508_02435_amd.build`")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64, dbl, sz = C.c_void_p, C.c_int32, C.c_int64, C.c_double, C.c_size_t
        L.pic_tree_create.argtypes = [i32, i32, vp, vp, C.POINTER(vp)]
        L.pic_tree_create.restype = i32
        L.pic_tree_destroy.argtypes = [vp]
        L.pic_tree_destroy.restype = None
        L.pic_tree_get_info.argtypes = [vp, C.POINTER(TreeInfo)]
        L.pic_tree_get_info.restype = i32
        L.pic_tree_get_instance.argtypes = [vp, i32, C.POINTER(InstanceInfo)]
        L.pic_tree_get_instance.restype = i32
        L.pic_tree_leaf_table.argtypes = [vp, vp, vp, vp, vp, vp]
        L.pic_tree_leaf_table.restype = i32
        L.pic_tree_vertex_table.argtypes = [vp, vp]
        L.pic_tree_vertex_table.restype = i32
        L.pic_tree_pidt_table.argtypes = [vp, vp, vp, vp]
        L.pic_tree_pidt_table.restype = i32
        L.pic_tree_upload.argtypes = [vp, vp, sz, vp]
        L.pic_tree_upload.restype = i32
        L.pic_status_sync.argtypes = [vp, vp]
        L.pic_status_sync.restype = i32
        L.pic_status_string.argtypes = [i32]
        L.pic_status_string.restype = C.c_char_p
        L.pic_locate.argtypes = [vp, i32, i32, C.POINTER(Particles), vp, vp, vp]
        L.pic_locate.restype = i32
        L.pic_gather_push.argtypes = [vp, i32, i32, C.POINTER(Particles), vp, dbl, dbl,
                                      C.POINTER(PushParams), vp, vp, vp, vp]
        L.pic_gather_push.restype = i32
        L.pic_free_stream.argtypes = [vp, i32, i32, C.POINTER(Particles), dbl, C.POINTER(PushParams), i32, i32,
                                      vp, vp]
        L.pic_free_stream.restype = i32
        L.pic_leaf_counts.argtypes = [vp, C.POINTER(Particles), vp, vp]
        L.pic_leaf_counts.restype = i32
        L.pic_tree_adapt.argtypes = [vp, vp, i64, i32, vp, sz, C.POINTER(C.c_size_t), C.POINTER(C.c_int32)]
        L.pic_tree_adapt.restype = i32
        L.pic_vmax.argtypes = [vp, i32, C.POINTER(Particles), vp, dbl, vp, vp, vp, sz, vp]
        L.pic_vmax.restype = i32
        L.pic_stream_step.argtypes = [vp, i32, C.POINTER(Particles), vp, dbl, i32, i32, i32, vp, vp, vp,
                                      C.POINTER(Particles), vp, vp, sz, vp, vp]
        L.pic_stream_step.restype = i32
        L.pic_scratch_bytes.argtypes = [vp, i64, i32, i32]
        L.pic_scratch_bytes.restype = sz
        L.pic_rebin.argtypes = [vp, i32, i64, vp, vp, i32, vp, vp, vp, vp, vp, sz, vp, vp]
        L.pic_rebin.restype = i32
        L.pic_deposit.argtypes = [vp, i32, i32, C.POINTER(Particles), vp, vp, dbl, vp, vp, sz, vp]
        L.pic_deposit.restype = i32
        L.pic_deposit_noalloc.argtypes = [vp, i32, i32, C.POINTER(Particles), vp, vp, dbl, vp, vp]
        L.pic_deposit_noalloc.restype = i32
        L.pic_stream_push.argtypes = [i32, i64, vp, vp, dbl, vp]
        L.pic_stream_push.restype = i32
        L.pic_profile_enable.argtypes = [i32]
        L.pic_profile_enable.restype = i32
        L.pic_profile_only.argtypes = [C.c_char_p]
        L.pic_profile_only.restype = i32
        L.pic_profile_read.argtypes = [vp, i32]
        L.pic_profile_read.restype = i32
        L.pic_step.argtypes = [vp, i32, i32, C.POINTER(Particles), vp, vp, dbl, dbl, C.POINTER(PushParams), i32,
                               vp, vp, vp, i32, dbl, C.POINTER(Particles), vp, vp, vp, sz, vp, vp]
        L.pic_step.restype = i32
        L.pic_convert.argtypes = [vp, i32, i32, C.POINTER(Particles), dbl, C.POINTER(PushParams), vp, vp, vp]
        L.pic_convert.restype = i32
        L.pic_tune_set.argtypes = [C.c_char_p, i64]
        L.pic_tune_set.restype = i32
        L.pic_tune_get.argtypes = [C.c_char_p]
        L.pic_tune_get.restype = i64
        L.pic_tree_tune_set.argtypes = [vp, C.c_char_p, i64]
        L.pic_tree_tune_set.restype = i32
        L.pic_tree_tune_get.argtypes = [vp, C.c_char_p]
        L.pic_tree_tune_get.restype = i64
        _lib = L
    return _lib


def status_string(code: int) -> str:
    return lib().pic_status_string(int(code)).decode()


def check(code: int, what: str):
    if code != PIC_OK:
        raise PicError(code, what)
