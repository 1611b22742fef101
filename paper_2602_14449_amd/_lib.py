"""ctypes loader for libtho.so (the HIP library).  No fallback: if the shared
library is missing or fails to load, importing the package raises."""

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtho.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        "libtho.so not found at %s; build it first with "
        "`python paper_2602_14449_amd/build.py`" % LIB_PATH)

lib = ctypes.CDLL(LIB_PATH)

c_i32 = ctypes.c_int32
c_i64 = ctypes.c_int64
c_vp = ctypes.c_void_p
c_sz = ctypes.c_size_t


class Opts(ctypes.Structure):
    _fields_ = [("p_choice", c_i32), ("panel", c_i32), ("flags", c_i32),
                ("reserved", c_i32)]


def _proto(name, restype, argtypes):
    f = getattr(lib, name)
    f.restype = restype
    f.argtypes = argtypes
    return f


tho_version = _proto("tho_version", ctypes.c_char_p, [])
tho_last_error = _proto("tho_last_error", ctypes.c_char_p, [])
tho_strerror = _proto("tho_strerror", ctypes.c_char_p, [ctypes.c_int])
tho_two_stage_workspace = _proto(
    "tho_two_stage_workspace", ctypes.c_int,
    [c_i32, c_i64, c_i64, c_i64, ctypes.POINTER(Opts), ctypes.POINTER(c_sz)])
tho_two_stage = _proto(
    "tho_two_stage", ctypes.c_int,
    [c_i32, c_i64, c_i64, c_i64, c_vp, c_i64, c_vp, c_i64, c_vp, c_i64, c_vp,
     c_i64, c_vp, c_i64, ctypes.POINTER(Opts), c_vp, c_sz, c_vp])
tho_two_stage_noalloc = _proto(
    "tho_two_stage_noalloc", ctypes.c_int,
    [c_i32, c_i64, c_i64, c_i64, c_vp, c_i64, c_vp, c_i64, c_vp, c_i64, c_vp,
     c_i64, c_vp, c_i64, ctypes.POINTER(Opts), c_vp])
NOALLOC_SCRATCH_BYTES = 256 << 20
tho_block_householder_workspace = _proto(
    "tho_block_householder_workspace", ctypes.c_int,
    [c_i32, c_i64, c_i64, ctypes.POINTER(Opts), ctypes.POINTER(c_sz)])
tho_block_householder = _proto(
    "tho_block_householder", ctypes.c_int,
    [c_i32, c_i64, c_i32, ctypes.POINTER(c_i64), c_vp, c_i64, c_vp, c_i64, c_vp, c_i64,
     ctypes.POINTER(Opts), c_vp, c_sz, c_vp])
tho_block_householder_step = _proto(
    "tho_block_householder_step", ctypes.c_int,
    [c_i32, c_i64, c_i32, ctypes.POINTER(c_i64), c_i64, c_vp, c_i64, c_vp, c_i64, c_vp, c_i64,
     ctypes.POINTER(Opts), c_vp, c_sz, c_vp])
tho_two_stage_weighted_workspace = _proto(
    "tho_two_stage_weighted_workspace", ctypes.c_int,
    [c_i32, c_i64, c_i64, c_i64, ctypes.POINTER(Opts), ctypes.POINTER(c_sz)])
tho_two_stage_weighted = _proto(
    "tho_two_stage_weighted", ctypes.c_int,
    [c_i32, c_i64, c_i64, c_i64, c_vp, c_vp, c_i64, c_vp, c_i64, c_vp, c_i64, c_vp,
     c_i64, c_vp, c_i64, ctypes.POINTER(Opts), c_vp, c_sz, c_vp])
tho_get_info = _proto("tho_get_info", ctypes.c_int, [c_vp, ctypes.POINTER(c_i32)])
CHECK_FINITE = 1
CHECK_VORTH = 2
INFO_NONFINITE = 1
INFO_V_NOT_ORTHONORMAL = 3

tho_hhqr_full_workspace = _proto(
    "tho_hhqr_full_workspace", ctypes.c_int,
    [c_i32, c_i64, c_i64, c_i64, ctypes.POINTER(Opts), ctypes.POINTER(c_sz)])
tho_hhqr_full = _proto(
    "tho_hhqr_full", ctypes.c_int,
    [c_i32, c_i64, c_i64, c_i64, c_vp, c_i64, c_vp, c_i64, c_vp, c_i64, c_vp,
     c_i64, c_vp, c_i64, ctypes.POINTER(Opts), c_vp, c_sz, c_vp])
tho_bcgs_workspace = _proto(
    "tho_bcgs_workspace", ctypes.c_int,
    [c_i32, c_i64, c_i64, c_i64, c_i32, c_i32, ctypes.POINTER(Opts), ctypes.POINTER(c_sz)])
tho_bcgs = _proto(
    "tho_bcgs", ctypes.c_int,
    [c_i32, c_i64, c_i64, c_i64, c_vp, c_i64, c_vp, c_i64, c_vp, c_i64, c_vp,
     c_i64, c_vp, c_i64, c_i32, c_i32, ctypes.POINTER(Opts), c_vp, c_sz, c_vp])
tho_two_stage_backward_workspace = _proto(
    "tho_two_stage_backward_workspace", ctypes.c_int,
    [c_i32, c_i64, c_i64, c_i64, ctypes.POINTER(Opts), ctypes.POINTER(c_sz)])
tho_two_stage_backward = _proto(
    "tho_two_stage_backward", ctypes.c_int,
    [c_i32, c_i64, c_i64, c_i64, c_vp, c_i64, c_vp, c_i64, c_vp, c_i64, c_vp, c_i64,
     c_vp, c_i64, c_vp, c_i64, c_vp, c_i64, c_vp, c_i64, c_vp, c_i64,
     ctypes.POINTER(Opts), c_vp, c_sz, c_vp])

class Problem(ctypes.Structure):
    _fields_ = [("n", c_i64), ("k0", c_i64), ("k", c_i64),
                ("V", c_vp), ("ldv", c_i64), ("A", c_vp), ("lda", c_i64),
                ("Q", c_vp), ("ldq", c_i64), ("R", c_vp), ("ldr", c_i64),
                ("S", c_vp), ("lds", c_i64)]


tho_batched_workspace = _proto(
    "tho_batched_workspace", ctypes.c_int,
    [c_i32, ctypes.POINTER(Problem), ctypes.POINTER(Opts), ctypes.POINTER(c_sz)])
tho_batched_plan_create = _proto(
    "tho_batched_plan_create", ctypes.c_int,
    [c_i32, ctypes.POINTER(Problem), c_vp, c_sz, ctypes.POINTER(Opts), c_vp, ctypes.POINTER(c_vp)])
tho_batched_run = _proto("tho_batched_run", ctypes.c_int, [c_vp, c_vp])
tho_batched_plan_info = _proto(
    "tho_batched_plan_info", ctypes.c_int,
    [c_vp, ctypes.POINTER(c_i32), ctypes.POINTER(c_i32), ctypes.POINTER(ctypes.c_double)])
tho_plan_destroy = _proto("tho_plan_destroy", ctypes.c_int, [c_vp])

EXPORTED = ["tho_version", "tho_last_error", "tho_strerror",
            "tho_two_stage_workspace", "tho_two_stage", "tho_two_stage_noalloc", "tho_get_info",
            "tho_block_householder_workspace", "tho_block_householder", "tho_block_householder_step",
            "tho_two_stage_weighted_workspace", "tho_two_stage_weighted",
            "tho_hhqr_full_workspace", "tho_hhqr_full",
            "tho_bcgs_workspace", "tho_bcgs",
            "tho_two_stage_backward_workspace", "tho_two_stage_backward",
            "tho_batched_workspace", "tho_batched_plan_create", "tho_batched_run",
            "tho_batched_plan_info", "tho_plan_destroy"]

THO_F64 = 0
THO_C128 = 1
PANELS = {"fp64": 0, "f32x2": 1, "bf16": 2}
PCHOICES = {"qr": 0, "mlu": 1, "polar": 2}


class ThoError(RuntimeError):
    pass


def check(rc, what):
    if rc != 0:
        msg = tho_last_error().decode(errors="replace")
        raise ThoError("%s failed (%d: %s): %s" % (
            what, rc, tho_strerror(rc).decode(), msg))

tho_profile_enable = _proto("tho_profile_enable", ctypes.c_int, [ctypes.c_int])
tho_profile_collect = _proto("tho_profile_collect", ctypes.c_int, [])
tho_profile_reset = _proto("tho_profile_reset", ctypes.c_int, [])
tho_profile_get = _proto("tho_profile_get", ctypes.c_int,
                         [ctypes.c_int, ctypes.c_char_p, ctypes.c_int,
                          ctypes.POINTER(ctypes.c_double), ctypes.POINTER(c_i64)])
EXPORTED += ["tho_profile_enable", "tho_profile_collect", "tho_profile_reset",
             "tho_profile_get"]


def profile_read():
    """Collect recorded kernel timings: {name: (total_ms, launches)}."""
    n = tho_profile_collect()
    if n < 0:
        check(n, "tho_profile_collect")
    out = {}
    buf = ctypes.create_string_buffer(64)
    for i in range(n):
        ms = ctypes.c_double(0)
        cnt = c_i64(0)
        check(tho_profile_get(i, buf, 64, ctypes.byref(ms), ctypes.byref(cnt)), "tho_profile_get")
        out[buf.value.decode()] = (ms.value, cnt.value)
    return out
