"""ctypes mirror of include/libnwmine.h (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libnwmine.so")

NWM_OK, NWM_EINVAL, NWM_ESHAPE, NWM_ENOMEM, NWM_EDEVICE, NWM_EUNSUPPORTED = range(6)
NWM_FP32, NWM_BF16 = 0, 1
STATUS_NAMES = {0: "NWM_OK", 1: "NWM_EINVAL", 2: "NWM_ESHAPE", 3: "NWM_ENOMEM", 4: "NWM_EDEVICE",
                5: "NWM_EUNSUPPORTED"}

# exported symbols declared by include/libnwmine.h
SYMBOLS = ["nwm_create", "nwm_destroy", "nwm_strerror", "nwm_plan_create", "nwm_plan_sizes",
           "nwm_plan_destroy", "nwm_score_pairs", "nwm_align_batch", "nwm_align_backward", "nwm_mine",
           "nwm_plan_set_graph", "nwm_plan_set_param", "nwm_plan_get_param", "nwm_plan_set_timing",
           "nwm_plan_kernel_ms", "nwm_union_kept", "nwm_align_check", "nwm_last_device_error",
           "nwm_align_batch_noalloc"]

PARAMS = {"fill_waves_per_cu": 0, "merge_waves_per_cu": 1, "score_xcd_map": 2, "dp_hot_percent": 3,
          "score_compact": 4, "dp_spin_limit": 5, "dp_test_hold": 6, "score_kgroup": 7,
          "fill_staging": 8, "expand_fused": 9}

P = ctypes.c_void_p


class Dict(ctypes.Structure):
    _fields_ = [("V", ctypes.c_int32), ("max_deg", ctypes.c_int32), ("row_off", P), ("col", P), ("val", P)]


class Scorer(ctypes.Structure):
    _fields_ = [("w0", ctypes.c_float), ("w1", ctypes.c_float), ("b", ctypes.c_float)]


class Batch(ctypes.Structure):
    _fields_ = [("B", ctypes.c_int32), ("V", ctypes.c_int32), ("n_host", P), ("m_host", P),
                ("src_tokens", ctypes.c_int64), ("tgt_tokens", ctypes.c_int64),
                ("max_sent_tokens", ctypes.c_int32),
                ("src_off", P), ("src_tok", P), ("tgt_off", P), ("tgt_tok", P)]


class Sizes(ctypes.Structure):
    _fields_ = [("S_elems", ctypes.c_size_t), ("kept_cap", ctypes.c_size_t), ("tb_bytes", ctypes.c_size_t),
                ("ws_bytes", ctypes.c_size_t)]


class NwmError(RuntimeError):
    def __init__(self, status: int, where: str):
        super().__init__("%s failed: %s" % (where, STATUS_NAMES.get(status, str(status))))
        self.status = status


_lib = None


def load(path: str | None = None):
    """Load libnwmine.so.  Raises if it has not been built: there is no
    fallback path."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    path = path or LIB_PATH
    if not os.path.exists(path):
        raise RuntimeError("libnwmine.so is not built (%s); run `python -m paper_1512_01641_amd.build`" % path)
    lib = ctypes.CDLL(path)
    I = ctypes.c_int
    lib.nwm_create.argtypes = [ctypes.POINTER(P), I]
    lib.nwm_create.restype = I
    lib.nwm_destroy.argtypes = [P]
    lib.nwm_destroy.restype = None
    lib.nwm_strerror.argtypes = [I]
    lib.nwm_strerror.restype = ctypes.c_char_p
    lib.nwm_plan_create.argtypes = [P, ctypes.POINTER(Batch), ctypes.c_int32, I, ctypes.POINTER(P)]
    lib.nwm_plan_create.restype = I
    lib.nwm_plan_sizes.argtypes = [P, ctypes.POINTER(Sizes)]
    lib.nwm_plan_sizes.restype = I
    lib.nwm_plan_destroy.argtypes = [P]
    lib.nwm_plan_destroy.restype = None
    lib.nwm_score_pairs.argtypes = [P, ctypes.POINTER(Batch), ctypes.POINTER(Dict), Scorer, P, P, P, P]
    lib.nwm_score_pairs.restype = I
    lib.nwm_align_batch.argtypes = [P, P, ctypes.c_float, ctypes.c_float, P, P, P, P, P, P, P]
    lib.nwm_align_batch.restype = I
    lib.nwm_align_backward.argtypes = [P, ctypes.POINTER(Batch), P, P, P, P, P, P, P, P, Scorer, P, P, P]
    lib.nwm_align_backward.restype = I
    lib.nwm_mine.argtypes = [P, ctypes.POINTER(Batch), ctypes.POINTER(Dict), Scorer, ctypes.c_float, ctypes.c_float,
                             P, P, P, P, P, P, P, P, P]
    lib.nwm_mine.restype = I
    lib.nwm_plan_set_graph.argtypes = [P, I]
    lib.nwm_plan_set_graph.restype = I
    lib.nwm_plan_set_param.argtypes = [P, I, ctypes.c_int32]
    lib.nwm_plan_set_param.restype = I
    lib.nwm_plan_get_param.argtypes = [P, I, ctypes.POINTER(ctypes.c_int32)]
    lib.nwm_plan_get_param.restype = I
    lib.nwm_plan_set_timing.argtypes = [P, I]
    lib.nwm_plan_set_timing.restype = I
    lib.nwm_plan_kernel_ms.argtypes = [P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int32), I]
    lib.nwm_plan_kernel_ms.restype = I
    lib.nwm_union_kept.argtypes = [P, P, P, P, P, P, P, P]
    lib.nwm_union_kept.restype = I
    lib.nwm_align_check.argtypes = [P, P, ctypes.POINTER(ctypes.c_int32), P]
    lib.nwm_align_check.restype = I
    lib.nwm_align_batch_noalloc.argtypes = [P, P, ctypes.c_float, ctypes.c_float, P, P, P, P, P, P]
    lib.nwm_align_batch_noalloc.restype = I
    lib.nwm_last_device_error.argtypes = []
    lib.nwm_last_device_error.restype = ctypes.c_char_p
    if path == LIB_PATH:
        _lib = lib
    return lib


def check(status: int, where: str):
    if status != NWM_OK:
        if status == NWM_EDEVICE and _lib is not None:
            where = "%s (%s)" % (where, _lib.nwm_last_device_error().decode())
        raise NwmError(status, where)
