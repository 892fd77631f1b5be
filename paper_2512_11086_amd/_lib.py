"""ctypes binding of libbf (include/bf.h).  Argument marshalling only.

Loading fails loudly (ImportError) when libbf.so has not been built: there is
no fallback implementation anywhere in this package.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
# BF_LIBRARY names another build of the same library (e.g. one with host-code
# sanitizers); the default is the in-tree build.
LIB_PATH = os.environ.get("BF_LIBRARY") or os.path.join(_HERE, "libbf.so")
ABI_VERSION = 8     # the bf.h version these structures and signatures follow

BF_OK = 0
BF_ERR_NULL, BF_ERR_SHAPE = -1, -2
MAX_FRAMES = 4096   # BF_MAX_FRAMES: frames of one bf_das_frames / bf_das_adjoint_frames call
STATUS = {0: "BF_OK", -1: "BF_ERR_NULL", -2: "BF_ERR_SHAPE", -3: "BF_ERR_NOT_HADAMARD",
          -4: "BF_ERR_GEOMETRY", -5: "BF_ERR_UNSUPPORTED", -6: "BF_ERR_TOO_LARGE",
          -7: "BF_ERR_HIP", -8: "BF_ERR_NO_DEVICE", -9: "BF_ERR_STATE"}
MODES = {"forces": 0, "hercules": 1, "tpw": 2, "vls": 3}
INTERPS = {"nearest": 0, "linear": 1, "cubic": 2}
ETYPES = {"f32": 0, "bf16": 1, "i32": 2}
DECODE_ALGOS = {"mfma": 0, "fma": 1}


class BfError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status


class Params(ctypes.Structure):
    _fields_ = [
        ("mode", ctypes.c_int32), ("n_tx", ctypes.c_int32), ("n_ch", ctypes.c_int32),
        ("n_samples", ctypes.c_int32), ("n_elem", ctypes.c_int32 * 2),
        ("pitch", ctypes.c_double * 2), ("xdc_transform", ctypes.c_double * 16),
        ("hadamard", ctypes.POINTER(ctypes.c_int8)),
        ("tx_elements", ctypes.POINTER(ctypes.c_int32)),
        ("channel_map", ctypes.POINTER(ctypes.c_int32)),
        ("fs", ctypes.c_double), ("fc", ctypes.c_double), ("c", ctypes.c_double),
        ("t0", ctypes.c_double), ("focal_depth", ctypes.c_double), ("f_number", ctypes.c_double),
        ("interp", ctypes.c_int32), ("e_type", ctypes.c_int32), ("decode_algo", ctypes.c_int32),
        ("out_dims", ctypes.c_int32 * 3), ("out_min", ctypes.c_double * 3),
        ("out_max", ctypes.c_double * 3), ("iq", ctypes.c_int32),
        ("tx_angles", ctypes.POINTER(ctypes.c_double)),
    ]


IQ_TYPES = {"i16": 0, "f32": 1}


class DemodParams(ctypes.Structure):
    _fields_ = [
        ("n_traces", ctypes.c_int32), ("n_samples", ctypes.c_int32),
        ("decimation", ctypes.c_int32), ("n_taps", ctypes.c_int32),
        ("taps_re", ctypes.POINTER(ctypes.c_double)), ("taps_im", ctypes.POINTER(ctypes.c_double)),
        ("fs", ctypes.c_double), ("fd", ctypes.c_double), ("out_type", ctypes.c_int32),
    ]


class PlanInfo(ctypes.Structure):
    _fields_ = [("n_frames", ctypes.c_int32), ("tile", ctypes.c_int32 * 3),
                ("variant", ctypes.c_int32), ("block", ctypes.c_int32 * 3), ("nb", ctypes.c_int32),
                ("workspace_bytes", ctypes.c_int64), ("e_elems", ctypes.c_int64),
                ("out_elems", ctypes.c_int64), ("channel_groups", ctypes.c_int32)]


class BatchFrameInfo(ctypes.Structure):
    _fields_ = [("das_path", ctypes.c_int32), ("das_class", ctypes.c_int32),
                ("channel_groups", ctypes.c_int32), ("decode_class", ctypes.c_int32),
                ("das_items", ctypes.c_int64)]


BATCH_PATHS = {0: "persistent_lds", 1: "gather", 2: "frame_lds"}

_lib = None


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                          "(there is no non-HIP fallback)")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    P = ctypes.POINTER
    sig = {
        "bf_abi_version": ([], i32),
        "bf_last_error": ([], ctypes.c_char_p),
        "bf_validate": ([P(Params)], ctypes.c_int),
        "bf_plan_create": ([P(Params), P(vp)], ctypes.c_int),
        "bf_plan_create_batch": ([P(Params), i32, P(vp)], ctypes.c_int),
        "bf_plan_destroy": ([vp], ctypes.c_int),
        "bf_plan_get_info": ([vp, P(PlanInfo)], ctypes.c_int),
        "bf_autotune": ([vp, ctypes.c_char_p], ctypes.c_int),
        "bf_set_tile": ([vp, i32, i32, i32], ctypes.c_int),
        "bf_set_das_config": ([vp, i32, i32, i32, i32, i32], ctypes.c_int),
        "bf_decode": ([vp, vp, vp, vp], ctypes.c_int),
        "bf_das": ([vp, vp, vp, dbl, vp], ctypes.c_int),
        "bf_das_noalloc": ([vp, vp, vp, dbl, vp], ctypes.c_int),
        "bf_das_fused": ([vp, vp, vp, dbl, vp], ctypes.c_int),
        "bf_das_adjoint": ([vp, vp, vp, dbl, vp, vp, vp], ctypes.c_int),
        "bf_das_frames": ([vp, vp, i32, vp, dbl, vp], ctypes.c_int),
        "bf_das_adjoint_frames": ([vp, vp, vp, i32, dbl, vp, vp, vp], ctypes.c_int),
        "bf_sharpness": ([vp, i64, i32, vp, vp, vp], ctypes.c_int),
        "bf_batch_run": ([vp, P(vp), P(vp), vp], ctypes.c_int),
        "bf_graph_launch": ([vp, P(vp), P(vp), vp], ctypes.c_int),
        "bf_batch_get_frame_info": ([vp, i32, P(BatchFrameInfo)], ctypes.c_int),
        "bf_test_hann_poly": ([dbl], dbl),
        "bf_test_set_stack_cap": ([vp, i32], ctypes.c_int),
        "bf_demod_create": ([P(DemodParams), P(vp)], ctypes.c_int),
        "bf_demod_destroy": ([vp], ctypes.c_int),
        "bf_demod_out_samples": ([vp, P(i32)], ctypes.c_int),
        "bf_demodulate": ([vp, vp, vp, vp], ctypes.c_int),
        "bf_env_create": ([i64, i32, i32, P(vp)], ctypes.c_int),
        "bf_env_destroy": ([vp], ctypes.c_int),
        "bf_envelope": ([vp, vp, vp, i32, dbl, dbl, vp], ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    if L.bf_abi_version() != ABI_VERSION:
        raise ImportError(f"{LIB_PATH} reports ABI {L.bf_abi_version()}, the binding "
                          f"follows ABI {ABI_VERSION}: rebuild libbf")
    _lib = L
    return L


def check(status: int) -> None:
    if status != BF_OK:
        raise BfError(status, lib().bf_last_error().decode(errors="replace"))


EXPORTED = ("bf_abi_version", "bf_last_error", "bf_validate", "bf_plan_create",
            "bf_plan_create_batch", "bf_plan_destroy", "bf_plan_get_info", "bf_autotune",
            "bf_set_tile", "bf_set_das_config", "bf_decode", "bf_das", "bf_das_noalloc",
            "bf_das_fused", "bf_das_adjoint",
            "bf_das_frames", "bf_das_adjoint_frames", "bf_sharpness",
            "bf_batch_run", "bf_graph_launch", "bf_batch_get_frame_info", "bf_demod_create",
            "bf_demod_destroy", "bf_demod_out_samples", "bf_demodulate", "bf_env_create",
            "bf_env_destroy", "bf_envelope")
TEST_HOOKS = ("bf_test_hann_poly", "bf_test_set_stack_cap")   # include/bf_test.h
COMPRESS = {"none": 0, "log": 1, "power": 2}
VARIANTS = {"lds": 0, "gather": 1, "lds2": 2}   # BF_DAS_LDS, BF_DAS_GATHER, BF_DAS_LDS_Z2
