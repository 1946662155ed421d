"""ctypes declarations of the C-ABI in ``include/pf.h`` (argument marshalling
only; every step of the filter runs in the HIP kernels of ``libpf.so``)."""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_char_p, c_double, c_int32, c_uint32, c_uint64, c_void_p

HERE = os.path.dirname(os.path.abspath(__file__))
# PF_LIBRARY may name another build of the same library (e.g. a tuning build)
LIB_PATH = os.environ.get("PF_LIBRARY") or os.path.join(HERE, "libpf.so")

PF_MAX_DIM = 16

PF_OK = 0
PF_E_OOM = -3
PF_E_NUMERIC = -5
STATUS_NAMES = {0: "PF_OK", -1: "PF_E_INVALID", -2: "PF_E_UNSUPPORTED", -3: "PF_E_OOM",
                -4: "PF_E_HIP", -5: "PF_E_NUMERIC", -6: "PF_E_STATE"}
PF_MODEL_LG, PF_MODEL_SV = 0, 1
PF_RESAMPLE_MULTINOMIAL, PF_RESAMPLE_SYSTEMATIC = 0, 1
PF_DTYPE_F32, PF_DTYPE_BF16, PF_DTYPE_F64 = 0, 1, 2

# Every symbol include/pf.h declares.
EXPORTS = ("pf_create", "pf_destroy", "pf_reset", "pf_step", "pf_run", "pf_estimate",
           "pf_history", "pf_get_state", "pf_set_state", "pf_get_ancestors", "pf_info",
           "pf_sync", "pf_status_string", "pf_last_error", "pf_save", "pf_load",
           "pf_batch_create", "pf_batch_destroy", "pf_batch_step", "pf_batch_run",
           "pf_batch_estimates", "pf_batch_filter_info", "pf_batch_tuning", "pf_batch_get_state",
           "pf_batch_set_state", "pf_batch_reset", "pf_batch_sync", "pf_batch_last_error",
           "pf_set_allocator", "pf_batch_estimates_async", "pf_batch_rebind", "pf_run_noalloc")

DPTR = POINTER(c_double)
# pf_set_allocator callbacks: alloc(bytes, ctx) -> device pointer, free_(ptr, ctx)
ALLOC_FN = ctypes.CFUNCTYPE(c_void_p, ctypes.c_size_t, c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, c_void_p, c_void_p)


class PfModel(ctypes.Structure):
    _fields_ = [("kind", c_int32), ("d", c_int32), ("A", DPTR), ("Q_chol", DPTR),
                ("H", DPTR), ("R_chol", DPTR), ("m0", DPTR), ("P0_chol", DPTR),
                ("phi", c_double), ("sigma", c_double), ("beta", c_double)]


class PfConfig(ctypes.Structure):
    _fields_ = [("n_particles", c_uint64), ("radix", c_uint64), ("resampler", c_int32),
                ("state_dtype", c_int32), ("seed", c_uint64), ("stream_id", c_uint32),
                ("history", c_uint32), ("keep_ancestors", c_uint32), ("full_cycle", c_uint32),
                ("island", c_uint32), ("island_swap", c_uint32), ("ess_threshold", c_double)]


class PfEstimate(ctypes.Structure):
    _fields_ = [("t", c_uint32), ("stage", c_uint32), ("radix", c_uint32), ("valid", c_uint32),
                ("log_normaliser", c_double), ("ess", c_double), ("max_log_weight", c_double),
                ("next_offset", c_double), ("mean", c_double * PF_MAX_DIM),
                ("var", c_double * PF_MAX_DIM)]


class PfInfo(ctypes.Structure):
    _fields_ = [("n_particles", c_uint64), ("d", c_uint32), ("n_stages", c_uint32),
                ("radices", c_uint32 * 32), ("global_path", c_uint32), ("state_dtype", c_uint32),
                ("device_bytes", c_uint64), ("t", c_uint32), ("tile_elems", c_uint32 * 32)]


class PfBatchTune(ctypes.Structure):
    _fields_ = [("class_index", c_uint32), ("dim", c_uint32), ("model_kind", c_uint32),
                ("pairs_per_thread", c_uint32), ("radix", c_uint32), ("chosen", c_uint32),
                ("ms_per_step", ctypes.c_float), ("reserved", c_uint32)]


_lib = None


def load():
    """Load ``libpf.so`` (built in-tree). Raises ImportError if it is missing:
    there is no fallback implementation."""
    global _lib
    if _lib is not None:
        return _lib
    try:  # one HIP runtime per process: bind to torch's copy when torch is present
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_1812_01502_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    H = c_void_p
    sig = {
        "pf_create": (c_int32, [POINTER(PfModel), POINTER(PfConfig), c_void_p, POINTER(H)]),
        "pf_destroy": (c_int32, [H]),
        "pf_reset": (c_int32, [H]),
        "pf_step": (c_int32, [H, DPTR]),
        "pf_run": (c_int32, [H, c_void_p, c_uint32, c_uint64, c_int32]),
        "pf_estimate": (c_int32, [H, POINTER(PfEstimate)]),
        "pf_history": (c_int32, [H, POINTER(PfEstimate), c_uint32, POINTER(c_uint32)]),
        "pf_get_state": (c_int32, [H, c_void_p, c_void_p, POINTER(c_uint32), DPTR]),
        "pf_set_state": (c_int32, [H, c_void_p, c_void_p, c_uint32, c_double]),
        "pf_get_ancestors": (c_int32, [H, POINTER(c_uint32)]),
        "pf_info": (c_int32, [H, POINTER(PfInfo)]),
        "pf_sync": (c_int32, [H]),
        "pf_save": (c_int32, [H, c_void_p, c_uint64, POINTER(c_uint64)]),
        "pf_load": (c_int32, [H, c_void_p, c_uint64]),
        "pf_batch_create": (c_int32, [POINTER(PfModel), POINTER(PfConfig), c_uint32, c_void_p,
                                      POINTER(H)]),
        "pf_batch_destroy": (c_int32, [H]),
        "pf_batch_step": (c_int32, [H, c_void_p, c_void_p]),
        "pf_batch_run": (c_int32, [H, c_void_p, c_uint32, c_uint64, c_void_p, c_int32]),
        "pf_batch_estimates": (c_int32, [H, POINTER(PfEstimate)]),
        "pf_batch_filter_info": (c_int32, [H, c_uint32, POINTER(PfInfo)]),
        "pf_batch_tuning": (c_int32, [H, POINTER(PfBatchTune), c_uint32, POINTER(c_uint32)]),
        "pf_batch_get_state": (c_int32, [H, c_uint32, c_void_p, c_void_p, POINTER(c_uint32), DPTR]),
        "pf_batch_set_state": (c_int32, [H, c_uint32, c_void_p, c_void_p, c_uint32, c_double]),
        "pf_batch_reset": (c_int32, [H, c_uint32, c_uint64, c_uint32]),
        "pf_batch_sync": (c_int32, [H]),
        "pf_batch_last_error": (c_char_p, [H]),
        "pf_batch_estimates_async": (c_int32, [H, c_void_p]),
        "pf_batch_rebind": (c_int32, [H, c_uint32, POINTER(c_uint32), POINTER(PfModel), POINTER(PfConfig)]),
        "pf_set_allocator": (c_int32, [ALLOC_FN, FREE_FN, c_void_p]),
        "pf_run_noalloc": (c_int32, [POINTER(PfModel), POINTER(PfConfig), c_void_p, c_void_p, c_void_p, c_uint32,
                                     c_uint64, c_uint32, c_void_p, c_void_p]),
        "pf_status_string": (c_char_p, [c_int32]),
        "pf_last_error": (c_char_p, [H]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib
