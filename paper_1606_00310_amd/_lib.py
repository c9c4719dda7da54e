"""ctypes binding of libsca.so (include/sca.h): argument marshalling only.

The library is loaded after torch so that both use the same HIP runtime.  There
is no fallback: if libsca.so is missing or fails to load, every call raises.
"""
from __future__ import annotations

import ctypes
import os

import torch  # noqa: F401  (loads the HIP runtime the library links against)

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsca.so")

SCA_OK, SCA_EINVAL, SCA_ENOMEM, SCA_EDEVICE, SCA_EOVERFLOW, SCA_ESTATE, SCA_EBUSY, SCA_ENOBUF = 0, -1, -2, -3, -4, -5, -6, -7
SCA_ESCRATCH = -8
SCA_NOALLOC_MAX_Y = 131072
SCA_FORCE_PERSITE = 1
SCA_STEP_GRAPH = 2
SCA_NO_FUSE = 4
SCA_AUX_LEN = 8
SCA_PATH_DRAWFREE, SCA_PATH_MASK, SCA_PATH_PERSITE = 0, 1, 2


class ScaError(RuntimeError):
    def __init__(self, code: int, what: str):
        self.code = code
        super().__init__(f"{what}: {_strerror(code)} ({code})")


class Req(ctypes.Structure):
    """sca_req: one realization of an ensemble."""
    _fields_ = [("X", ctypes.c_int64), ("Y", ctypes.c_int64), ("p", ctypes.c_double), ("q", ctypes.c_double),
                ("n_mcs", ctypes.c_int64), ("seed", ctypes.c_uint64), ("flags", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32)]


class BatchConfig(ctypes.Structure):
    """sca_batch_config: launch shape and schedule of the persistent kernel."""
    _fields_ = [("block_threads", ctypes.c_int32), ("blocks_per_cu", ctypes.c_int32),
                ("lds_bytes", ctypes.c_int32), ("order", ctypes.c_int32), ("words_per_lane", ctypes.c_int32),
                ("depth", ctypes.c_int32), ("max_parts", ctypes.c_int32)]

    def as_dict(self):
        return {f: int(getattr(self, f)) for f, _ in self._fields_}


class StepPlan(ctypes.Structure):
    """sca_step_plan: the launches sca_step_ex would enqueue."""
    _fields_ = [("path", ctypes.c_int32), ("depth", ctypes.c_int32), ("band", ctypes.c_int32),
                ("tail1", ctypes.c_int32), ("tail2", ctypes.c_int32), ("n_pass", ctypes.c_int64),
                ("n_unfused", ctypes.c_int64), ("kernel", ctypes.c_char * 80), ("tail_kernel", ctypes.c_char * 80),
                ("halfstep_kernel", ctypes.c_char * 80)]

    def as_dict(self):
        return {f: (getattr(self, f).decode() if isinstance(getattr(self, f), bytes) else int(getattr(self, f)))
                for f, _ in self._fields_}


class SlotInfo(ctypes.Structure):
    _fields_ = [("X", ctypes.c_int64), ("Y", ctypes.c_int64), ("t", ctypes.c_int64), ("n_mcs", ctypes.c_int64),
                ("seed", ctypes.c_uint64), ("slopes_dev", ctypes.c_void_p), ("h0_dev", ctypes.c_void_p)]


_lib = None
_vp, _i64, _u64, _u32, _int, _dbl = (ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint64, ctypes.c_uint32,
                                      ctypes.c_int, ctypes.c_double)
_i64p = ctypes.POINTER(ctypes.c_int64)
_dblp = ctypes.POINTER(ctypes.c_double)

_SIGNATURES = {
    "sca_state_words": ([_i64, _i64], ctypes.c_size_t),
    "sca_strerror": ([_int], ctypes.c_char_p),
    "sca_init": ([ctypes.POINTER(_vp), _i64, _i64, _u64, _vp, _vp, _vp], _int),
    "sca_step": ([_vp, _i64, _dbl, _dbl], _int),
    "sca_step_ex": ([_vp, _i64, _dbl, _dbl, ctypes.c_uint], _int),
    "sca_heights": ([_vp, _i64, _i64, _vp], _int),
    "sca_roughness": ([_vp, _i64p, _dblp], _int),
    "sca_roughness_noalloc": ([_vp, _vp, _i64, _i64, _vp, _i64p, _dblp], _int),
    "sca_snapshot_bytes": ([_vp], ctypes.c_size_t),
    "sca_snapshot": ([_vp, _vp], _int),
    "sca_autocorr": ([_vp, _vp, _i64p, _dblp], _int),
    "sca_get_meta": ([_vp, _i64p, _i64p], _int),
    "sca_set_time": ([_vp, _i64], _int),
    "sca_plan_step": ([_vp, _i64, _dbl, _dbl, ctypes.c_uint, ctypes.POINTER(StepPlan)], _int),
    "sca_set_pass_buffer": ([_vp, _vp, ctypes.c_size_t], _int),
    "sca_reset": ([_vp], _int),
    "sca_restore": ([_vp, _vp, _i64], _int),
    "sca_set_blocking": ([_vp, ctypes.c_int32, ctypes.c_int32], _int),
    "sca_debug_halfstep": ([_vp, _int, _vp, _vp], _int),
    "sca_debug_philox": ([_vp, _u32, _u32, _i64, _vp, _vp], _int),
    "sca_debug_philox_rate": ([_i64, ctypes.c_int32, _vp, _vp], _int),
    "sca_destroy": ([_vp], None),
    "sca_batch_state_bytes": ([_i64, _i64], ctypes.c_size_t),
    "sca_batch_create": ([ctypes.POINTER(_vp), ctypes.c_int32, _vp, ctypes.c_size_t, _vp], _int),
    "sca_batch_set_config": ([_vp, ctypes.POINTER(BatchConfig)], _int),
    "sca_batch_get_config": ([_vp, ctypes.POINTER(BatchConfig)], _int),
    "sca_batch_admit": ([_vp, ctypes.POINTER(Req), ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)], _int),
    "sca_batch_run": ([_vp, _i64, ctypes.POINTER(ctypes.c_int32)], _int),
    "sca_batch_run_work": ([_vp, _i64, ctypes.POINTER(ctypes.c_int32)], _int),
    "sca_batch_slot": ([_vp, ctypes.c_int32, ctypes.POINTER(SlotInfo)], _int),
    "sca_batch_roughness": ([_vp, ctypes.c_int32, _i64p, _dblp], _int),
    "sca_batch_release": ([_vp, ctypes.c_int32], _int),
    "sca_batch_destroy": ([_vp], None),
}


def lib():
    """The loaded library; raises if it was not built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1606_00310_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in _SIGNATURES.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def _strerror(code: int) -> str:
    try:
        return lib().sca_strerror(code).decode()
    except Exception:  # pragma: no cover - library not loadable
        return "status"


def check(code: int, what: str):
    if code != SCA_OK:
        raise ScaError(code, what)
