"""ctypes binding of libspt.so (the C ABI declared in include/spt.h).

Argument marshalling only: every step of the computation runs in the library's HIP kernels.
Loading fails loudly when the library has not been built; there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libspt.so")

SPT_OK, SPT_EINVAL, SPT_ERANGE, SPT_EHIP, SPT_ESINGULAR = 0, -1, -2, -3, -4
SPT_EWORKSPACE, SPT_EUNSUPPORTED, SPT_ESTATE = -5, -6, -7
SPT_F64, SPT_F32, SPT_BF16 = 0, 1, 2
TUNE_BATCH_CONFIGS, TUNE_NO_ATOMIC, TUNE_NO_PERMUTED = 1, 2, 4
ALGO_AUTO, ALGO_ATOMIC, ALGO_PERMUTED, ALGO_PERMUTED_COPY, ALGO_PRIVATIZED = 0, 1, 2, 3, 4

_c_p = ctypes.c_void_p
_c_i = ctypes.c_int
_c_i64 = ctypes.c_int64
_c_sz = ctypes.c_size_t
_c_d = ctypes.c_double


class SptTune(ctypes.Structure):
    _fields_ = [("algo", ctypes.c_int32), ("lanes_per_nnz", ctypes.c_int32),
                ("cols_per_lane", ctypes.c_int32), ("nnz_per_wave", ctypes.c_int32),
                ("flags", ctypes.c_int32), ("lds_kib", ctypes.c_int32)]


TUNE_DETERMINISTIC = 1
GCP_LOSSES = {"poisson": 0, "bernoulli": 1, "gaussian": 2, "gamma": 3}


# name -> (restype, argtypes); every symbol include/spt.h declares
SIGNATURES = {
    "spt_status_string": (ctypes.c_char_p, [_c_i]),
    "spt_version": (_c_i, []),
    "spt_tensor_workspace_bytes": (_c_sz, [_c_i, _c_p, _c_i64, _c_i]),
    "spt_tensor_create": (_c_i, [_c_p, _c_i, _c_p, _c_i64, _c_p, _c_p, _c_i, _c_p, _c_sz, _c_p]),
    "spt_tensor_create_begin": (_c_i, [_c_p, _c_i, _c_p, _c_i64, _c_i, _c_p, _c_sz, _c_p]),
    "spt_tensor_append": (_c_i, [_c_p, _c_i64, _c_i64, _c_p, _c_p, _c_p]),
    "spt_tensor_validate": (_c_i, [_c_p, _c_p, _c_p]),
    "spt_tensor_status": (_c_i, [_c_p, _c_p]),
    "spt_tensor_permute": (_c_i, [_c_p, _c_i, _c_p]),
    "spt_tensor_perm": (_c_i, [_c_p, _c_i, _c_p, _c_p]),
    "spt_tensor_sorted_copy_bytes": (_c_sz, [_c_p, _c_i, _c_i]),
    "spt_tensor_sort_copy": (_c_i, [_c_p, _c_i, _c_i, _c_p, _c_sz, _c_p]),
    "spt_tensor_drop_sorted_copy": (_c_i, [_c_p, _c_i]),
    "spt_tensor_info": (_c_i, [_c_p, _c_p, _c_p, _c_p, _c_p]),
    "spt_tensor_destroy": (_c_i, [_c_p]),
    "spt_mttkrp": (_c_i, [_c_p, _c_i, _c_i, _c_p, _c_i, _c_p, _c_p, _c_p, _c_p, _c_p]),
    "spt_mttkrp_default_tune": (_c_i, [_c_p, _c_i, _c_i, _c_i, _c_i, _c_p]),
    "spt_cp_workspace_bytes": (_c_sz, [_c_p, _c_i]),
    "spt_cp_gram": (_c_i, [_c_i64, _c_i, _c_p, _c_i, _c_p, _c_p, _c_sz, _c_p]),
    "spt_cp_als_mode": (_c_i, [_c_p, _c_i, _c_i, _c_p, _c_i, _c_p, _c_p, _c_p, _c_sz, _c_p, _c_p]),
    "spt_cp_als_sweep": (_c_i, [_c_p, _c_i, _c_p, _c_i, _c_p, _c_p, _c_p, _c_sz, _c_p, _c_p]),
    "spt_cp_solution": (_c_i, [_c_p, _c_i, _c_p, _c_sz, _c_p]),
    "spt_cp_fit_noalloc": (_c_i, [_c_p, _c_i, _c_p, _c_i, _c_p, _c_p, _c_p, _c_p, _c_p]),
    "spt_cp_fit": (_c_i, [_c_p, _c_i, _c_p, _c_i, _c_p, _c_p, _c_p, _c_sz, _c_p, _c_p, _c_p]),
    "spt_cp_fit_after_mode": (_c_i, [_c_p, _c_i, _c_i, _c_p, _c_i, _c_p, _c_p, _c_p, _c_sz, _c_p,
                                     _c_p, _c_p]),
    "spt_model_values": (_c_i, [_c_p, _c_i, _c_p, _c_i, _c_p, _c_p, _c_p]),
    "spt_gcp_poisson_forward": (_c_i, [_c_p, _c_i, _c_p, _c_i, _c_p, _c_p, _c_p, _c_p, _c_sz,
                                       _c_p]),
    "spt_gcp_poisson_backward": (_c_i, [_c_p, _c_i, _c_p, _c_i, _c_p, _c_p, _c_p, _c_p, _c_p,
                                        _c_p, _c_p]),
    "spt_paper_block_sizes": (_c_i, [_c_i, _c_p, _c_p]),
    "spt_mttkrp_autotune": (_c_i, [_c_p, _c_i, _c_i, _c_p, _c_i, _c_p, _c_i, _c_i, _c_p, _c_p,
                                   _c_p]),
    "spt_batch_workspace_bytes": (_c_sz, [_c_i]),
    "spt_batch_supported_tune": (_c_i, [_c_i, _c_i, _c_i, _c_i, _c_i]),
    "spt_batch_create": (_c_i, [_c_p, _c_i, _c_p, _c_p, _c_p, _c_p, _c_i, _c_p, _c_p, _c_p,
                                _c_sz, _c_p]),
    "spt_batch_launch": (_c_i, [_c_p, _c_p]),
    "spt_batch_info": (_c_i, [_c_p, _c_p, _c_p]),
    "spt_batch_destroy": (_c_i, [_c_p]),
    "spt_gcp_forward": (_c_i, [_c_p, _c_i, _c_p, _c_i, _c_i, _c_p, _c_p, _c_p, _c_p, _c_sz,
                               _c_p]),
    "spt_gcp_backward": (_c_i, [_c_p, _c_i, _c_p, _c_i, _c_i, _c_p, _c_p, _c_p, _c_p, _c_p,
                                _c_p, _c_p]),
    "spt_gcp_fused": (_c_i, [_c_p, _c_i, _c_p, _c_i, _c_i, _c_p, _c_p, _c_p, _c_p, _c_p]),
    "spt_scale_values": (_c_i, [_c_p, _c_p, _c_i64, _c_i, _c_p, _c_p]),
    "spt_gcp_sample": (_c_i, [_c_p, ctypes.c_uint64, _c_i64, _c_i64, _c_i64, _c_p, _c_p, _c_p,
                              _c_i, _c_p]),
    "spt_adam_step": (_c_i, [_c_p, _c_p, _c_p, _c_p, _c_i64, _c_i, ctypes.c_double,
                             ctypes.c_double, ctypes.c_double, ctypes.c_double, _c_i64,
                             ctypes.c_double, _c_p]),
    "spt_f32_to_bf16": (_c_i, [_c_p, _c_p, _c_i64, _c_p]),
    "spt_f64_to_bf16": (_c_i, [_c_p, _c_p, _c_i64, _c_p]),
    "spt_stream_triad": (_c_i, [_c_p, _c_p, _c_p, ctypes.c_float, _c_i64, _c_p]),
}

_lib = None


class SptError(RuntimeError):
    def __init__(self, code, where=""):
        self.code = code
        msg = string(code) if _lib is not None else str(code)
        super().__init__(f"{where}: spt status {code} ({msg})")


class SptUnavailable(ImportError):
    pass


def load():
    """Load libspt.so; raise SptUnavailable (never fall back) if it is missing or incomplete."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise SptUnavailable(
            f"{LIB_PATH} is not built; run __graft_entry__.build() (hipcc, gfx950) first")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        try:
            f = getattr(lib, name)
        except AttributeError as e:
            raise SptUnavailable(f"{LIB_PATH} lacks symbol {name}") from e
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def string(code: int) -> str:
    return load().spt_status_string(int(code)).decode()


def check(code: int, where: str = "") -> None:
    if code != SPT_OK:
        raise SptError(code, where)


def ptr_array(ptrs):
    return (ctypes.c_void_p * len(ptrs))(*[p if p else None for p in ptrs])
