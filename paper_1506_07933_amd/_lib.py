"""ctypes loader for libmifft.so (the C ABI of include/mifft.h).

The binding only marshals arguments: every step of a transform runs in the
library's HIP kernels.  There is no fallback: if the library is missing or
does not load, importing the binding raises.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmifft.so")

MIFFT_C2C, MIFFT_R2C = 0, 1
MIFFT_FP32, MIFFT_FP64 = 0, 1
MIFFT_HEURISTIC, MIFFT_TUNE, MIFFT_PLAN_ONLY, MIFFT_BATCH_KERNELS, MIFFT_BATCH_GROUPED = 0, 1, 2, 4, 8
MIFFT_STAGE_Z, MIFFT_STAGE_PACK, MIFFT_STAGE_UNPACK, MIFFT_STAGE_Y = 1, 2, 4, 8
MIFFT_SLAB_Z, MIFFT_SLAB_Y, MIFFT_SLAB_X, MIFFT_SLAB_PACK, MIFFT_SLAB_UNPACK = 1, 2, 4, 8, 16
MIFFT_SLAB_INVERSE = 256
MIFFT_OP_POISSON, MIFFT_OP_LAPLACIAN, MIFFT_OP_HELMHOLTZ, MIFFT_OP_DX, MIFFT_OP_DY, MIFFT_OP_DZ = range(6)
STATUS = {0: "MIFFT_OK", 1: "MIFFT_ERR_INVALID", 2: "MIFFT_ERR_UNSUPPORTED",
          3: "MIFFT_ERR_NOMEM", 4: "MIFFT_ERR_DEVICE", 5: "MIFFT_ERR_BADPLAN"}

# name -> (restype, argtypes); mirrors include/mifft.h
_vp, _cvp, _i, _u, _sz = ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_uint, ctypes.c_size_t
_vpp = ctypes.POINTER(ctypes.c_void_p)
SIGNATURES = {
    "mifft_plan_create": (_i, [_vpp, _i, _i, _i, _i, _i, _u]),
    "mifft_execute_forward": (_i, [_vp, _cvp, _vp, _vp]),
    "mifft_execute_inverse": (_i, [_vp, _cvp, _vp, _vp]),
    "mifft_workspace_bytes": (_sz, [_vp]),
    "mifft_execute_forward_ws": (_i, [_vp, _cvp, _vp, _vp, _vp]),
    "mifft_execute_inverse_ws": (_i, [_vp, _cvp, _vp, _vp, _vp]),
    "mifft_execute_forward_static": (_i, [_vp, _cvp, _vp, _vp]),
    "mifft_plan_destroy": (_i, [_vp]),
    "mifft_last_error": (ctypes.c_char_p, []),
    "mifft_plan_create_pencil": (_i, [_vpp, _i, _i, _i, _i, _i, _i, _i, _u]),
    "mifft_execute_pencil_stages": (_i, [_vp, _u, _vp, _vp, _vp, _vp, _vp]),
    "mifft_plan_create_slab": (_i, [_vpp, _i, _i, _i, _i, _i, _i, _u]),
    "mifft_plan_create_nd": (_i, [_vpp, _i, ctypes.POINTER(ctypes.c_int), _i, _i, _u]),
    "mifft_execute_slab_stages": (_i, [_vp, _u, _cvp, _vp, _vp, _vp, _vp]),
    "mifft_poisson_ws_bytes": (_sz, [_vp]),
    "mifft_poisson_solve": (_i, [_vp, _cvp, _vp, _vp, _vp]),
    "mifft_spectral_apply": (_i, [_vp, _i, ctypes.c_double, _cvp, _vp, _vp, _vp]),
    "mifft_spectral_ws_bytes": (_sz, [_vp]),
    "mifft_spectral_gradient": (_i, [_vp, _cvp, _vp, _vp, _vp, _vp, _vp]),
    "mifft_spectral_divergence": (_i, [_vp, _cvp, _cvp, _cvp, _vp, _vp, _vp]),
    "mifft_batch_create": (_i, [_vpp, _i, ctypes.POINTER(ctypes.c_int), _i, _i, _u]),
    "mifft_batch_execute_forward": (_i, [_vp, _vpp, _vpp, _vp]),
    "mifft_batch_graph_launch": (_i, [_vp, _vpp, _vpp, _vp]),
    "mifft_batch_destroy": (_i, [_vp]),
    "mifft_batch_check": (_i, [_vp, ctypes.POINTER(ctypes.c_int)]),
    "mifft_batch_describe": (_i, [_vp, ctypes.c_char_p, _sz]),
    "mifft_plan_describe": (_i, [_vp, ctypes.c_char_p, _sz]),
    "mifft_profile_begin": (_i, [_vp, _i]),
    "mifft_profile_end": (_i, [_vp, ctypes.POINTER(ctypes.c_float), _i,
                               ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]),
    "mifft_version": (ctypes.c_char_p, []),
    "mifft_variants_describe": (_i, [_i, ctypes.c_char_p, _sz]),
    "mifft_pattern_copy": (_i, [_i, _cvp, _sz, _vp, _sz, _i, _i, _i, ctypes.c_longlong, ctypes.c_longlong,
                                ctypes.c_longlong, ctypes.c_longlong, _i, _i, ctypes.c_uint, _vp]),
    "mifft_copy_reference": (_i, [_cvp, _vp, _sz, ctypes.c_uint, _i, _vp]),
}


class MifftError(RuntimeError):
    def __init__(self, status: int, where: str, message: str):
        self.status = status
        self.status_name = STATUS.get(status, str(status))
        super().__init__("%s: %s (%s)" % (where, message, self.status_name))


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError("libmifft.so is not built: run `python -m paper_1506_07933_amd.build` "
                          "(expected at %s)" % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


lib = _load()


def check(status: int, where: str) -> None:
    if status != 0:
        msg = lib.mifft_last_error()
        raise MifftError(status, where, msg.decode() if msg else "")
