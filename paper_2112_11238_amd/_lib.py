"""ctypes loader for libkp.so and the C-ABI descriptor structs of include/kp.h.

torch is imported before the library is opened so that the process has a
single HIP runtime (torch's); libkp.so then binds to it by soname.
The product path has no fallback: if the library is missing, importing the
package's ops raises.
"""
from __future__ import annotations

import ctypes
import os

import torch  # noqa: F401  (must precede the CDLL: one HIP runtime per process)

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libkp.so")

KP_MAX_ORDER = 8
KP_F64, KP_F32 = 0, 1
KP_PREC_NATIVE, KP_PREC_BF16X3, KP_PREC_BF16X6 = 0, 3, 6
KP_OPT_FUSE = 1

STATUS = {
    0: "KP_OK", -1: "KP_ERR_NULL", -2: "KP_ERR_ORDER", -3: "KP_ERR_MODE",
    -4: "KP_ERR_SHAPE", -5: "KP_ERR_DTYPE", -6: "KP_ERR_ALIAS",
    -7: "KP_ERR_WORKSPACE", -8: "KP_ERR_HIP", -9: "KP_ERR_VALUE", -10: "KP_ERR_SCRATCH",
}


class KpTensor(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int32), ("dtype", ctypes.c_int32),
                ("dims", ctypes.c_int64 * KP_MAX_ORDER), ("data", ctypes.c_void_p)]


class KpMatrix(ctypes.Structure):
    _fields_ = [("rows", ctypes.c_int64), ("cols", ctypes.c_int64),
                ("rs", ctypes.c_int64), ("cs", ctypes.c_int64),
                ("dtype", ctypes.c_int32), ("pad_", ctypes.c_int32),
                ("data", ctypes.c_void_p)]


class KpBatchItem(ctypes.Structure):
    _fields_ = [("T", KpTensor), ("S", KpTensor), ("L", KpMatrix * KP_MAX_ORDER),
                ("G", KpTensor), ("dT", KpTensor), ("dL", KpMatrix * KP_MAX_ORDER)]


class KpTuneEntry(ctypes.Structure):
    _fields_ = [("form", ctypes.c_int32), ("pad0_", ctypes.c_int32),
                ("Il", ctypes.c_int64), ("m", ctypes.c_int64), ("n", ctypes.c_int64),
                ("Ir", ctypes.c_int64),
                ("nb", ctypes.c_int32), ("fb", ctypes.c_int32), ("bk", ctypes.c_int32),
                ("occ", ctypes.c_int32), ("pf", ctypes.c_int32), ("kind", ctypes.c_int32)]


class KpError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        name = STATUS.get(status, str(status))
        msg = f"{where}: {name}"
        if status == -8 and _lib is not None:
            msg += f" (hipError {_lib.kp_last_hip_error()})"
        super().__init__(msg)


P = ctypes.POINTER
_T, _M, _V, _S = P(KpTensor), P(KpMatrix), ctypes.c_void_p, ctypes.c_size_t
_MA = P(P(KpMatrix))

# name -> (restype, argtypes); mirrors include/kp.h
SIGNATURES = {
    "kp_mump": (ctypes.c_int, [_T, _M, ctypes.c_int, _T, ctypes.c_int, ctypes.c_int, _V]),
    "kp_kronsum": (ctypes.c_int, [_T, _MA, _T, ctypes.c_int, _V]),
    "kp_tucker_workspace": (_S, [_T, _MA, ctypes.c_int]),
    "kp_tucker_cache_size": (_S, [_T, _MA]),
    "kp_tucker_order": (ctypes.c_int, [_T, _MA, P(ctypes.c_int), P(ctypes.c_int)]),
    "kp_tucker": (ctypes.c_int, [_T, _MA, _T, ctypes.c_int, _V, _S, _V, _S, _V]),
    "kp_noalloc_scratch_bytes": (_S, []),
    "kp_tucker_noalloc": (ctypes.c_int, [_T, _MA, _T, ctypes.c_int, _V]),
    "kp_tucker_complex_workspace": (_S, [_T, _MA, _MA, ctypes.c_int, ctypes.c_int]),
    "kp_tucker_complex": (ctypes.c_int, [_T, _MA, _MA, _T, ctypes.c_int, ctypes.c_int, _V, _S,
                                         _V]),
    "kp_tucker_backward_workspace": (_S, [_T, _MA, ctypes.c_int]),
    "kp_tucker_backward": (ctypes.c_int, [_T, _T, _MA, _V, _S, _T, _MA, ctypes.c_int,
                                          _V, _S, _V]),
    "kp_expm_workspace": (_S, [ctypes.c_int64, ctypes.c_int64]),
    "kp_expm_f64": (ctypes.c_int, [_V, ctypes.c_int64, ctypes.c_int64, ctypes.c_double, _V, _V,
                                   _S, _V]),
    "kp_tridiag_inverse_f64": (ctypes.c_int, [_V, _V, _V, ctypes.c_int64, ctypes.c_int64,
                                              ctypes.c_double, ctypes.c_double, _V, _V]),
    "kp_pcg_workspace": (_S, [_T, _MA]),
    "kp_pcg_kronsum": (ctypes.c_int, [_T, _MA, _MA, _T, ctypes.c_double, ctypes.c_int, _V, _S,
                                      P(ctypes.c_int), P(ctypes.c_double), _V]),
    "kp_semilinear_workspace": (_S, [ctypes.c_int, P(ctypes.c_int64)]),
    "kp_semilinear_imex_f64": (ctypes.c_int, [_T, P(_V), P(_V), P(_V), P(ctypes.c_double),
                                              ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                              ctypes.c_double, ctypes.c_int, ctypes.c_int, _V, _S,
                                              P(ctypes.c_int), _V]),
    "kp_batch_workspace": (_S, [ctypes.c_int, P(KpBatchItem), ctypes.c_int]),
    "kp_batch_plan_bytes": (_S, [ctypes.c_int, P(KpBatchItem), ctypes.c_int]),
    "kp_batch_plan": (ctypes.c_int, [ctypes.c_int, P(KpBatchItem), ctypes.c_int, _V, _S, _V, _S]),
    "kp_batch_info": (ctypes.c_int, [_V, P(ctypes.c_int64), P(ctypes.c_int), P(ctypes.c_int)]),
    "kp_tucker_batched": (ctypes.c_int, [_V, _V, _V, _S, _V]),
    "kp_force_tile": (ctypes.c_int, [ctypes.c_int] * 6),
    "kp_tune_set": (ctypes.c_int, [P(KpTuneEntry)]),
    "kp_tune_lookup": (ctypes.c_int, [ctypes.c_int, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
                                      ctypes.c_int64, P(KpTuneEntry)]),
    "kp_tune_count": (ctypes.c_int, []),
    "kp_tune_list": (ctypes.c_int, [P(KpTuneEntry), ctypes.c_int]),
    "kp_tune_clear": (ctypes.c_int, []),
    "kp_tucker_products": (ctypes.c_int, [_T, _MA, ctypes.c_int, ctypes.c_int, P(KpTuneEntry),
                                          ctypes.c_int]),
    "kp_tile_variants": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, P(ctypes.c_int32),
                                        ctypes.c_int]),
    "kp_set_option": (ctypes.c_int, [ctypes.c_int, ctypes.c_int]),
    "kp_get_option": (ctypes.c_int, [ctypes.c_int]),
    "kp_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "kp_version": (ctypes.c_int, []),
    "kp_last_hip_error": (ctypes.c_int, []),
}

_lib = None


def load(path=None):
    """Open libkp.so and declare its prototypes. Raises if it is missing.
    KP_LIBRARY in the environment names another build of the same library
    (the host-sanitizer build used by the host-side tests)."""
    global _lib
    if _lib is not None:
        return _lib
    if path is None:
        path = os.environ.get("KP_LIBRARY") or LIB_PATH
    if not os.path.exists(path):
        raise ImportError(
            f"{path} is missing: build it with `python -m paper_2112_11238_amd.build` "
            "(hipcc, gfx950). There is no CPU fallback.")
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        if not hasattr(lib, name):
            continue
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(status, where):
    if status != 0:
        raise KpError(status, where)
