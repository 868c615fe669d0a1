"""ctypes loader of libbp4.so (the HIP library) and its C ABI signatures.

The library is the only compute path: if it cannot be loaded, every call
raises.  There is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
# BP4_SANITIZE=1: the library whose host ABI layer is built with AddressSanitizer and
# UndefinedBehaviorSanitizer (the process must preload clang's ASan runtime)
LIB_PATH = os.path.join(PKG, "libbp4_san.so" if os.environ.get("BP4_SANITIZE") == "1" else "libbp4.so")

BP4_OK = 0
ERRORS = {-1: "EINVAL", -2: "ENONCOMM", -3: "EDEGREE", -4: "EWORKSPACE", -5: "EHIP", -6: "EUNSUPPORTED"}


class BP4Error(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"bp4 {ERRORS.get(code, code)}: {msg}")
        self.code = code
        self.name = ERRORS.get(code, str(code))


class Params(ctypes.Structure):
    _fields_ = [("variant", ctypes.c_int32), ("max_iter", ctypes.c_int32),
                ("stop_on_syndrome", ctypes.c_int32), ("adagrad_g_from_t1", ctypes.c_int32),
                ("alpha", ctypes.c_float), ("gamma", ctypes.c_float),
                ("eps", ctypes.c_float), ("llr_clamp", ctypes.c_float),
                ("alpha_last", ctypes.c_float), ("alpha_steps", ctypes.c_int32), ("serial", ctypes.c_int32)]


class Tuning(ctypes.Structure):
    _fields_ = [("group_lanes", ctypes.c_int32), ("lds_bytes", ctypes.c_int32), ("kernel", ctypes.c_int32),
                ("soa_lanes", ctypes.c_int32), ("soa_iter_block", ctypes.c_int32), ("block_shots", ctypes.c_int32),
                ("gather_waves", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class CodeBatch(ctypes.Structure):
    _fields_ = [("graph", ctypes.c_void_p), ("dev_graph", ctypes.c_void_p), ("params", Params),
                ("shots", ctypes.c_int64), ("prior_llr", ctypes.c_void_p), ("synd", ctypes.c_void_p),
                ("est", ctypes.c_void_p), ("conv", ctypes.c_void_p), ("iters", ctypes.c_void_p),
                ("group_lanes", ctypes.c_int32), ("block_shots", ctypes.c_int32)]


_u8p = ctypes.POINTER(ctypes.c_uint8)
_i32p = ctypes.POINTER(ctypes.c_int32)
_vp = ctypes.c_void_p
_sz = ctypes.c_size_t

# name -> (restype, argtypes); every exported symbol of include/bp4.h is listed here
SIGNATURES = {
    "bp4_graph_create": (ctypes.c_int, [_u8p, _u8p, ctypes.c_int32, ctypes.c_int32, ctypes.c_uint32,
                                        ctypes.POINTER(_vp)]),
    "bp4_graph_set_logicals": (ctypes.c_int, [_vp, _u8p, _u8p, ctypes.c_int32]),
    "bp4_graph_set_coords": (ctypes.c_int, [_vp, _i32p]),
    "bp4_graph_info": (ctypes.c_int, [_vp, _i32p, _i32p, _i32p, _i32p, _i32p]),
    "bp4_graph_device_bytes": (ctypes.c_int, [_vp, ctypes.POINTER(_sz)]),
    "bp4_graph_upload": (ctypes.c_int, [_vp, _vp, _sz, _vp]),
    "bp4_graph_destroy": (None, [_vp]),
    "bp4_graph_edges": (ctypes.c_int, [_vp, _i32p, _i32p]),
    "bp4_workspace_bytes": (ctypes.c_int, [_vp, ctypes.POINTER(Params), ctypes.c_int64,
                                           ctypes.POINTER(_sz)]),
    "bp4_sample": (ctypes.c_int, [_vp, _vp, ctypes.c_int64, ctypes.c_int64,
                                  ctypes.POINTER(ctypes.c_uint32), ctypes.c_uint64, ctypes.c_uint64,
                                  _vp, _vp, _vp]),
    "bp4_decode": (ctypes.c_int, [_vp, _vp, ctypes.POINTER(Params), ctypes.c_int64, _vp, _vp, _vp,
                                  _vp, _vp, _vp, _sz, _vp]),
    "bp4_decode_ex": (ctypes.c_int, [_vp, _vp, ctypes.POINTER(Params), ctypes.POINTER(Tuning),
                                     ctypes.c_int64, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _sz, _vp]),
    "bp4_bookkeep": (ctypes.c_int, [_vp, _vp, ctypes.c_int64, _vp, _vp, _vp, _vp, _vp]),
    "bp4_mixed_workspace_bytes": (ctypes.c_int, [ctypes.c_int32, ctypes.POINTER(_sz)]),
    "bp4_soa_workspace_bytes": (ctypes.c_int, [_vp, ctypes.POINTER(Params), ctypes.c_int64, ctypes.c_int32,
                                               ctypes.POINTER(_sz)]),
    "bp4_gather_workspace_bytes": (ctypes.c_int, [_vp, ctypes.POINTER(Params), ctypes.c_int64, ctypes.c_int32,
                                                  ctypes.POINTER(_sz)]),
    "bp4_lds_layout_bytes": (ctypes.c_int, [_vp, ctypes.POINTER(Params), ctypes.c_int32, ctypes.c_int32,
                                            ctypes.POINTER(_sz)]),
    "bp4_decode_mixed": (ctypes.c_int, [ctypes.c_int32, ctypes.POINTER(CodeBatch), _vp, _sz, _vp]),
    "bp4_decode_mixed_noalloc": (ctypes.c_int, [ctypes.c_int32, ctypes.POINTER(CodeBatch), _vp]),
    "bp4_plain_workspace_bytes": (ctypes.c_int, [_vp, ctypes.POINTER(Params), ctypes.c_int64,
                                                 ctypes.POINTER(_sz)]),
    "bp4_decode_plain": (ctypes.c_int, [_vp, _vp, ctypes.POINTER(Params), ctypes.c_int64, _vp, _vp, _vp,
                                        _vp, _vp, _vp, _sz, _vp, ctypes.POINTER(ctypes.c_int32)]),
    "bp4_prior_llr": (ctypes.c_int, [ctypes.c_int32, _vp, _vp, _vp]),
    "bp4_unrolled_sizes": (ctypes.c_int, [_vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int64,
                                          ctypes.POINTER(_sz), ctypes.POINTER(_sz)]),
    "bp4_unrolled_forward": (ctypes.c_int, [_vp, _vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                            ctypes.c_float, ctypes.c_int64, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _sz,
                                            _vp, _sz, _vp]),
    "bp4_unrolled_backward": (ctypes.c_int, [_vp, _vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                             ctypes.c_float, ctypes.c_int64, _vp, _vp, _vp, _vp, _vp, _vp, _sz, _vp,
                                             _vp, _vp, _sz, _vp]),
    "bp4_last_error": (ctypes.c_char_p, []),
    "bp4_version": (ctypes.c_char_p, []),
}

_lib = None


def load(path: str = LIB_PATH):
    """Load libbp4.so, building it first only if no built library exists."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        from . import build as _build
        _build.build()
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(rc: int) -> None:
    if rc != BP4_OK:
        msg = load().bp4_last_error()
        raise BP4Error(rc, msg.decode() if msg else "")
