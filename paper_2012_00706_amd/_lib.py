"""ctypes bindings of libmpid.so (the C ABI of include/mpid.h).

Loading fails loudly when the library has not been built: there is no
fallback implementation.
"""
from __future__ import annotations

import ctypes
import os
import re

PKG_DIR = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG_DIR, "libmpid.so")
HEADER = os.path.join(os.path.dirname(PKG_DIR), "include", "mpid.h")


class IdOpts(ctypes.Structure):
    _fields_ = [
        ("prec", ctypes.c_int32),
        ("rank_rule", ctypes.c_int32),
        ("k_fixed", ctypes.c_int64),
        ("rel_tol", ctypes.c_double),
        ("k_max", ctypes.c_int64),
        ("nb", ctypes.c_int32),
        ("flags", ctypes.c_int32),
    ]


class IdProfile(ctypes.Structure):
    _fields_ = [
        ("sweep_launches", ctypes.c_int64),
        ("sweep_ms", ctypes.c_double),
        ("sweep_bytes", ctypes.c_double),
        ("finalize_launches", ctypes.c_int64),
        ("finalize_ms", ctypes.c_double),
        ("gemm_launches", ctypes.c_int64),
        ("gemm_ms", ctypes.c_double),
        ("gemm_bytes", ctypes.c_double),
        ("other_ms", ctypes.c_double),
        ("total_ms", ctypes.c_double),
    ]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class IdBatchItem(ctypes.Structure):
    _fields_ = [
        ("A", ctypes.c_void_p),
        ("m", ctypes.c_int64),
        ("n", ctypes.c_int64),
        ("lda", ctypes.c_int64),
        ("work", ctypes.c_void_p),
        ("perm", ctypes.c_void_p),
        ("R", ctypes.c_void_p),
        ("ldr", ctypes.c_int64),
        ("T", ctypes.c_void_p),
        ("ldt", ctypes.c_int64),
        ("k", ctypes.c_int64),
        ("info", ctypes.c_int32),
        ("groups", ctypes.c_int32),
    ]


def _constants():
    """#define ID_* integer constants parsed from the public header."""
    out = {}
    with open(HEADER) as f:
        for line in f:
            m = re.match(r"#define\s+(ID_\w+)\s+\(?(-?\d+)\)?", line)
            if m:
                out[m.group(1)] = int(m.group(2))
    return out


C = _constants()

_vp = ctypes.c_void_p
_i32, _i64, _f64, _sz = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_size_t
_P = ctypes.POINTER

SIGNATURES = {
    "id_workspace_size": (_sz, [_i64, _i64, _i32, _P(IdOpts)]),
    "id_factor": (ctypes.c_int, [_vp, _i32, _i64, _i64, _i64, _P(IdOpts), _vp, _sz, _vp, _vp, _i64,
                                 _P(_i64), _P(_i32), _vp]),
    "id_noalloc_scratch_bytes": (_sz, []),
    "id_factor_noalloc": (ctypes.c_int, [_vp, _i32, _i64, _i64, _i64, _P(IdOpts), _vp, _vp, _i64,
                                         _P(_i64), _P(_i32), _vp]),
    "id_solve_T": (ctypes.c_int, [_vp, _i64, _i64, _i64, _vp, _i64, _vp, _vp]),
    "id_round": (ctypes.c_int, [_vp, _i64, _i64, _i64, _i32, _vp]),
    "id_reconstruct": (ctypes.c_int, [_vp, _i32, _i64, _i64, _i64, _vp, _i64, _vp, _i64, _vp,
                                      _i64, _i32, _vp]),
    "id_backward_workspace_size": (_sz, [_i64, _i64, _i64]),
    "id_backward": (ctypes.c_int, [_vp, _i32, _i64, _i64, _i64, _vp, _i64, _vp, _i64, _vp, _i64,
                                   _vp, _i64, _vp, _i64, _vp, _i64, _vp, _sz, _P(_i32), _vp]),
    "id_sketch_workspace_size": (_sz, [_i64, _i64, _i64]),
    "id_sketch": (ctypes.c_int, [_vp, _i32, _i64, _i64, _i64, _vp, _i64, _i64, _vp, _i64, _vp,
                                 _sz, _vp]),
    "id_batch_item_workspace_size": (_sz, [_i64, _i64, _P(IdOpts)]),
    "id_factor_batched": (ctypes.c_int, [_vp, _i32, _vp, _i32, _vp, _i64, _i32, _P(IdOpts), _i32,
                                         _i32, _vp]),
    "id_lockstep_workspace_size": (_sz, [_P(IdBatchItem), _i32, _i32, _P(IdOpts)]),
    "id_factor_lockstep": (ctypes.c_int, [_P(IdBatchItem), _i32, _i32, _P(IdOpts), _vp, _sz, _vp]),
    "id_last_profile": (ctypes.c_int, [_P(IdProfile)]),
    "id_status_string": (ctypes.c_char_p, [ctypes.c_int]),
}

_lib = None


def load():
    """The loaded library (raises if it is missing)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"{LIB_PATH} is not built; run paper_2012_00706_amd.build.build_library() "
                "(hipcc, gfx950) first -- there is no fallback path")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


class MpidError(RuntimeError):
    def __init__(self, code, where):
        msg = load().id_status_string(code).decode()
        super().__init__(f"{where}: {msg} (code {code})")
        self.code = code


def check(code, where):
    if code != 0:
        raise MpidError(code, where)
