"""ctypes binding of libdcs.so (the C ABI declared in include/dcs.h).

Argument marshalling only: every computation runs in the library's HIP
kernels.  Importing this module fails loudly if the library is not built.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdcs.so")

DCS_OK = 0
DCS_EINVAL = -1
DCS_ERANGE = -2
DCS_ENOMEM = -3
DCS_EHIP = -4
DCS_EUNSUPPORTED = -5
DCS_F32 = 0
DCS_F64 = 1
DCS_C64 = 2
DCS_C128 = 3
DCS_REORTH_NONE = 0
DCS_REORTH_LOCAL = 1
DCS_REORTH_FULL = 2
DCS_INVALID_INDEX = (1 << 64) - 1
FORM_NAMES = {-1: "untuned", 0: "split_staged", 1: "split_global", 2: "split_fused", 3: "single",
              4: "split_tiled"}

# every entry point of include/dcs.h: name -> (restype, argtypes)
_vp, _i, _sz, _u64 = C.c_void_p, C.c_int, C.c_size_t, C.c_uint64
_pp = C.POINTER(C.c_void_p)
_ip = C.POINTER(C.c_int)
_dp = C.POINTER(C.c_double)
_u64p = C.POINTER(C.c_uint64)
_szp = C.POINTER(C.c_size_t)
_i32p = C.POINTER(C.c_int32)

SIGNATURES = {
    "dcs_last_error": (C.c_char_p, []),
    "dcs_version": (_i, []),
    "dcs_sector_create": (_i, [_i, _i, _i, _i, _ip, _i, _pp]),
    "dcs_sector_create_mixed": (_i, [_i, _i, _i32p, _i, _ip, _i, _pp]),
    "dcs_sector_local_dims": (_i, [_vp, _i32p]),
    "dcs_sector_destroy": (_i, [_vp]),
    "dcs_sector_dim": (_i, [_vp, _u64p]),
    "dcs_sector_split": (_i, [_vp, _ip, _ip]),
    "dcs_sector_tables": (_i, [_vp, _ip, _szp]),
    "dcs_lex_rank": (_i, [_i, _i, _vp, _vp, _sz, _vp, _vp]),
    "dcs_lex_unrank": (_i, [_i, _i, _vp, _vp, _sz, _vp, _vp]),
    "dcs_lex_rank_q": (_i, [_i, _i, _i, _vp, _vp, _sz, _vp, _vp]),
    "dcs_lex_unrank_q": (_i, [_i, _i, _i, _vp, _vp, _sz, _vp, _vp]),
    "dcs_lex_rank_mixed": (_i, [_i, _i, _i32p, _vp, _vp, _sz, _vp, _vp]),
    "dcs_lex_unrank_mixed": (_i, [_i, _i, _i32p, _vp, _vp, _sz, _vp, _vp]),
    "dcs_rank": (_i, [_vp, _vp, _vp, _sz, _vp, _vp]),
    "dcs_rank_search": (_i, [_vp, _vp, _vp, _sz, _vp, _vp]),
    "dcs_unrank": (_i, [_vp, _vp, _vp, _sz, _vp, _vp]),
    "dcs_enumerate": (_i, [_vp, _u64, _sz, _vp, _vp]),
    "dcs_terms_create": (_i, [_i, _i32p, _i32p, _pp]),
    "dcs_terms_destroy": (_i, [_vp]),
    "dcs_hamiltonian_apply": (_i, [_vp, _vp, _vp, _vp, _vp, _i, _i, _vp, _vp, _vp]),
    "dcs_hamiltonian_form": (_i, [_vp, _vp, _i, _i, _ip]),
    "dcs_adjoint_workspace_size": (_i, [_vp, _vp, _i, _szp]),
    "dcs_hamiltonian_apply_adjoint": (_i, [_vp, _vp, _vp, _vp, _vp, _i, _i, _vp, _vp, _vp, _vp, _vp,
                                           _vp, _vp, _sz, _vp]),
    "dcs_hamiltonian_apply_adjoint_noalloc": (_i, [_vp, _vp, _vp, _vp, _vp, _i, _vp, _vp, _vp, _vp,
                                                   _vp, _vp, _vp]),
    "dcs_plan_create": (_i, [_i, _pp, _pp, _pp, _pp, _pp]),
    "dcs_plan_destroy": (_i, [_vp]),
    "dcs_plan_apply": (_i, [_vp, _i, _pp, _pp, _vp]),
    "dcs_lanczos_workspace_size": (_i, [_vp, _i, _i, _i, _i, _szp]),
    "dcs_lanczos": (_i, [_vp, _vp, _vp, _vp, _vp, _i, _i, _i, _vp, _dp, _dp, _ip, _i, _dp, _vp,
                         _i, _vp, _sz, _vp]),
    "dcs_expectation_workspace_size": (_i, [_vp, _vp, _szp]),
    "dcs_expectation_values": (_i, [_vp, _vp, _i, _i, _vp, _vp, _vp, _vp, _vp, _sz, _vp]),
    "dcs_tridiag_eigvals": (_i, [_dp, _dp, _i, _i, _dp, _i]),
    "dcs_lanczos_operator": (_i, [_vp, _vp, _i, _i, _i, _vp, _dp, _dp, _ip, _i, _dp, _vp, _i, _vp, _sz, _vp]),
    "dcs_operator_create": (_i, [_i, _i, _i, _i32p, _i32p, _dp, _dp, _i, _i, _i, _pp]),
    "dcs_operator_create_mixed": (_i, [_i, _i32p, _i, _i32p, _i32p, _dp, _dp, _i, _i, _i, _pp]),
    "dcs_operator_destroy": (_i, [_vp]),
    "dcs_operator_info": (_i, [_vp, _ip, _u64p, _ip, _ip]),
    "dcs_operator_apply": (_i, [_vp, _vp, _i, _i, _vp, _vp, _vp]),
    "dcs_operator_expectation_workspace_size": (_i, [_vp, _vp, _i, _szp]),
    "dcs_operator_expectation": (_i, [_vp, _vp, _i, _i, _vp, _vp, _vp, _sz, _vp]),
}


class DcsError(RuntimeError):
    def __init__(self, code: int, name: str, msg: str):
        super().__init__(f"{name} failed with status {code}: {msg}")
        self.code = code


_lib = None


def lib():
    """The loaded library (raises if it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"{LIB_PATH} is missing: build it with `python -m paper_2407_14591_amd.build` "
                "(there is no CPU fallback)")
        l = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(l, name)
            f.restype = res
            f.argtypes = args
        _lib = l
    return _lib


def call(name: str, *args) -> int:
    """Call an entry point; raise DcsError on a non-zero status."""
    r = getattr(lib(), name)(*args)
    if r != DCS_OK:
        msg = lib().dcs_last_error()
        raise DcsError(r, name, msg.decode() if msg else "")
    return r
