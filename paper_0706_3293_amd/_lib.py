"""ctypes declarations of libhm.so (include/hm.h).

Argument marshalling only.  The library must have been built in-tree
(``python -m paper_0706_3293_amd.build`` or ``__graft_entry__.build()``);
a missing library is an error, never a fallback.
"""
import ctypes
import os

import torch  # noqa: F401  (load torch's HIP runtime first: one runtime per process)

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhm.so")

HM_OK, HM_EINVAL, HM_ERANGE, HM_ENOMEM, HM_EDEVICE, HM_EWORKSPACE = 0, -1, -2, -3, -4, -5
HM_F64, HM_F32 = 0, 1
HM_PREC_F64, HM_PREC_F32_MIXED = 0, 1

_NAMES = {HM_EINVAL: "HM_EINVAL", HM_ERANGE: "HM_ERANGE", HM_ENOMEM: "HM_ENOMEM",
          HM_EDEVICE: "HM_EDEVICE", HM_EWORKSPACE: "HM_EWORKSPACE"}


class HMError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_NAMES.get(code, code)}: {msg}")
        self.code = code


class LanczosOpts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("full_reorth", ctypes.c_int32),
                ("breakdown_tol", ctypes.c_double), ("use_graph", ctypes.c_int32),
                ("kernel", ctypes.c_int32)]


_vp = ctypes.c_void_p
_i32, _i64, _dbl = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
_dblp = ctypes.POINTER(ctypes.c_double)
_i32p = ctypes.POINTER(ctypes.c_int32)
_i64p = ctypes.POINTER(ctypes.c_int64)
_u8p = ctypes.POINTER(ctypes.c_uint8)
_szp = ctypes.POINTER(ctypes.c_size_t)
_optp = ctypes.POINTER(LanczosOpts)

SIGNATURES = {
    "hm_last_error": (ctypes.c_char_p, []),
    "hm_version": (ctypes.c_char_p, []),
    "hm_count": (_i32, [_i32, _i32, _i32, _i64p]),
    "hm_basis_init": (_i32, [_i32, _i32, _i32, ctypes.POINTER(_vp)]),
    "hm_basis_free": (_i32, [_vp]),
    "hm_basis_dim": (_i32, [_vp, _i64p]),
    "hm_basis_info": (_i32, [_vp, _i32p, _i32p, _i32p, _i32p]),
    "hm_basis_set_schedule": (_i32, [_vp, _i32, _i32, _i32]),
    "hm_basis_set_staging": (_i32, [_vp, _i32]),
    "hm_unrank": (_i32, [_vp, _i64, _u8p]),
    "hm_rank": (_i32, [_vp, _u8p, _i64p]),
    "hm_unrank_dev": (_i32, [_vp, _vp, _i64, _vp, _vp]),
    "hm_rank_dev": (_i32, [_vp, _vp, _i64, _vp, _vp]),
    "hm_apply": (_i32, [_vp, _dblp, _vp, _vp, _i32, _vp]),
    "hm_apply_kernel": (_i32, [_vp, _dblp, _vp, _vp, _i32, _i32, _vp]),
    "hm_lanczos_workspace": (_i32, [_vp, _i32, _optp, _szp]),
    "hm_lanczos": (_i32, [_vp, _dblp, _vp, _i32, _optp, _vp, ctypes.c_size_t, _dblp, _dblp,
                          _dblp, _i32p, _vp]),
    "hm_lanczos_ritz": (_i32, [_vp, _dblp, _vp, _i32, _dblp, _optp, _vp, ctypes.c_size_t,
                               _vp, _dblp, _dblp, _vp]),
    "hm_tridiag_lowest": (_i32, [_i32, _dblp, _dblp, _dblp, _dblp]),
    "hm_tridiag_ritz": (_i32, [_i32, _dblp, _dblp, _dblp, _dblp]),
    "hm_block_tridiag_eigenvalues": (_i32, [_i32, _i32, _dblp, _dblp, _dblp]),
    "hm_basis_set_items_per_wave": (_i32, [_vp, _i32]),
    "hm_ftl_sums": (_i32, [_i32, _i32p, _dblp, _dblp, _dblp, _i32, _dblp, _dblp, _dblp,
                            _dblp, _dblp]),
    "hm_block_lanczos_workspace": (_i32, [_vp, _i32, _i32, _szp]),
    "hm_block_lanczos": (_i32, [_vp, _dblp, _vp, _i32, _i32, _vp, ctypes.c_size_t, _dblp, _dblp,
                                _i32p, _vp]),
    "hm_bond_corr_workspace": (_i32, [_vp, _i32, _szp]),
    "hm_bond_corr": (_i32, [_vp, _i32p, _i32, _vp, _vp, ctypes.c_size_t, _dblp, _vp]),
    "hm_basis_cached_couplings": (_i32, [_vp, _i32p]),
    "hm_bond_corr_noalloc": (_i32, [_vp, _i32p, _i32, _vp, _dblp, _vp]),
    "hm_lanczos_batched_workspace": (_i32, [_i32, ctypes.POINTER(_vp), _i32, _i32, _szp]),
    "hm_lanczos_batched": (_i32, [_i32, ctypes.POINTER(_vp), ctypes.POINTER(_dblp),
                                  ctypes.POINTER(_vp), _i32, _i32, _dbl, _i32, _i32, _vp,
                                  ctypes.c_size_t, _dblp, _dblp, _dblp, _i32p, _vp]),
    "hm_set_timing": (_i32, [_i32]),
    "hm_last_timing": (_i32, [_dblp, _i32p, _dblp]),
}

_lib = None


def lib():
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                "or python -m paper_0706_3293_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(rc):
    if rc != HM_OK:
        raise HMError(rc, lib().hm_last_error().decode())
    return rc
