"""ctypes declarations of liblsdm.so (the C ABI in include/lsdm.h)."""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
SO = os.path.join(HERE, "liblsdm.so")

OK, EINVAL, EPATTERN, ENOMEM, EDEVICE, EUNSUPPORTED = 0, -1, -2, -3, -4, -5
FP64, FP32, BF16, FP32_RC = 0, 1, 2, 3

# every function of include/lsdm.h: name -> (restype, argtypes)
_P = ctypes.c_void_p
_PP = ctypes.POINTER(ctypes.c_void_p)
_I = ctypes.c_int
_I32 = ctypes.c_int32
_I64P = ctypes.POINTER(ctypes.c_int64)
_D = ctypes.c_double
SIGNATURES = {
    "lsdm_system_create": (_I, [_I32, _P, _P, _P, _PP]),
    "lsdm_system_destroy": (None, [_P]),
    "lsdm_pattern_create": (_I, [_P, _D, _PP]),
    "lsdm_pattern_info": (_I, [_P, _I64P, _I64P]),
    "lsdm_pattern_export": (_I, [_P, _P, _P, _P, _P]),
    "lsdm_pattern_destroy": (None, [_P]),
    "lsdm_plan_create": (_I, [_P, _I, _P, _I, _P, _PP]),
    "lsdm_plan_info": (_I, [_P, _I64P, ctypes.POINTER(_D), _I64P]),
    "lsdm_plan_destroy": (None, [_P]),
    "lsdm_multiply": (_I, [_P, _I, _D, _P, _P, _D, _P, _P]),
    "lsdm_multiply_adjoint": (_I, [_P, _I, _P, _P, _P, _P, _P, _P]),
    "lsdm_dot": (_I, [_P, _P, _P, _P, _P]),
    "lsdm_dot_noalloc": (_I, [_P, _P, _P, _P, _P]),
    "lsdm_lnv_create": (_I, [_P, _D, _D, _D, _PP]),
    "lsdm_lnv_create_ex": (_I, [_P, _D, _D, _D, _I, _PP]),
    "lsdm_lnv_pattern": (_I, [_P, _I, _PP]),
    "lsdm_lnv_info": (_I, [_P, _I, _I64P, ctypes.POINTER(_D)]),
    "lsdm_lnv_energy": (_I, [_P, _I, _P, _P, _P, _P, _P, _P]),
    "lsdm_lnv_energy_grad": (_I, [_P, _I, _P, _P, _P, _P, _P, _P]),
    "lsdm_lnv_line": (_I, [_P, _I, _P, _P, _P, _P, _D, _P, _P]),
    "lsdm_lnv_minimise": (_I, [_P, _I, _P, _P, _P, _I, _D, _D, _P, _P, _P, _P]),
    "lsdm_lnv_shift": (_I, [_P, _D, _P, _D, _P, _P, _P]),
    "lsdm_lnv_electrons": (_I, [_P, _I, _P, _P, _P, _P, _P]),
    "lsdm_lnv_purify": (_I, [_P, _I, _P, _P, _P, _P]),
    "lsdm_lnv_profile": (_I, [_P, _I]),
    "lsdm_lnv_profile_read": (_I, [_P, _P, _P, _P]),
    "lsdm_lnv_destroy": (None, [_P]),
    "lsdm_set_allocator": (_I, [_P, _P, _P]),
    "lsdm_last_error": (ctypes.c_char_p, []),
    "lsdm_version": (ctypes.c_char_p, []),
}

_lib = None


class LsdmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"lsdm error {code}: {msg}")
        self.code = code


def lib():
    """The loaded library.  It must have been built (build() of the package or
    of __graft_entry__); a missing library is an error, never a fallback."""
    global _lib
    if _lib is None:
        if not os.path.exists(SO):
            raise ImportError(f"{SO} is missing: build the HIP library first (python -m paper_0911_3584_amd.build)")
        L = ctypes.CDLL(SO)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def check(rc):
    if rc != OK:
        raise LsdmError(rc, lib().lsdm_last_error().decode())
    return rc
