"""ctypes view of the C ABI in include/mrtfd.h (argument marshalling only).

Every function of the header is exposed under the same name with the same
arguments.  Loading fails loudly when libmrtfd.so is missing: there is no
fallback path.
"""
import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmrtfd.so")

MRTFD_OK = 0
MRTFD_ERR_ARG = -1
MRTFD_ERR_HIP = -2
MRTFD_ERR_UNSTABLE = -3
MRTFD_ERR_NONFINITE = -4
MRTFD_ERR_STATE = -5
MRTFD_ERR_UNSUPPORTED = -6

MRTFD_BC_PERIODIC = 0
MRTFD_BC_DIRICHLET = 1
MRTFD_BC_REFLECT = 2
MRTFD_BC_EXTRAPOLATE = 3
MRTFD_BC_WALL = 4
BC_KINDS = {"periodic": MRTFD_BC_PERIODIC, "dirichlet": MRTFD_BC_DIRICHLET,
            "reflect": MRTFD_BC_REFLECT, "extrapolate": MRTFD_BC_EXTRAPOLATE,
            "wall": MRTFD_BC_WALL}

MRTFD_FP32 = 0
MRTFD_BF16X3 = 1
MRTFD_FP64 = 2

MRTFD_LAYOUT_ROWS = 0
MRTFD_LAYOUT_PLANES = 1
MRTFD_LAYOUT_TILES = 2

MRTFD_COLLISION_MRT = 0
MRTFD_COLLISION_SRT = 1

MRTFD_KERNEL_AUTO = 0
MRTFD_KERNEL_SIMPLE = 1
MRTFD_KERNEL_ROWS = 2
MRTFD_KERNEL_MFMA = 3


class mrtfd_side(C.Structure):
    _fields_ = [
        ("kind_lo", C.c_int32), ("kind_hi", C.c_int32),
        ("state_lo", C.c_double * 4), ("state_hi", C.c_double * 4),
        ("split0", C.c_double), ("split_rate", C.c_double),
    ]


class mrtfd_batch_params(C.Structure):
    _fields_ = [
        ("ntubes", C.c_int32),
        ("dx", C.c_double), ("dt", C.c_double),
        ("s", C.c_double * 16),
        ("seg_cols", C.c_int32), ("round_steps", C.c_int32), ("use_graph", C.c_int32),
    ]


class mrtfd_params(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32),
        ("dx", C.c_double), ("dy", C.c_double), ("dt", C.c_double),
        ("s", C.c_double * 16),
        ("side", mrtfd_side * 4),
        ("precision", C.c_int32), ("kernel", C.c_int32),
        ("rows", C.c_int32), ("graph_steps", C.c_int32),
        ("collision", C.c_int32), ("layout", C.c_int32),
        ("flux_budget", C.c_int32),
        ("ref_rho", C.c_double), ("ref_T", C.c_double),
    ]


_vp = C.c_void_p
_fp = C.c_void_p  # device float*
_PROTOS = {
    "mrtfd_workspace_bytes": (C.c_size_t, [C.POINTER(mrtfd_params)]),
    "mrtfd_check_params": (C.c_int32, [C.POINTER(mrtfd_params), C.c_char_p, C.c_size_t]),
    "mrtfd_create": (C.c_int32, [C.POINTER(mrtfd_params), _vp, C.c_size_t, _vp, C.POINTER(_vp)]),
    "mrtfd_destroy": (C.c_int32, [_vp]),
    "mrtfd_init_macro": (C.c_int32, [_vp, _fp, _fp, _fp, _fp]),
    "mrtfd_step": (C.c_int32, [_vp, C.c_int64]),
    "mrtfd_outflow": (C.c_int32, [_vp, C.POINTER(C.c_double)]),
    "mrtfd_read_macro": (C.c_int32, [_vp, _fp, _fp, _fp, _fp, _fp]),
    "mrtfd_sums": (C.c_int32, [_vp, C.POINTER(C.c_double)]),
    "mrtfd_sums_noalloc": (C.c_int32, [_vp, _vp]),
    "mrtfd_get_f": (C.c_int32, [_vp, _fp]),
    "mrtfd_set_f": (C.c_int32, [_vp, _fp]),
    "mrtfd_get_f64": (C.c_int32, [_vp, _vp]),
    "mrtfd_set_f64": (C.c_int32, [_vp, _vp]),
    "mrtfd_ref_populations": (C.c_int32, [C.POINTER(mrtfd_params), C.POINTER(C.c_double)]),
    "mrtfd_screen": (C.c_int32, [C.POINTER(mrtfd_params), C.POINTER(C.c_double), _vp, C.c_int32, _vp, _vp, _vp]),
    "mrtfd_screen_sets": (C.c_int32, [C.POINTER(mrtfd_params), C.c_int32, _vp, _vp, _vp, C.c_int32, _vp, _vp, _vp]),
    "mrtfd_time": (C.c_int32, [_vp, C.POINTER(C.c_int64), C.POINTER(C.c_double)]),
    "mrtfd_set_step": (C.c_int32, [_vp, C.c_int64]),
    "mrtfd_kernel_info": (C.c_int32, [_vp, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                      C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    "mrtfd_model": (C.c_int32, [C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "mrtfd_struct_sizes": (C.c_int32, [C.POINTER(C.c_size_t), C.POINTER(C.c_size_t)]),
    "mrtfd_status_string": (C.c_char_p, [C.c_int32]),
    "mrtfd_last_error": (C.c_char_p, [_vp]),
    "mrtfd_batch_workspace_bytes": (C.c_size_t, [C.POINTER(mrtfd_batch_params), C.POINTER(C.c_int32)]),
    "mrtfd_batch_create": (C.c_int32, [C.POINTER(mrtfd_batch_params), C.POINTER(C.c_int32),
                                       C.POINTER(C.c_int64), C.POINTER(C.c_double),
                                       C.POINTER(C.c_double), _vp, C.c_size_t, _vp, C.POINTER(_vp)]),
    "mrtfd_batch_init": (C.c_int32, [_vp]),
    "mrtfd_batch_run": (C.c_int32, [_vp]),
    "mrtfd_batch_read_macro": (C.c_int32, [_vp, C.c_int32, _fp, _fp, _fp, _fp, _fp]),
    "mrtfd_batch_get_f": (C.c_int32, [_vp, C.c_int32, _fp]),
    "mrtfd_batch_info": (C.c_int32, [_vp, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                     C.POINTER(C.c_int32)]),
    "mrtfd_batch_destroy": (C.c_int32, [_vp]),
    "mrtfd_batch_last_error": (C.c_char_p, [_vp]),
}

_lib = None


def lib():
    """The loaded libmrtfd.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                "(or python paper_0908_3749_amd/build_lib.py); there is no fallback")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _PROTOS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def exported_names():
    return list(_PROTOS)


class MrtfdError(RuntimeError):
    def __init__(self, status, msg=""):
        self.status = status
        name = lib().mrtfd_status_string(status).decode()
        super().__init__(f"mrtfd status {status} ({name}){': ' + msg if msg else ''}")


def check(status, ctx=None, batch=None):
    if status != MRTFD_OK:
        msg = ""
        if ctx is not None:
            raw = lib().mrtfd_last_error(ctx)
            msg = raw.decode() if raw else ""
        elif batch is not None:
            raw = lib().mrtfd_batch_last_error(batch)
            msg = raw.decode() if raw else ""
        raise MrtfdError(status, msg)
    return status
