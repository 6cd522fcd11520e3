"""ctypes declarations of include/ups.h (argument marshalling only)."""
import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
# UPS_LIB names another in-tree build of the same library (the sanitizer
# build libups_san.so); the default is libups.so
LIB_PATH = os.path.join(_HERE, os.path.basename(os.environ.get("UPS_LIB") or "libups.so"))

UPS_OK = 0
UPS_ERR_INVALID_ARG = 1
UPS_ERR_UNSUPPORTED = 2
UPS_ERR_WORKSPACE = 3
UPS_ERR_DEVICE = 4
UPS_ERR_NONFINITE = 5
UPS_ERR_INTERNAL = 6
UPS_ERR_STATE = 7
STATUS_NAMES = {0: "UPS_OK", 1: "UPS_ERR_INVALID_ARG", 2: "UPS_ERR_UNSUPPORTED", 3: "UPS_ERR_WORKSPACE",
                4: "UPS_ERR_DEVICE", 5: "UPS_ERR_NONFINITE", 6: "UPS_ERR_INTERNAL", 7: "UPS_ERR_STATE"}

UPS_BC_UNB, UPS_BC_PER, UPS_BC_EVEN, UPS_BC_ODD = 0, 1, 2, 3
UPS_GREEN_LGF2, UPS_GREEN_LGF4_MEHR, UPS_GREEN_LGF6_MEHR = 0, 1, 2
UPS_F64, UPS_F32 = 0, 1
UPS_CELL, UPS_NODE = 0, 1
UPS_NOALLOC_MAX_WORK = 64 << 20
UPS_MG_MAX_LEVELS = 8


class ups_problem(C.Structure):
    _fields_ = [
        ("n", C.c_int * 3),
        ("h", C.c_double * 3),
        ("bc", (C.c_int * 2) * 3),
        ("green", C.c_int),
        ("prec", C.c_int),
        ("center", C.c_int),
        ("ncomp", C.c_int),
        ("pad", C.c_int * 3),
    ]


class ups_mg_hierarchy(C.Structure):
    _fields_ = [
        ("levels", C.c_int),
        ("origin", (C.c_int * 3) * UPS_MG_MAX_LEVELS),
        ("cells", (C.c_int * 3) * UPS_MG_MAX_LEVELS),
    ]


class UpsError(RuntimeError):
    def __init__(self, status, message):
        self.status = status
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, status), message))


# name -> (restype, argtypes); every function declared in include/ups.h
SIGNATURES = {
    "ups_abi_version": (C.c_int, []),
    "ups_last_error": (C.c_char_p, []),
    "ups_supported_length": (C.c_int, [C.c_int, C.c_int]),
    "ups_problem_init": (None, [C.POINTER(ups_problem)]),
    "ups_plan_create": (C.c_int, [C.POINTER(ups_problem), C.POINTER(C.c_void_p)]),
    "ups_plan_sizes": (C.c_int, [C.c_void_p, C.POINTER(C.c_size_t), C.POINTER(C.c_size_t)]),
    "ups_plan_setup": (C.c_int, [C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p, C.c_size_t, C.c_void_p]),
    "ups_solve": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "ups_solve_noalloc": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "ups_solve_adjoint": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "ups_plan_kernel": (C.c_char_p, [C.c_void_p, C.c_int]),
    "ups_plan_set_kernel": (C.c_int, [C.c_void_p, C.c_int, C.c_char_p]),
    "ups_kernel_variants": (C.c_int, [C.c_int, C.c_int, C.c_int, C.POINTER(C.c_char_p), C.c_int]),
    "ups_kernel_fill_variants": (C.c_int, [C.c_int, C.c_int, C.c_int, C.POINTER(C.c_char_p), C.c_int]),
    "ups_run_pass": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p]),
    "ups_plan_layout": (C.c_int, [C.c_void_p, C.POINTER(C.c_int), C.POINTER(C.c_longlong),
                                  C.POINTER(C.c_longlong), C.POINTER(C.c_size_t), C.POINTER(C.c_longlong)]),
    "ups_plan_set_slab": (C.c_int, [C.c_void_p, C.c_int]),
    "ups_plan_slab": (C.c_int, [C.c_void_p]),
    "ups_plan_set_side_stream": (C.c_int, [C.c_void_p, C.c_int]),
    "ups_plan_side_stream": (C.c_int, [C.c_void_p]),
    "ups_plan_model_bytes": (C.c_double, [C.c_void_p, C.c_int]),
    "ups_plan_destroy": (C.c_int, [C.c_void_p]),
    "ups_autotune": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_double]),
    "ups_plan_set_check_finite": (C.c_int, [C.c_void_p, C.c_int]),
    "ups_plan_guard_mode": (C.c_int, [C.c_void_p]),
    "ups_plan_work_offset": (C.c_size_t, [C.c_void_p]),
    "ups_plan_nyquist_packed": (C.c_int, [C.c_void_p]),
    "ups_batch_create": (C.c_int, [C.POINTER(ups_problem), C.c_int, C.POINTER(C.c_void_p)]),
    "ups_batch_sizes": (C.c_int, [C.c_void_p, C.POINTER(C.c_size_t), C.POINTER(C.c_size_t)]),
    "ups_batch_setup": (C.c_int, [C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p, C.c_size_t, C.c_void_p]),
    "ups_batch_solve": (C.c_int, [C.c_void_p, C.POINTER(C.c_void_p), C.POINTER(C.c_void_p), C.c_void_p]),
    "ups_batch_launches": (C.c_int, [C.c_void_p, C.c_int]),
    "ups_batch_destroy": (C.c_int, [C.c_void_p]),
    "ups_mg_create": (C.c_int, [C.c_void_p, C.POINTER(ups_mg_hierarchy), C.POINTER(C.c_void_p)]),
    "ups_mg_level_shape": (C.c_int, [C.c_void_p, C.c_int, C.POINTER(C.c_int)]),
    "ups_mg_sizes": (C.c_int, [C.c_void_p, C.POINTER(C.c_size_t)]),
    "ups_mg_setup": (C.c_int, [C.c_void_p, C.c_void_p, C.c_size_t]),
    "ups_mg_cycle": (C.c_int, [C.c_void_p, C.POINTER(C.c_void_p), C.POINTER(C.c_void_p), C.c_int, C.c_int,
                               C.c_void_p]),
    "ups_mg_residual": (C.c_int, [C.c_void_p, C.POINTER(C.c_void_p), C.POINTER(C.c_void_p),
                                  C.POINTER(C.c_double), C.c_void_p]),
    "ups_mg_destroy": (C.c_int, [C.c_void_p]),
}

_lib = None


def lib():
    """Load libups.so once; raise loudly if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libups.so is not built (expected at %s); run "
                               "`python -m paper_2512_08555_amd.build` or __graft_entry__.build()" % LIB_PATH)
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(status):
    if status != UPS_OK:
        msg = lib().ups_last_error()
        raise UpsError(status, msg.decode() if msg else "")
    return status
