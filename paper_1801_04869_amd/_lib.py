"""ctypes loader of libmagfft.so (the HIP library built from csrc/).

Argument marshalling only.  Loading fails loudly when the library has not
been built: there is no fallback implementation.
"""
import ctypes
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmagfft.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "magfft.h")

_lib = None

c_int, c_double, c_void_p = ctypes.c_int, ctypes.c_double, ctypes.c_void_p
P_int = ctypes.POINTER(ctypes.c_int)
P_double = ctypes.POINTER(ctypes.c_double)

SIGNATURES = {
    "mag_create": (c_int, [ctypes.POINTER(c_void_p), c_int, c_int, c_void_p]),
    "mag_destroy": (None, [c_void_p]),
    "mag_set_grid": (c_int, [c_void_p, c_int, c_int, c_int, c_double, c_double, c_double]),
    "mag_set_domain": (c_int, [c_void_p, c_void_p]),
    "mag_set_params": (c_int, [c_void_p, c_void_p, c_double, c_double, c_double, c_double]),
    "mag_set_solver": (c_int, [c_void_p, c_double, c_double, c_int, c_int]),
    "mag_set_field": (c_int, [c_void_p, c_int, P_double, c_double, c_double, c_double]),
    "mag_rhs": (c_int, [c_void_p, c_void_p, c_double, c_void_p, P_int]),
    "mag_rhs_status": (c_int, [c_void_p, P_int]),
    "mag_step": (c_int, [c_void_p, c_void_p, P_double, P_double, c_double, c_double, P_int]),
    "mag_integrate": (c_int, [c_void_p, c_void_p, c_double, c_double, c_double, c_double, P_double, c_int, P_int]),
    "mag_integrate_captured": (c_int, [c_void_p, c_void_p, c_double, c_double, c_double, c_double, c_int,
                                       ctypes.c_longlong, P_int, P_int, P_double]),
    "mag_observe": (c_int, [c_void_p, c_void_p, c_double, c_void_p, c_void_p, P_double]),
    "mag_rhs_vjp": (c_int, [c_void_p, c_void_p, c_double, c_void_p, c_void_p, c_void_p]),
    "mag_reset_warm_start": (c_int, [c_void_p]),
    "mag_set_warm_start": (c_int, [c_void_p, c_int]),
    "mag_set_derivatives": (c_int, [c_void_p, c_int, c_double]),
    "mag_step_fixed": (c_int, [c_void_p, c_void_p, c_double, c_double]),
    "mag_step_vjp": (c_int, [c_void_p, c_void_p, c_double, c_double, c_void_p, c_void_p, c_void_p]),
    "mag_observe_vjp": (c_int, [c_void_p, c_void_p, c_void_p]),
    "mag_last_error": (ctypes.c_char_p, [c_void_p]),
    "mag_prof_enable": (c_int, [c_void_p, c_int]),
    "mag_prof_read": (c_int, [c_void_p, c_int, P_int, P_double]),
    "mag_prof_kernel_name": (ctypes.c_char_p, [c_int]),
    "mag_film_moment_noalloc": (c_int, [c_void_p, c_int, c_int, c_double, c_double, c_void_p, c_void_p]),
    "mag_stats": (c_int, [c_void_p, c_int, ctypes.POINTER(ctypes.c_longlong), ctypes.POINTER(ctypes.c_longlong)]),
}


def header_symbols():
    """Names of the functions declared in include/magfft.h."""
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(mag_[a-z_]+)\s*\(", txt)))


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libmagfft.so is not built; run `python -m paper_1801_04869_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib
