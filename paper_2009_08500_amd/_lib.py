"""ctypes loader for librr.so and the declarations of its C ABI (include/rr.h).

The HIP library is the product: if it has not been built this module raises
ImportError instead of falling back to anything else.
"""

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librr.so")

RR_OK, RR_EINVAL, RR_ENOMEM, RR_EDEVICE, RR_ELIMIT, RR_EBUSY, RR_ENOTFOUND = 0, -1, -2, -3, -4, -5, -6
RR_FP64, RR_MIXED = 0, 1
RR_MAX_PB, RR_MAX_LC, RR_MAX_NSS = 16, 64, 1024
RR_NOALLOC_MAX_PV = 16384
RR_KERNEL_TILES, RR_KERNEL_SPLIT, RR_KERNEL_SPLIT_FUSED = 0, 1, 2

c_double_p = ctypes.POINTER(ctypes.c_double)
c_int32_p = ctypes.POINTER(ctypes.c_int32)
c_void_p = ctypes.c_void_p


class RRGrid(ctypes.Structure):
    """Mirror of rr_grid."""
    _fields_ = [("zcut", ctypes.c_double), ("nzin", ctypes.c_int32),
                ("nzlimb", ctypes.c_int32), ("ng", ctypes.c_int32),
                ("nk", ctypes.c_int32), ("k0", ctypes.c_double),
                ("k1", ctypes.c_double)]


class RRError(RuntimeError):
    def __init__(self, code, where, detail=""):
        self.code = code
        msg = f"{where}: {strerror(code)} ({code})"
        if detail:
            msg += f": {detail}"
        super().__init__(msg)


_lib = None


def lib():
    """The loaded library (loaded once)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"{LIB_PATH} is missing: build the HIP library first "
                "(python -c 'import __graft_entry__ as g; g.build()')")
        L = ctypes.CDLL(LIB_PATH)
        _declare(L)
        _lib = L
    return _lib


def _declare(L):
    i32, i64, dbl = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    L.rr_strerror.argtypes = [ctypes.c_int]
    L.rr_strerror.restype = ctypes.c_char_p
    L.rr_last_error.argtypes = []
    L.rr_last_error.restype = ctypes.c_char_p
    L.rr_prepare_ld.argtypes = [c_void_p, c_void_p, i32, i32, ctypes.POINTER(RRGrid),
                                ctypes.POINTER(c_void_p)]
    L.rr_prepare_ld.restype = ctypes.c_int
    L.rr_set_profile.argtypes = [c_void_p, c_void_p, c_void_p]
    L.rr_set_profile.restype = ctypes.c_int
    L.rr_evaluate.argtypes = [c_void_p, c_void_p, c_void_p, i32, c_void_p, c_void_p,
                              c_void_p, i32, c_void_p, i32, i32, i32, c_void_p, c_void_p]
    L.rr_evaluate.restype = ctypes.c_int
    L.rr_evaluate_noalloc.argtypes = L.rr_evaluate.argtypes
    L.rr_evaluate_noalloc.restype = ctypes.c_int
    L.rr_series_create.argtypes = [c_void_p, c_void_p, i32, c_void_p, c_void_p, c_void_p, i32,
                                   ctypes.POINTER(c_void_p)]
    L.rr_series_create.restype = ctypes.c_int
    L.rr_series_free.argtypes = [c_void_p]
    L.rr_series_free.restype = None
    L.rr_evaluate_series.argtypes = [c_void_p, c_void_p, c_void_p, i32, i32, i32, c_void_p,
                                     c_void_p]
    L.rr_evaluate_series.restype = ctypes.c_int
    L.rr_series_kernel.argtypes = [c_void_p, c_void_p, i32, i32, c_int32_p]
    L.rr_series_kernel.restype = ctypes.c_int
    L.rr_evaluate_ld.argtypes = [c_void_p, c_void_p, c_void_p, i32, c_void_p, c_void_p,
                                 c_void_p, i32, c_void_p, i32, i32, c_void_p, i32, c_void_p,
                                 c_void_p]
    L.rr_evaluate_ld.restype = ctypes.c_int
    L.rr_evaluate_direct.argtypes = [c_void_p, c_void_p, c_void_p, i32, c_void_p, c_void_p,
                                     c_void_p, i32, c_void_p, i32, i32, i32, c_void_p,
                                     c_void_p]
    L.rr_evaluate_direct.restype = ctypes.c_int
    L.rr_evaluate_variant.argtypes = [c_void_p, c_void_p, c_void_p, i32, c_void_p, c_void_p,
                                      c_void_p, i32, c_void_p, i32, i32, i32, i32, c_void_p,
                                      c_void_p]
    L.rr_evaluate_variant.restype = ctypes.c_int
    L.rr_select_variant.argtypes = [c_void_p, c_void_p, c_void_p, i32, c_void_p, c_void_p,
                                    c_void_p, i32, c_void_p, i32, i32, i32, c_void_p, i32,
                                    c_void_p, c_void_p, c_void_p]
    L.rr_select_variant.restype = ctypes.c_int
    L.rr_loglik_grad_small_planet.argtypes = [c_void_p, c_void_p, c_void_p, i32, c_void_p,
                                              c_void_p, c_void_p, i32, c_void_p, i32, i32,
                                              dbl, i32, c_void_p, dbl, c_void_p, c_void_p,
                                              c_void_p]
    L.rr_loglik_grad_small_planet.restype = ctypes.c_int
    L.rr_evaluate_small_planet.argtypes = [c_void_p, c_void_p, c_void_p, i32, c_void_p,
                                           c_void_p, c_void_p, i32, c_void_p, i32, i32, dbl,
                                           i32, c_void_p, c_void_p]
    L.rr_evaluate_small_planet.restype = ctypes.c_int
    L.rr_flux_at_z.argtypes = [c_void_p, c_void_p, c_void_p, dbl, i64, i32, i32, c_void_p,
                               c_void_p]
    L.rr_flux_at_z.restype = ctypes.c_int
    L.rr_set_kernel_events.argtypes = [c_void_p, c_void_p]
    L.rr_set_kernel_events.restype = ctypes.c_int
    L.rr_free_tables.argtypes = [c_void_p]
    L.rr_free_tables.restype = None
    L.rr_tables_copy.argtypes = [c_void_p, i32, c_void_p, i64, ctypes.POINTER(i64)]
    L.rr_tables_copy.restype = ctypes.c_int
    L.rr_tables_info.argtypes = [c_void_p, ctypes.POINTER(RRGrid), c_int32_p]
    L.rr_tables_info.restype = ctypes.c_int
    if hasattr(L, "rr_loglik_grad"):
        L.rr_loglik_grad.argtypes = [c_void_p, c_void_p, c_void_p, i32, c_void_p, c_void_p,
                                     c_void_p, i32, c_void_p, i32, i32, i32, c_void_p, dbl,
                                     c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]
        L.rr_loglik_grad.restype = ctypes.c_int
        L.rr_loglik_grad_ld.argtypes = [c_void_p, c_void_p, c_void_p, i32, c_void_p,
                                        c_void_p, c_void_p, i32, c_void_p, i32, i32, c_void_p,
                                        i32, c_void_p, dbl, c_void_p, c_void_p, c_void_p,
                                        c_void_p]
        L.rr_loglik_grad_ld.restype = ctypes.c_int
        L.rr_loglik_grad_istar.argtypes = L.rr_loglik_grad.argtypes[:-1] + [c_void_p, c_void_p]
        L.rr_loglik_grad_istar.restype = ctypes.c_int
    L.rr_set_istar.argtypes = [c_void_p, c_void_p, c_void_p]
    L.rr_set_istar.restype = ctypes.c_int
    _ = dbl


def strerror(code):
    return lib().rr_strerror(int(code)).decode()


def last_error():
    return lib().rr_last_error().decode()


def check(code, where):
    if code != RR_OK:
        raise RRError(code, where, last_error())
