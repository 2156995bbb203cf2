"""ctypes declarations of libchemmi.so (include/chem.h).  Argument
marshalling only; every step of the computation runs in the library's
kernels.  Loading fails loudly if the library has not been built."""
from __future__ import annotations

import ctypes as C
import pathlib

LIB_PATH = pathlib.Path(__file__).resolve().parent / "libchemmi.so"
NOALLOC_MAX_CELLS = 2097152        # CHEM_NOALLOC_MAX_CELLS

CHEM_OK = 0
ERRORS = {-1: "CHEM_E_INVAL", -2: "CHEM_E_PARSE", -3: "CHEM_E_MECH_INVALID", -4: "CHEM_E_HIP",
          -5: "CHEM_E_NOMEM", -6: "CHEM_E_CELL_FAILED", -7: "CHEM_E_COMPILE", -8: "CHEM_E_UNSUPPORTED"}
FORM_AUTO, FORM_PLAIN, FORM_PERSISTENT = 0, 1, 2
ORDER_COST, ORDER_NATURAL = 1, 2

EXPORTS = ["chem_load_mechanism", "chem_load_chemkin", "chem_load_openfoam", "chem_free_mechanism", "chem_mechanism_info", "chem_get_params",
           "chem_set_params", "chem_eval_source", "chem_step_fixed", "chem_integrate",
           "chem_integrate_source", "chem_euler1d_init", "chem_euler1d_step", "chem_integrate_batched", "chem_integrate_adjoint",
           "chem_integrate_noalloc",
           "chem_last_error", "chem_version"]


class Options(C.Structure):
    _fields_ = [("form", C.c_int), ("max_substeps", C.c_int), ("hmin_rel", C.c_double),
                ("h0", C.c_void_p), ("checkpoint_every", C.c_int), ("block", C.c_int),
                ("waves_per_simd", C.c_int), ("refill", C.c_int), ("order", C.c_int),
                ("cost", C.POINTER(C.c_void_p)), ("adjoint_nacc", C.c_void_p)]


class Stats(C.Structure):
    _fields_ = [("cells", C.c_int64), ("accepted", C.c_int64), ("rejected", C.c_int64),
                ("max_substeps", C.c_int64), ("failed", C.c_int64), ("kernel_ms", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class ChemError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not LIB_PATH.exists():
            raise ImportError(f"{LIB_PATH} is not built; run python -m paper_2508_16105_amd.build")
        L = C.CDLL(str(LIB_PATH))
        vp, i64, dbl, i32 = C.c_void_p, C.c_int64, C.c_double, C.c_int
        L.chem_load_mechanism.argtypes = [C.c_char_p, C.POINTER(vp)]
        L.chem_load_chemkin.argtypes = [C.c_char_p, C.c_char_p, C.POINTER(vp)]
        L.chem_load_openfoam.argtypes = [C.c_char_p, C.c_char_p, C.POINTER(vp)]
        L.chem_free_mechanism.argtypes = [vp]
        L.chem_free_mechanism.restype = None
        L.chem_mechanism_info.argtypes = [vp, C.POINTER(i32), C.POINTER(i32)]
        L.chem_get_params.argtypes = [vp, vp, vp, vp]
        L.chem_set_params.argtypes = [vp, vp, vp, vp]
        L.chem_eval_source.argtypes = [vp, i64, vp, vp, vp, vp, vp, vp]
        L.chem_step_fixed.argtypes = [vp, i64, vp, vp, vp, dbl, dbl, dbl, vp, vp, vp, vp]
        L.chem_integrate.argtypes = [vp, i64, vp, vp, vp, dbl, dbl, dbl, C.POINTER(Options),
                                     C.POINTER(Stats), vp, vp, vp, vp]
        L.chem_integrate_noalloc.argtypes = [vp, i64, vp, vp, vp, dbl, dbl, dbl, C.POINTER(Options),
                                             vp, vp, vp, vp]
        L.chem_euler1d_init.argtypes = [vp, i64, vp, vp, vp, vp, vp, vp]
        L.chem_euler1d_step.argtypes = [vp, i64, dbl, dbl, vp, vp, vp, dbl, dbl, C.POINTER(Options),
                                        C.POINTER(Stats), C.POINTER(dbl), vp]
        L.chem_integrate_source.argtypes = [vp, i64, vp, vp, vp, dbl, dbl, dbl, vp, vp, C.POINTER(Options),
                                            C.POINTER(Stats), vp, vp]
        L.chem_integrate_batched.argtypes = [vp, i32, vp, vp, vp, vp, dbl, dbl, dbl,
                                             C.POINTER(Options), C.POINTER(Stats), vp]
        L.chem_integrate_adjoint.argtypes = [vp, i64, vp, vp, vp, dbl, dbl, dbl, vp, vp, vp, vp,
                                             vp, vp, vp, vp, vp, C.POINTER(Options),
                                             C.POINTER(Stats), vp]
        L.chem_last_error.restype = C.c_char_p
        L.chem_last_error.argtypes = []
        L.chem_version.restype = C.c_char_p
        L.chem_version.argtypes = []
        _lib = L
    return _lib


def check(rc, allow=()):
    if rc != CHEM_OK and rc not in allow:
        raise ChemError(rc, lib().chem_last_error().decode())
    return rc


def load_mechanism_handle(path: str, thermo: str | None = None, fmt: str | None = None) -> C.c_void_p:
    """chem_load_mechanism; chem_load_chemkin when a thermo file is given;
    chem_load_openfoam for fmt == "openfoam" (path: reactions, thermo: thermo)."""
    h = C.c_void_p()
    if fmt == "openfoam":
        check(lib().chem_load_openfoam(str(path).encode(), str(thermo).encode(), C.byref(h)))
    elif thermo is None:
        check(lib().chem_load_mechanism(str(path).encode(), C.byref(h)))
    else:
        check(lib().chem_load_chemkin(str(path).encode(), str(thermo).encode(), C.byref(h)))
    return h
