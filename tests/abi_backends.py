"""The chemistry-step C ABI behind one Python interface, served either by the
GPU library (include/chem.h, device buffers through torch) or by the oracle's
host ABI (oracle/oracle_abi.h), so a test runs unchanged against both.

Test infrastructure: argument marshalling only; arrays in and out are numpy.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

CELL_OK, CELL_MAXSTEPS, CELL_HMIN, CELL_NONFINITE, CELL_BADINPUT = range(5)
E_INVAL, E_PARSE, E_MECH_INVALID, E_CELL_FAILED, E_UNSUPPORTED = -1, -2, -3, -6, -8


class _Opts(C.Structure):
    # the layout both headers declare for the options
    _fields_ = [("form", C.c_int), ("max_substeps", C.c_int), ("hmin_rel", C.c_double),
                ("h0", C.c_void_p), ("checkpoint_every", C.c_int), ("block", C.c_int),
                ("waves_per_simd", C.c_int), ("refill", C.c_int), ("order", C.c_int),
                ("cost", C.c_void_p), ("adjoint_nacc", C.c_void_p)]


class _Stats(C.Structure):
    _fields_ = [("cells", C.c_int64), ("accepted", C.c_int64), ("rejected", C.c_int64),
                ("max_substeps", C.c_int64), ("failed", C.c_int64), ("kernel_ms", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class _Backend:
    prefix = ""
    stream_arg = False

    def __init__(self, lib):
        self.L = lib
        vp, i64, dbl = C.c_void_p, C.c_int64, C.c_double
        s = [vp] if self.stream_arg else []
        f = lambda nm: getattr(lib, self.prefix + nm)  # noqa: E731
        f("load_mechanism").argtypes = [C.c_char_p, C.POINTER(vp)]
        f("free_mechanism").argtypes = [vp]
        f("free_mechanism").restype = None
        f("mechanism_info").argtypes = [vp, C.POINTER(C.c_int), C.POINTER(C.c_int)]
        f("get_params").argtypes = [vp, vp, vp, vp]
        f("set_params").argtypes = [vp, vp, vp, vp]
        f("eval_source").argtypes = [vp, i64, vp, vp, vp, vp, vp] + s
        f("step_fixed").argtypes = [vp, i64, vp, vp, vp, dbl, dbl, dbl, vp, vp, vp] + s
        f("integrate").argtypes = [vp, i64, vp, vp, vp, dbl, dbl, dbl, C.POINTER(_Opts), C.POINTER(_Stats),
                                   vp, vp, vp] + s
        f("integrate_adjoint").argtypes = [vp, i64, vp, vp, vp, dbl, dbl, dbl, vp, vp, vp, vp, vp, vp, vp, vp,
                                           vp, C.POINTER(_Opts), C.POINTER(_Stats)] + s
        f("last_error").restype = C.c_char_p
        self.f = f

    # buffers: subclasses turn numpy arrays into pointers the library takes
    def _in(self, a, dtype=np.float64):
        raise NotImplementedError

    def _out(self, shape, dtype=np.float64):
        raise NotImplementedError

    def _get(self, buf):
        raise NotImplementedError

    def _ptr(self, buf):
        raise NotImplementedError

    def _sync(self):
        pass

    def _call(self, nm, *args):
        extra = [None] if self.stream_arg else []
        rc = self.f(nm)(*args, *extra)
        self._sync()
        return rc

    def last_error(self) -> str:
        return self.f("last_error")().decode()

    def load(self, path):
        h = C.c_void_p()
        rc = self.f("load_mechanism")(str(path).encode(), C.byref(h))
        return rc, h

    def free(self, h):
        self.f("free_mechanism")(h)

    def info(self, h):
        ns, nr = C.c_int(), C.c_int()
        rc = self.f("mechanism_info")(h, C.byref(ns), C.byref(nr))
        return rc, ns.value, nr.value

    def get_params(self, h, nr):
        a, b, e = (np.zeros(nr) for _ in range(3))
        rc = self.f("get_params")(h, a.ctypes.data, b.ctypes.data, e.ctypes.data)
        return rc, a, b, e

    def set_params(self, h, a, b, e):
        a, b, e = (np.ascontiguousarray(x, dtype=np.float64) for x in (a, b, e))
        return self.f("set_params")(h, a.ctypes.data, b.ctypes.data, e.ctypes.data)

    def eval_source(self, h, T, p, Y, jac=False):
        n = Y.shape[1] + 1
        bufs = [self._in(x) for x in (T, p, Y)]
        fo = self._out((len(T), n))
        Jo = self._out((len(T), n, n)) if jac else None
        rc = self._call("eval_source", h, len(T), *map(self._ptr, bufs), self._ptr(fo),
                        self._ptr(Jo) if jac else None)
        return rc, self._get(fo), self._get(Jo) if jac else None

    def step_fixed(self, h, T, p, Y, step, rtol, atol):
        n = Y.shape[1] + 1
        bufs = [self._in(x) for x in (T, p, Y)]
        yn, en, ok = self._out((len(T), n)), self._out((len(T),)), self._out((len(T),), np.int32)
        rc = self._call("step_fixed", h, len(T), *map(self._ptr, bufs), step, rtol, atol, self._ptr(yn),
                        self._ptr(en), self._ptr(ok))
        return rc, self._get(yn), self._get(en), self._get(ok)

    def integrate(self, h, T, p, Y, dt, rtol, atol, max_substeps=0, hmin_rel=0.0, stats=True, null=()):
        bT, bp, bY = self._in(T), self._in(p), self._in(Y)
        st, na, nj = (self._out((len(T),), np.int32) for _ in range(3))
        o = _Opts(max_substeps=max_substeps, hmin_rel=hmin_rel)
        s = _Stats()
        ptr = lambda nm, b: None if nm in null else self._ptr(b)  # noqa: E731
        rc = self._call("integrate", h, len(T), ptr("T", bT), ptr("p", bp), ptr("Y", bY), dt, rtol, atol,
                        C.byref(o), C.byref(s) if stats else None, self._ptr(st), self._ptr(na), self._ptr(nj))
        return (rc, self._get(bT), self._get(bY), self._get(st), self._get(na), self._get(nj),
                s.as_dict() if stats else None)

    def adjoint(self, h, T0, p, Y0, dt, rtol, atol, gT, gY, nr, checkpoint_every=0, ends=(True, True),
                stats=True):
        bufs = [self._in(x) for x in (T0, p, Y0, gT, gY)]
        gT0, gY0 = self._out(T0.shape), self._out(Y0.shape)
        ga, gb, ge = (self._out((nr,)) for _ in range(3))
        Te = self._out(T0.shape) if ends[0] else None
        Ye = self._out(Y0.shape) if ends[1] else None
        o = _Opts(checkpoint_every=checkpoint_every)
        s = _Stats()
        rc = self._call("integrate_adjoint", h, len(T0), *map(self._ptr, bufs[:3]), dt, rtol, atol,
                        *map(self._ptr, bufs[3:]), self._ptr(gT0), self._ptr(gY0),
                        self._ptr(ga), self._ptr(gb), self._ptr(ge), self._ptr(Te) if ends[0] else None,
                        self._ptr(Ye) if ends[1] else None, C.byref(o), C.byref(s) if stats else None)
        out = [self._get(x) for x in (gT0, gY0, ga, gb, ge)]
        out += [self._get(Te) if ends[0] else None, self._get(Ye) if ends[1] else None]
        return (rc, *out, s.as_dict() if stats else None)


class OracleBackend(_Backend):
    """The oracle's host ABI: numpy buffers passed as they are."""
    name = "oracle"
    prefix = "oracle_"

    def __init__(self):
        import oracle
        oracle.lib()                                   # built and loaded
        super().__init__(C.CDLL(str(oracle.LIB)))     # own handle: own argtypes

    def _in(self, a, dtype=np.float64):
        return np.array(a, dtype=dtype, copy=True, order="C")

    def _out(self, shape, dtype=np.float64):
        return np.full(shape, np.nan if dtype == np.float64 else -99, dtype=dtype)

    def _get(self, buf):
        return buf

    def _ptr(self, buf):
        return None if buf is None else buf.ctypes.data


class GpuBackend(_Backend):
    """The GPU library: every buffer a device tensor on cuda:0, the default
    stream, a synchronisation after each call."""
    name = "gpu"
    prefix = "chem_"
    stream_arg = True

    def __init__(self):
        import torch

        from paper_2508_16105_amd import _lib
        self.torch = torch
        self.dev = torch.device("cuda:0")
        _lib.lib()                                     # built and loaded
        super().__init__(C.CDLL(str(_lib.LIB_PATH)))  # own handle: the package's declarations stay

    def _in(self, a, dtype=np.float64):
        return self.torch.tensor(np.ascontiguousarray(a, dtype=dtype), device=self.dev)

    def _out(self, shape, dtype=np.float64):
        t = self.torch.float64 if dtype == np.float64 else self.torch.int32
        return self.torch.full(shape, float("nan") if dtype == np.float64 else -99, dtype=t, device=self.dev)

    def _get(self, buf):
        return buf.cpu().numpy()

    def _ptr(self, buf):
        return None if buf is None else buf.data_ptr()

    def _sync(self):
        self.torch.cuda.synchronize()


def backend(name):
    return OracleBackend() if name == "oracle" else GpuBackend()
