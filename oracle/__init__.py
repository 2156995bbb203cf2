"""ctypes binding of the CPU FP64 oracle (oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
benchmark's CPU-baseline leg.  The product path never imports this package.
"""
from __future__ import annotations

import ctypes as C
import os
import pathlib
import subprocess

import numpy as np

HERE = pathlib.Path(__file__).resolve().parent
LIB = HERE / "liboracle.so"
SOURCES = [HERE / "oracle.c", HERE / "chem_generic.inc", HERE / "oracle.h", HERE / "oracle_internal.h",
           HERE / "count.cpp", HERE / "abi.c", HERE / "oracle_abi.h"]

RODAS4 = 0
ROS4 = 1
CELL_OK, CELL_MAXSTEPS, CELL_HMIN, CELL_NONFINITE, CELL_BADINPUT = range(5)

_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_ip = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")


class Opts(C.Structure):
    _fields_ = [("method", C.c_int), ("max_substeps", C.c_int), ("hmin_rel", C.c_double)]


def build(force: bool = True) -> pathlib.Path:
    """Compile liboracle.so: oracle.c with gcc (plain C11 + OpenMP), the
    counted instantiation count.cpp with g++ and the C ABI layer abi.c,
    linked into one library."""
    if not force and LIB.exists() and all(LIB.stat().st_mtime >= s.stat().st_mtime for s in SOURCES):
        return LIB
    import tempfile
    tmp = LIB.with_suffix(".so.tmp")
    with tempfile.TemporaryDirectory() as d:
        co, cc, ca = os.path.join(d, "oracle.o"), os.path.join(d, "count.o"), os.path.join(d, "abi.o")
        subprocess.run(["gcc", "-O2", "-std=gnu11", "-fopenmp", "-fPIC", "-fcx-limited-range", "-Wall",
                        "-c", str(HERE / "oracle.c"), "-o", co], check=True)
        subprocess.run(["gcc", "-O2", "-std=gnu11", "-fPIC", "-Wall", "-c", str(HERE / "abi.c"), "-o", ca],
                       check=True)
        subprocess.run(["g++", "-O1", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
                        "-c", str(HERE / "count.cpp"), "-o", cc], check=True)
        subprocess.run(["g++", "-shared", "-fopenmp", "-o", str(tmp), co, cc, ca, "-lm"], check=True)
    os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not LIB.exists():
            build()
        L = C.CDLL(str(LIB))
        L.om_load.argtypes = [C.c_char_p, C.POINTER(C.c_void_p), C.c_char_p, C.c_int]
        L.om_free.argtypes = [C.c_void_p]
        L.om_nspecies.argtypes = [C.c_void_p]
        L.om_nreactions.argtypes = [C.c_void_p]
        L.om_weights.argtypes = [C.c_void_p, _dp]
        L.om_params.argtypes = [C.c_void_p, _dp, _dp, _dp]
        L.om_thermo.argtypes = [C.c_void_p, C.c_double, _dp, _dp, _dp]
        L.om_rates.argtypes = [C.c_void_p, C.c_void_p, C.c_double, _dp, _dp, _dp, _dp]
        for nm in ("om_rhs", "om_jac", "om_jac_cs"):
            getattr(L, nm).argtypes = [C.c_void_p, C.c_void_p, C.c_double, _dp, _dp]
        L.om_lu.argtypes = [C.c_int, _dp, _ip]
        L.om_lu_solve.argtypes = [C.c_int, _dp, _ip, _dp]
        L.om_tableau.argtypes = [C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_double), _dp, _dp, _dp, _dp]
        L.om_step.argtypes = [C.c_void_p, C.c_void_p, C.c_int, C.c_double, _dp, C.c_double, _dp, _dp]
        L.om_integrate.argtypes = [C.c_void_p, C.c_void_p, C.c_long, _dp, _dp, _dp, C.c_double,
                                   C.c_double, C.c_double, C.POINTER(Opts), _ip, _ip, _ip, C.c_int]
        L.om_step_sizes.argtypes = [C.c_void_p, C.c_void_p, C.c_double, C.c_double, _dp, C.c_double,
                                    C.c_double, C.c_double, C.POINTER(Opts), C.c_int, _dp,
                                    C.POINTER(C.c_int)]
        L.om_replay.argtypes = [C.c_void_p, C.c_void_p, C.c_int, C.c_double, _dp, C.c_int, _dp, _dp]
        L.om_replay_dir.argtypes = [C.c_void_p, C.c_int, C.c_double, _dp, C.c_int, _dp,
                                    C.c_void_p, C.c_void_p, _dp]
        L.om_count_step.argtypes = [C.c_void_p, C.c_double, _dp, C.c_double,
                                    np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")]
        L.om_adjoint.argtypes = [C.c_void_p, C.c_int, C.c_long, _dp, _dp, _dp, C.c_double,
                                 C.c_double, C.c_double, C.POINTER(Opts), _dp, _dp, _dp, _dp,
                                 _dp, _dp, _dp, C.c_int]
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


class Mechanism:
    """A mechanism loaded by the oracle's own reader."""

    def __init__(self, path):
        h = C.c_void_p()
        err = C.create_string_buffer(512)
        rc = lib().om_load(str(path).encode(), C.byref(h), err, 512)
        if rc != 0:
            raise ValueError(f"oracle could not load {path}: {err.value.decode()} (rc={rc})")
        self.h = h
        self.ns = lib().om_nspecies(h)
        self.nr = lib().om_nreactions(h)
        self.n = self.ns + 1

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.om_free(self.h)
            self.h = None

    # ---- data ----
    def weights(self):
        w = np.zeros(self.ns)
        lib().om_weights(self.h, w)
        return w

    def params(self):
        a, b, e = np.zeros(self.nr), np.zeros(self.nr), np.zeros(self.nr)
        lib().om_params(self.h, a, b, e)
        return a, b, e

    # ---- point functions ----
    def thermo(self, T):
        cp, h, s = np.zeros(self.ns), np.zeros(self.ns), np.zeros(self.ns)
        lib().om_thermo(self.h, float(T), cp, h, s)
        return cp, h, s

    def rates(self, p, y, par=None):
        kf, kr, q = np.zeros(self.nr), np.zeros(self.nr), np.zeros(self.nr)
        lib().om_rates(self.h, _ptr(par), float(p), np.ascontiguousarray(y, dtype=float), kf, kr, q)
        return kf, kr, q

    def rhs(self, p, y, par=None):
        f = np.zeros(self.n)
        lib().om_rhs(self.h, _ptr(par), float(p), np.ascontiguousarray(y, dtype=float), f)
        return f

    def jac(self, p, y, par=None):
        J = np.zeros((self.n, self.n))
        lib().om_jac(self.h, _ptr(par), float(p), np.ascontiguousarray(y, dtype=float), J.reshape(-1))
        return J

    def jac_cs(self, p, y, par=None):
        J = np.zeros((self.n, self.n))
        lib().om_jac_cs(self.h, _ptr(par), float(p), np.ascontiguousarray(y, dtype=float), J.reshape(-1))
        return J

    # ---- Rosenbrock ----
    def step(self, p, y, h, method=RODAS4, par=None):
        yn, e = np.zeros(self.n), np.zeros(self.n)
        rc = lib().om_step(self.h, _ptr(par), method, float(p), np.ascontiguousarray(y, dtype=float),
                           float(h), yn, e)
        if rc:
            raise RuntimeError("singular step matrix")
        return yn, e

    def count_step(self, p, y, h):
        """Counted mode: the arithmetic of one RODAS4 step attempt from y with
        step h (the mechanism's own parameters), as a dict of add (including
        subtractions), mul, div, exp and log counts, plus flop = add + mul + div."""
        out = np.zeros(5, dtype=np.int64)
        rc = lib().om_count_step(self.h, float(p), np.ascontiguousarray(y, dtype=float), float(h), out)
        if rc:
            raise RuntimeError("singular step matrix")
        d = dict(zip(("add", "mul", "div", "exp", "log"), (int(v) for v in out)))
        d["flop"] = d["add"] + d["mul"] + d["div"]
        return d

    def integrate(self, T, p, Y, dt, rtol, atol, method=RODAS4, max_substeps=100000,
                  hmin_rel=1e-20, par=None, nthreads=0):
        """Returns (T_end, Y_end, nacc, nrej, status); inputs are not modified."""
        T = np.array(T, dtype=float, copy=True).reshape(-1)
        Y = np.array(Y, dtype=float, copy=True).reshape(T.size, self.ns)
        p = np.ascontiguousarray(np.broadcast_to(np.asarray(p, dtype=float), T.shape))
        nacc = np.zeros(T.size, dtype=np.int32)
        nrej = np.zeros(T.size, dtype=np.int32)
        st = np.zeros(T.size, dtype=np.int32)
        o = Opts(method, max_substeps, hmin_rel)
        lib().om_integrate(self.h, _ptr(par), T.size, T, p, Y.reshape(-1), float(dt), float(rtol),
                           float(atol), C.byref(o), nacc, nrej, st, int(nthreads))
        return T, Y, nacc, nrej, st

    def step_sizes(self, T, p, Y, dt, rtol, atol, method=RODAS4, par=None, cap=1 << 16):
        hs = np.zeros(cap)
        nh = C.c_int(0)
        o = Opts(method, 100000, 1e-20)
        rc = lib().om_step_sizes(self.h, _ptr(par), float(T), float(p),
                                 np.ascontiguousarray(Y, dtype=float), float(dt), float(rtol),
                                 float(atol), C.byref(o), cap, hs, C.byref(nh))
        if rc != 0:
            raise RuntimeError(f"oracle step_sizes failed rc={rc}")
        return hs[: nh.value].copy()

    def replay(self, p, y0, hs, method=RODAS4, par=None):
        out = np.zeros(self.n)
        hs = np.ascontiguousarray(hs, dtype=float)
        rc = lib().om_replay(self.h, _ptr(par), method, float(p), np.ascontiguousarray(y0, dtype=float),
                             hs.size, hs, out)
        if rc:
            raise RuntimeError("replay failed")
        return out

    def replay_dir(self, p, y0, hs, dy0=None, dpar=None, method=RODAS4):
        out = np.zeros(self.n)
        hs = np.ascontiguousarray(hs, dtype=float)
        dy0 = None if dy0 is None else np.ascontiguousarray(dy0, dtype=float)
        dpar = None if dpar is None else np.ascontiguousarray(dpar, dtype=float)
        rc = lib().om_replay_dir(self.h, method, float(p), np.ascontiguousarray(y0, dtype=float),
                                 hs.size, hs, _ptr(dy0), _ptr(dpar), out)
        if rc:
            raise RuntimeError("replay_dir failed")
        return out

    def adjoint(self, T0, p, Y0, dt, rtol, atol, gT, gY, method=RODAS4, nthreads=0):
        T0 = np.ascontiguousarray(T0, dtype=float).reshape(-1)
        n = T0.size
        Y0 = np.ascontiguousarray(Y0, dtype=float).reshape(-1)
        p = np.ascontiguousarray(np.broadcast_to(np.asarray(p, dtype=float), T0.shape))
        gT = np.ascontiguousarray(np.broadcast_to(np.asarray(gT, dtype=float), T0.shape))
        gY = np.ascontiguousarray(np.broadcast_to(np.asarray(gY, dtype=float), (n, self.ns))).reshape(-1)
        gT0, gY0 = np.zeros(n), np.zeros(n * self.ns)
        ga, gb, ge = np.zeros(self.nr), np.zeros(self.nr), np.zeros(self.nr)
        o = Opts(method, 100000, 1e-20)
        rc = lib().om_adjoint(self.h, method, n, T0, p, Y0, float(dt), float(rtol), float(atol),
                              C.byref(o), gT, gY, gT0, gY0, ga, gb, ge, int(nthreads))
        if rc:
            raise RuntimeError("oracle adjoint failed")
        return gT0, gY0.reshape(n, self.ns), ga, gb, ge


def chemkin_mechanism(path, thermo=None):
    """A Mechanism from a CHEMKIN-format file (thermo: optional separate
    thermo file), through the converter in oracle/chemkin.py."""
    import os
    import tempfile
    from . import chemkin
    text = pathlib.Path(path).read_text()
    ttext = pathlib.Path(thermo).read_text() if thermo else None
    fd, tmp = tempfile.mkstemp(suffix=".mech")
    try:
        with os.fdopen(fd, "w") as f:
            f.write(chemkin.convert(text, ttext, name=pathlib.Path(path).stem))
        return Mechanism(tmp)
    finally:
        os.unlink(tmp)


def openfoam_mechanism(reactions, thermo):
    """A Mechanism from an OpenFOAM reactions/thermo dictionary pair, through
    the converter in oracle/foam.py."""
    import os
    import tempfile
    from . import foam
    text = foam.convert(pathlib.Path(reactions).read_text(), pathlib.Path(thermo).read_text(),
                        name=pathlib.Path(reactions).stem)
    fd, tmp = tempfile.mkstemp(suffix=".mech")
    try:
        with os.fdopen(fd, "w") as f:
            f.write(text)
        return Mechanism(tmp)
    finally:
        os.unlink(tmp)


def tableau(method=RODAS4):
    s, g = C.c_int(0), C.c_double(0)
    a, c, m, e = np.zeros(36), np.zeros(36), np.zeros(6), np.zeros(6)
    if lib().om_tableau(method, C.byref(s), C.byref(g), a, c, m, e):
        raise ValueError("unknown method")
    k = s.value
    return dict(s=k, gamma=g.value, a=a.reshape(6, 6)[:k, :k], c=c.reshape(6, 6)[:k, :k],
                m=m[:k], e=e[:k])


def lu(A):
    A = np.array(A, dtype=float, copy=True)
    n = A.shape[0]
    piv = np.zeros(n, dtype=np.int32)
    rc = lib().om_lu(n, A.reshape(-1), piv)
    return A, piv, rc


def lu_solve(LU, piv, b):
    b = np.array(b, dtype=float, copy=True)
    lib().om_lu_solve(LU.shape[0], np.ascontiguousarray(LU), piv, b)
    return b
