"""MI355X (gfx950) per-cell stiff-chemistry step.

Python binding of libchemmi.so: torch supplies device memory and streams, the
library's HIP kernels do every step of the computation.  Nothing here falls
back to the CPU: without the built library (or without a gfx950 device) the
calls raise.

    mech = Mechanism("workloads/mech/m9.mech")
    T, Y, stats = integrate(mech, T, p, Y, dt=5e-9, rtol=1e-8, atol=1e-12)
"""
from __future__ import annotations

import ctypes as C

from . import _lib
from ._lib import ChemError, FORM_AUTO, FORM_PERSISTENT, FORM_PLAIN, ORDER_COST, ORDER_NATURAL

__all__ = ["Mechanism", "integrate", "integrate_noalloc", "integrate_source", "integrate_batched", "integrate_adjoint", "eval_source",
           "step_fixed", "euler1d_init", "euler1d_step", "ChemIntegrate", "ChemError", "FORM_AUTO", "FORM_PLAIN",
           "FORM_PERSISTENT", "ORDER_COST", "ORDER_NATURAL", "version"]


def _torch():
    import torch
    return torch


def version() -> str:
    return _lib.lib().chem_version().decode()


def _stream(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _check_tensor(t, name, shape=None, dtype=None):
    torch = _torch()
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if not t.is_cuda:
        raise ValueError(f"{name} must be on the GPU")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.dtype != (dtype or torch.float64):
        raise ValueError(f"{name} must be {dtype or torch.float64}")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")


class Mechanism:
    """A loaded mechanism: a `chemmi-mech 1` or CHEMKIN file
    (chem_load_mechanism), a CHEMKIN file with its thermo data in a second
    file (chem_load_chemkin), or an OpenFOAM reactions/thermo pair
    (fmt="openfoam", chem_load_openfoam)."""

    def __init__(self, path, thermo=None, fmt=None):
        self.path = str(path)
        self.h = _lib.load_mechanism_handle(self.path, thermo, fmt)
        ns, nr = C.c_int(), C.c_int()
        _lib.check(_lib.lib().chem_mechanism_info(self.h, C.byref(ns), C.byref(nr)))
        self.ns, self.nr = ns.value, nr.value
        self.n = self.ns + 1

    def __del__(self, _libmod=_lib):
        # the module is bound as a default: at interpreter exit the global name
        # may already be gone, and then the library is left to the process end
        h = getattr(self, "h", None)
        lib = getattr(_libmod, "_lib", None)
        if h and lib is not None:
            lib.chem_free_mechanism(h)
            self.h = None

    def get_params(self):
        import numpy as np
        a, b, e = (np.zeros(self.nr) for _ in range(3))
        _lib.check(_lib.lib().chem_get_params(self.h, a.ctypes.data, b.ctypes.data, e.ctypes.data))
        return a, b, e

    def set_params(self, lnA, b, Ea):
        import numpy as np
        a, bb, e = (np.ascontiguousarray(np.asarray(x, dtype=float).reshape(self.nr)) for x in (lnA, b, Ea))
        _lib.check(_lib.lib().chem_set_params(self.h, a.ctypes.data, bb.ctypes.data, e.ctypes.data))


def _options(form=FORM_AUTO, max_substeps=0, hmin_rel=0.0, h0=None, checkpoint_every=0, block=0,
             waves_per_simd=0, refill=0, order=0, cost=None, adjoint_nacc=None):
    """cost: None, or a list with one int32 GPU tensor (or None) per field."""
    carr = None
    if cost is not None:
        carr = (C.c_void_p * max(len(cost), 1))(*[None if c is None else c.data_ptr() for c in cost])
    o = _lib.Options(form, max_substeps, hmin_rel, None if h0 is None else h0.data_ptr(),
                     checkpoint_every, block, waves_per_simd, refill, order,
                     C.cast(carr, C.POINTER(C.c_void_p)) if carr is not None else None,
                     None if adjoint_nacc is None else adjoint_nacc.data_ptr())
    o._keep = carr
    return o


def integrate(mech: Mechanism, T, p, Y, dt, rtol, atol, *, form=FORM_PLAIN, stats=True,
              inplace=False, return_counts=False, stream=None, allow_failed=False, **opts):
    """Advance every cell over dt.  T, p: [ncell], Y: [ncell, ns], float64 on
    the GPU.  Returns (T_end, Y_end, stats dict or None[, status, nacc, nrej])."""
    torch = _torch()
    n = T.shape[0]
    for t, nm, sh in ((T, "T", (n,)), (p, "p", (n,)), (Y, "Y", (n, mech.ns))):
        _check_tensor(t, nm, sh)
    if not inplace:
        T, Y = T.clone(), Y.clone()
    st = nacc = nrej = None
    if return_counts:
        st, nacc, nrej = (torch.empty(n, dtype=torch.int32, device=T.device) for _ in range(3))
    s = _lib.Stats() if stats else None
    if opts.get("cost") is not None and not isinstance(opts["cost"], (list, tuple)):
        opts["cost"] = [opts["cost"]]
    o = _options(form=form, **opts)
    rc = _lib.lib().chem_integrate(mech.h, n, _ptr(T), _ptr(p), _ptr(Y), float(dt), float(rtol),
                                   float(atol), C.byref(o), C.byref(s) if s is not None else None,
                                   _ptr(st), _ptr(nacc), _ptr(nrej), _stream(stream))
    _lib.check(rc, allow=(-6,) if allow_failed else ())
    out = (T, Y, s.as_dict() if s is not None else None)
    return out + (st, nacc, nrej) if return_counts else out


def integrate_noalloc(mech: Mechanism, T, p, Y, dt, rtol, atol, *, status=None, nacc=None, nrej=None,
                      stream=None, **opts):
    """chem_integrate_noalloc: advance T [ncell] and Y [ncell, ns] in place
    with no device allocation (persistent form, the library's fixed scratch);
    status/nacc/nrej: optional int32 [ncell] GPU tensors.  Asynchronous."""
    n = T.shape[0]
    for t, nm, sh in ((T, "T", (n,)), (p, "p", (n,)), (Y, "Y", (n, mech.ns))):
        _check_tensor(t, nm, sh)
    torch = _torch()
    for t, nm in ((status, "status"), (nacc, "nacc"), (nrej, "nrej")):
        if t is not None:
            _check_tensor(t, nm, (n,), torch.int32)
    if opts.get("cost") is not None and not isinstance(opts["cost"], (list, tuple)):
        opts["cost"] = [opts["cost"]]
    o = _options(**opts)
    _lib.check(_lib.lib().chem_integrate_noalloc(mech.h, n, _ptr(T), _ptr(p), _ptr(Y), float(dt), float(rtol),
                                                  float(atol), C.byref(o), _ptr(status), _ptr(nacc), _ptr(nrej),
                                                  _stream(stream)))
    return T, Y


def integrate_source(mech: Mechanism, T, p, Y, dt, rtol, atol, *, form=FORM_PLAIN, stats=True,
                     inplace=False, return_status=False, stream=None, allow_failed=False, **opts):
    """Integrate as `integrate` does and return the operator-split reaction
    terms of the step (chem_integrate_source): (T_end, Y_end, wdot [ncell, ns]
    in kg/(m^3 s), qdot [ncell] in W/m^3, stats dict or None[, status])."""
    torch = _torch()
    n = T.shape[0]
    for t, nm, sh in ((T, "T", (n,)), (p, "p", (n,)), (Y, "Y", (n, mech.ns))):
        _check_tensor(t, nm, sh)
    if not inplace:
        T, Y = T.clone(), Y.clone()
    wdot = torch.empty((n, mech.ns), dtype=torch.float64, device=T.device)
    qdot = torch.empty(n, dtype=torch.float64, device=T.device)
    st = torch.empty(n, dtype=torch.int32, device=T.device) if return_status else None
    s = _lib.Stats() if stats else None
    if opts.get("cost") is not None and not isinstance(opts["cost"], (list, tuple)):
        opts["cost"] = [opts["cost"]]
    o = _options(form=form, **opts)
    rc = _lib.lib().chem_integrate_source(mech.h, n, _ptr(T), _ptr(p), _ptr(Y), float(dt), float(rtol),
                                          float(atol), _ptr(wdot), _ptr(qdot), C.byref(o),
                                          C.byref(s) if s is not None else None, _ptr(st), _stream(stream))
    _lib.check(rc, allow=(-6,) if allow_failed else ())
    out = (T, Y, wdot, qdot, s.as_dict() if s is not None else None)
    return out + (st,) if return_status else out


def euler1d_init(mech: Mechanism, T, p, Y, u=None, stream=None):
    """The 1D driver's conserved state [ncell, 3 + ns] from T, p, Y [ncell,
    ns] and u (None: at rest), on the GPU (chem_euler1d_init)."""
    torch = _torch()
    n = T.shape[0]
    for t, nm, sh in ((T, "T", (n,)), (p, "p", (n,)), (Y, "Y", (n, mech.ns))):
        _check_tensor(t, nm, sh)
    if u is not None:
        _check_tensor(u, "u", (n,))
    U = torch.empty((n, 3 + mech.ns), dtype=torch.float64, device=T.device)
    _lib.check(_lib.lib().chem_euler1d_init(mech.h, n, _ptr(T), _ptr(p), _ptr(Y), _ptr(u), _ptr(U),
                                            _stream(stream)))
    return U


def euler1d_step(mech: Mechanism, U, dx, dt, T=None, rtol=1e-8, atol=1e-12, *, form=FORM_PLAIN, stats=True,
                 stream=None, allow_failed=False, **opts):
    """One step of the 1D reactive-Euler driver (chem_euler1d_step).  U:
    [ncell, 3 + ns] conserved state (rho, rho u, rho E_s, rho Y_k) on the GPU;
    T: [ncell] temperature guess (None: 1000 K).  Returns (U_new, T of U,
    stats dict or None, max CFL number)."""
    torch = _torch()
    n = U.shape[0]
    _check_tensor(U, "U", (n, 3 + mech.ns))
    if T is None:
        T = torch.zeros(n, dtype=torch.float64, device=U.device)
    else:
        _check_tensor(T, "T", (n,))
        T = T.clone()
    Un = torch.empty_like(U)
    s = _lib.Stats() if stats else None
    o = _options(form=form, **opts)
    cfl = C.c_double(0.0)
    rc = _lib.lib().chem_euler1d_step(mech.h, n, float(dx), float(dt), _ptr(U), _ptr(Un), _ptr(T), float(rtol),
                                      float(atol), C.byref(o), C.byref(s) if s is not None else None,
                                      C.byref(cfl), _stream(stream))
    _lib.check(rc, allow=(-6,) if allow_failed else ())
    return Un, T, s.as_dict() if s is not None else None, cfl.value


def integrate_batched(mech: Mechanism, Ts, ps, Ys, dt, rtol, atol, *, form=FORM_PERSISTENT,
                      stats=True, stream=None, allow_failed=False, **opts):
    """Advance several fields in one launch (in place).  Returns stats."""
    nf = len(Ts)
    for i in range(nf):
        n = Ts[i].shape[0]
        _check_tensor(Ts[i], f"T[{i}]", (n,))
        _check_tensor(ps[i], f"p[{i}]", (n,))
        _check_tensor(Ys[i], f"Y[{i}]", (n, mech.ns))
    arr = C.c_void_p * max(nf, 1)
    Tp = arr(*[t.data_ptr() for t in Ts])
    pp = arr(*[t.data_ptr() for t in ps])
    Yp = arr(*[t.data_ptr() for t in Ys])
    nc = (C.c_int64 * max(nf, 1))(*[t.shape[0] for t in Ts])
    s = _lib.Stats() if stats else None
    o = _options(form=form, **opts)
    rc = _lib.lib().chem_integrate_batched(mech.h, nf, Tp, pp, Yp, nc, float(dt), float(rtol),
                                           float(atol), C.byref(o),
                                           C.byref(s) if s is not None else None, _stream(stream))
    _lib.check(rc, allow=(-6,) if allow_failed else ())
    return s.as_dict() if s is not None else None


def eval_source(mech: Mechanism, T, p, Y, jacobian=True, stream=None):
    """Source terms f = dy/dt [ncell, n] and Jacobian [ncell, n, n] (or None)."""
    torch = _torch()
    n = T.shape[0]
    for t, nm, sh in ((T, "T", (n,)), (p, "p", (n,)), (Y, "Y", (n, mech.ns))):
        _check_tensor(t, nm, sh)
    f = torch.empty((n, mech.n), dtype=torch.float64, device=T.device)
    J = torch.empty((n, mech.n, mech.n), dtype=torch.float64, device=T.device) if jacobian else None
    _lib.check(_lib.lib().chem_eval_source(mech.h, n, _ptr(T), _ptr(p), _ptr(Y), _ptr(f), _ptr(J),
                                           _stream(stream)))
    return f, J


def step_fixed(mech: Mechanism, T, p, Y, h, rtol=1e-8, atol=1e-12, stream=None):
    """One RODAS4 step of size h: (ynew [ncell, n], errnorm [ncell], ok [ncell])."""
    torch = _torch()
    n = T.shape[0]
    for t, nm, sh in ((T, "T", (n,)), (p, "p", (n,)), (Y, "Y", (n, mech.ns))):
        _check_tensor(t, nm, sh)
    yn = torch.empty((n, mech.n), dtype=torch.float64, device=T.device)
    en = torch.empty(n, dtype=torch.float64, device=T.device)
    ok = torch.empty(n, dtype=torch.int32, device=T.device)
    _lib.check(_lib.lib().chem_step_fixed(mech.h, n, _ptr(T), _ptr(p), _ptr(Y), float(h), float(rtol),
                                          float(atol), _ptr(yn), _ptr(en), _ptr(ok), _stream(stream)))
    return yn, en, ok


def integrate_adjoint(mech: Mechanism, T0, p, Y0, dt, rtol, atol, gT, gY, *, stats=True,
                      stream=None, checkpoint_every=0, allow_failed=False, forward_nacc=None, **opts):
    """Discrete adjoint of the frozen-step map.  Returns
    (gT0, gY0, g_lnA, g_b, g_Ea, T_end, Y_end, stats).  Failed cells (with
    allow_failed) get NaN gT0/gY0 and add nothing to the parameter gradients.
    forward_nacc: the int32 per-cell accepted steps of a forward integration
    of the same input (integrate's nacc), which spares the adjoint its own
    sizing pass."""
    torch = _torch()
    n = T0.shape[0]
    for t, nm, sh in ((T0, "T0", (n,)), (p, "p", (n,)), (Y0, "Y0", (n, mech.ns)),
                      (gT, "gT", (n,)), (gY, "gY", (n, mech.ns))):
        _check_tensor(t, nm, sh)
    dev = T0.device
    gT0 = torch.empty(n, dtype=torch.float64, device=dev)
    gY0 = torch.empty((n, mech.ns), dtype=torch.float64, device=dev)
    ga, gb, ge = (torch.empty(mech.nr, dtype=torch.float64, device=dev) for _ in range(3))
    Te = torch.empty(n, dtype=torch.float64, device=dev)
    Ye = torch.empty((n, mech.ns), dtype=torch.float64, device=dev)
    s = _lib.Stats() if stats else None
    if forward_nacc is not None:
        _check_tensor(forward_nacc, "forward_nacc", (n,), dtype=torch.int32)
    o = _options(checkpoint_every=checkpoint_every, adjoint_nacc=forward_nacc, **opts)
    rc = _lib.lib().chem_integrate_adjoint(
        mech.h, n, _ptr(T0), _ptr(p), _ptr(Y0), float(dt), float(rtol), float(atol), _ptr(gT),
        _ptr(gY), _ptr(gT0), _ptr(gY0), _ptr(ga), _ptr(gb), _ptr(ge), _ptr(Te), _ptr(Ye),
        C.byref(o), C.byref(s) if s is not None else None, _stream(stream))
    _lib.check(rc, allow=(-6,) if allow_failed else ())
    return gT0, gY0, ga, gb, ge, Te, Ye, (s.as_dict() if s is not None else None)


def _make_autograd():
    torch = _torch()

    class ChemIntegrate(torch.autograd.Function):
        """(T_end, Y_end) = step(T, Y; p, lnA, b, Ea) with the discrete adjoint
        as backward.  lnA, b, Ea: [n_reactions] tensors (their values are
        loaded into the mechanism before the forward)."""

        @staticmethod
        def forward(ctx, mech, T, p, Y, lnA, b, Ea, dt, rtol, atol):
            mech.set_params(lnA.detach().cpu().numpy(), b.detach().cpu().numpy(),
                            Ea.detach().cpu().numpy())
            # with stats the call waits for the result and raises ChemError
            # (CHEM_E_CELL_FAILED) if a cell failed, instead of handing back a
            # failed cell's last accepted partial state
            Te, Ye, _, _, nacc, _ = integrate(mech, T.detach(), p.detach(), Y.detach(), dt, rtol, atol,
                                              stats=True, return_counts=True)
            ctx.mech, ctx.dt, ctx.rtol, ctx.atol = mech, dt, rtol, atol
            ctx.nacc = nacc                  # spares the backward its sizing pass
            ctx.save_for_backward(T.detach(), p.detach(), Y.detach())
            ctx.params = (lnA.detach().cpu().numpy(), b.detach().cpu().numpy(), Ea.detach().cpu().numpy())
            return Te, Ye

        @staticmethod
        def backward(ctx, gTe, gYe):
            T, p, Y = ctx.saved_tensors
            mech = ctx.mech
            mech.set_params(*ctx.params)
            gTe = torch.zeros_like(T) if gTe is None else gTe.contiguous().to(torch.float64)
            gYe = torch.zeros_like(Y) if gYe is None else gYe.contiguous().to(torch.float64)
            gT0, gY0, ga, gb, ge, _, _, _ = integrate_adjoint(mech, T, p, Y, ctx.dt, ctx.rtol,
                                                              ctx.atol, gTe, gYe, stats=False,
                                                              forward_nacc=ctx.nacc)
            return None, gT0, None, gY0, ga, gb, ge, None, None, None

    return ChemIntegrate


class _Lazy:
    _cls = None

    def __getattr__(self, name):
        if _Lazy._cls is None:
            _Lazy._cls = _make_autograd()
        return getattr(_Lazy._cls, name)


ChemIntegrate = _Lazy()
