"""One suite over both servers of the chemistry-step C ABI: the oracle's host
ABI (runs here, on the CPU) and the GPU library (marked gpu).  Each test
checks conventions the ABI states -- argument errors, the no-op of zero
cells, per-cell status codes and what a failed cell keeps, the statistics,
the parameter set/get round trip -- on whichever backend it is given, and the
last test compares the two backends' results on the same cells."""
import math

import numpy as np
import pytest

from abi_backends import (CELL_BADINPUT, CELL_HMIN, CELL_MAXSTEPS, CELL_OK, E_CELL_FAILED, E_INVAL,
                          E_MECH_INVALID, E_PARSE, backend)
from workloads import mech_path, mech_text
from workloads.states import uniform_cells

BACKENDS = ["oracle", pytest.param("gpu", marks=pytest.mark.gpu)]
RTOL, ATOL = 1e-8, 1e-12


@pytest.fixture(scope="module", params=BACKENDS)
def be(request):
    if request.param == "gpu":
        torch = pytest.importorskip("torch")
        assert torch.cuda.is_available(), "GPU tests need a GPU"
    return backend(request.param)


@pytest.fixture(scope="module")
def m9(be):
    rc, h = be.load(mech_path("m9"))
    assert rc == 0, be.last_error()
    yield h
    be.free(h)


def _cells(n, seed):
    return uniform_cells(mech_text("m9"), n, seed)


def test_load_errors(be, tmp_path):
    rc, _ = be.load(tmp_path / "missing.mech")
    assert rc == E_INVAL and be.last_error()
    text = mech_text("m9")
    bad = tmp_path / "syntax.mech"
    bad.write_text(text.replace("reaction elementary", "reaction bogus-kind", 1))
    rc, _ = be.load(bad)
    assert rc == E_PARSE, be.last_error()
    # H2O2 + H -> H2O + OH with one O atom dropped from the products
    unbal = tmp_path / "unbalanced.mech"
    unbal.write_text(text.replace("reaction elementary H=1,H2O2=1 H2O=1,OH=1",
                                  "reaction elementary H=1,H2O2=1 H2O=1,H=1", 1))
    rc, _ = be.load(unbal)
    assert rc == E_MECH_INVALID, be.last_error()


def test_info_and_params_round_trip(be, m9):
    rc, ns, nr = be.info(m9)
    assert rc == 0 and (ns, nr) == (9, 21)
    rc, a, b, e = be.get_params(m9, nr)
    assert rc == 0 and np.all(np.isfinite(a)) and np.all(e > 0)
    T, p, Y = _cells(16, 3)
    base = be.integrate(m9, T, p, Y, 1e-8, RTOL, ATOL)
    assert be.set_params(m9, a + math.log(2.0), b, e) == 0     # every rate doubles
    fast = be.integrate(m9, T, p, Y, 1e-8, RTOL, ATOL)
    assert not np.array_equal(fast[1], base[1])
    assert be.set_params(m9, a, b, e) == 0
    again = be.integrate(m9, T, p, Y, 1e-8, RTOL, ATOL)
    assert np.array_equal(again[1], base[1]) and np.array_equal(again[2], base[2])
    bad = a.copy()
    bad[4] = np.nan
    assert be.set_params(m9, bad, b, e) == E_INVAL and be.last_error()
    assert np.array_equal(be.get_params(m9, nr)[1], a)


def test_zero_cells_is_a_no_op(be, m9):
    e, e2 = np.zeros(0), np.zeros((0, 9))
    rc, T, Y, st, na, nj, s = be.integrate(m9, e, e, e2, 1e-8, RTOL, ATOL)
    assert rc == 0 and s["cells"] == 0 and s["failed"] == 0
    assert be.eval_source(m9, e, e, e2)[0] == 0
    assert be.step_fixed(m9, e, e, e2, 1e-9, RTOL, ATOL)[0] == 0
    out = be.adjoint(m9, e, e, e2, 1e-8, RTOL, ATOL, e, e2, 21)
    assert out[0] == 0 and np.all(out[3] == 0) and np.all(out[4] == 0) and np.all(out[5] == 0)


@pytest.mark.parametrize("what", ["dt0", "dtinf", "rtol0", "atolneg", "nullT"])
def test_argument_errors(be, m9, what):
    T, p, Y = _cells(4, 4)
    dt, rtol, atol, null = 1e-8, RTOL, ATOL, ()
    if what == "dt0":
        dt = 0.0
    elif what == "dtinf":
        dt = math.inf
    elif what == "rtol0":
        rtol = 0.0
    elif what == "atolneg":
        atol = -1.0
    else:
        null = ("T",)
    rc, Tout, Yout = be.integrate(m9, T, p, Y, dt, rtol, atol, null=null)[:3]
    assert rc == E_INVAL and be.last_error()
    if what != "nullT":
        assert np.array_equal(Tout, T) and np.array_equal(Yout, Y)      # nothing was done
    if what in ("dt0", "rtol0"):
        assert be.step_fixed(m9, T, p, Y, dt, rtol, atol)[0] == E_INVAL


def test_adjoint_argument_errors(be, m9):
    T, p, Y = _cells(4, 5)
    gT, gY = np.ones(4), np.ones((4, 9))
    assert be.adjoint(m9, T, p, Y, 1e-8, RTOL, ATOL, gT, gY, 21, ends=(True, False))[0] == E_INVAL
    assert be.adjoint(m9, T, p, Y, 1e-8, RTOL, ATOL, gT, gY, 21, checkpoint_every=17)[0] == E_INVAL
    assert be.last_error()


def test_bad_input_cells_are_untouched_and_counted(be, m9):
    T, p, Y = _cells(12, 6)
    T[2], p[5], Y[8, 3] = -1.0, 0.0, np.nan
    rc, Tout, Yout, st, na, nj, s = be.integrate(m9, T, p, Y, 1e-8, RTOL, ATOL)
    bad = [2, 5, 8]
    assert rc == E_CELL_FAILED and be.last_error()
    assert s["failed"] == 3 and s["cells"] == 12
    assert np.all(st[bad] == CELL_BADINPUT)
    assert np.array_equal(Tout[bad], T[bad]) and np.array_equal(Yout[bad], Y[bad], equal_nan=True)
    good = [i for i in range(12) if i not in bad]
    assert np.all(st[good] == CELL_OK)
    alone = be.integrate(m9, T[good], p[good], Y[good], 1e-8, RTOL, ATOL)
    assert alone[0] == 0
    assert np.array_equal(alone[1], Tout[good]) and np.array_equal(alone[2], Yout[good])
    # without statistics the call reports success; the status still shows the failures
    rc2, _, _, st2 = be.integrate(m9, T, p, Y, 1e-8, RTOL, ATOL, stats=False)[:4]
    assert rc2 == 0 and np.array_equal(st2, st)


def test_substep_limit_and_step_floor(be, m9):
    T, p, Y = _cells(32, 7)
    full = be.integrate(m9, T, p, Y, 1e-7, RTOL, ATOL)
    assert full[0] == 0
    rc, Tout, Yout, st, na, nj, s = be.integrate(m9, T, p, Y, 1e-7, RTOL, ATOL, max_substeps=3)
    over = full[4] + full[5] > 3
    assert over.sum() >= 8 and rc == E_CELL_FAILED
    assert np.all(st[over] == CELL_MAXSTEPS) and np.all(na[over] + nj[over] == 3)
    assert np.all(st[~over] == CELL_OK) and s["failed"] == over.sum()
    assert np.all(np.isfinite(Tout)) and np.all(Tout[over] != full[1][over])   # last accepted state
    rc, Tout, Yout, st, na, nj, s = be.integrate(m9, T, p, Y, 1e-7, RTOL, ATOL, hmin_rel=0.5)
    assert rc == E_CELL_FAILED and np.any(st == CELL_HMIN) and s["failed"] == (st != CELL_OK).sum()
    assert np.all(st[full[4] + full[5] == 1] == CELL_OK)          # one step of dt never falls below


def test_statistics_match_the_counters(be, m9):
    T, p, Y = _cells(40, 8)
    rc, Tout, Yout, st, na, nj, s = be.integrate(m9, T, p, Y, 1e-8, RTOL, ATOL)
    assert rc == 0 and s["cells"] == 40 and s["failed"] == 0
    assert s["accepted"] == na.sum() and s["rejected"] == nj.sum()
    assert s["max_substeps"] == (na + nj).max()


def test_adjoint_conventions(be, m9):
    T, p, Y = _cells(10, 9)
    gT, gY = np.full(10, 1e-3), np.ones((10, 9))
    out = be.adjoint(m9, T, p, Y, 1e-8, RTOL, ATOL, gT, gY, 21)
    assert out[0] == 0 and np.all(np.isfinite(out[1])) and np.all(np.isfinite(out[2]))
    fwd = be.integrate(m9, T, p, Y, 1e-8, RTOL, ATOL)
    assert np.array_equal(out[6], fwd[1]) and np.array_equal(out[7], fwd[2])     # forward result
    T[4] = -5.0
    bad = be.adjoint(m9, T, p, Y, 1e-8, RTOL, ATOL, gT, gY, 21)
    assert bad[0] == E_CELL_FAILED and np.isnan(bad[1][4]) and np.all(np.isnan(bad[2][4]))
    # the other cells' gradients are unchanged up to the order of a step's
    # second-order sum (the GPU may split it over lanes for other cells)
    keep = [i for i in range(10) if i != 4]
    assert np.allclose(bad[1][keep], out[1][keep], rtol=1e-11, atol=0)
    only = be.adjoint(m9, T[keep], p[keep], Y[keep], 1e-8, RTOL, ATOL, gT[keep], gY[keep], 21)
    for i in (3, 4, 5):       # a failed cell adds nothing to the parameter sums
        assert np.allclose(bad[i], only[i], rtol=1e-11, atol=0)


@pytest.mark.gpu
def test_backends_agree():
    """The same cells through both servers: source terms and Jacobian, one
    fixed step, the adaptive integration and the adjoint."""
    torch = pytest.importorskip("torch")
    assert torch.cuda.is_available()
    o, g = backend("oracle"), backend("gpu")
    ho, hg = o.load(mech_path("m9"))[1], g.load(mech_path("m9"))[1]
    T, p, Y = _cells(64, 10)
    fo, Jo = o.eval_source(ho, T, p, Y, jac=True)[1:]
    fg, Jg = g.eval_source(hg, T, p, Y, jac=True)[1:]
    assert np.all(np.abs(fg - fo) <= 1e-11 * np.abs(fo).max(axis=1, keepdims=True))
    assert np.all(np.abs(Jg - Jo) <= 1e-9 * np.abs(Jo).max(axis=(1, 2), keepdims=True))
    so, sg = o.step_fixed(ho, T, p, Y, 1e-10, RTOL, ATOL), g.step_fixed(hg, T, p, Y, 1e-10, RTOL, ATOL)
    assert np.array_equal(so[3], sg[3])
    assert np.all(np.abs(sg[1] - so[1]) <= 1e-12 * np.abs(so[1]).max(axis=1, keepdims=True))
    io, ig = o.integrate(ho, T, p, Y, 1e-8, RTOL, ATOL), g.integrate(hg, T, p, Y, 1e-8, RTOL, ATOL)
    assert io[0] == ig[0] == 0 and np.array_equal(io[3], ig[3])
    assert np.all(np.abs(ig[1] - io[1]) <= 1e-6 * io[1])
    assert np.all(np.abs(ig[2] - io[2]) <= 1e-8)
    gT, gY = np.full(64, 1e-3), np.ones((64, 9))
    ao = o.adjoint(ho, T, p, Y, 1e-8, RTOL, ATOL, gT, gY, 21)
    ag = g.adjoint(hg, T, p, Y, 1e-8, RTOL, ATOL, gT, gY, 21)
    assert ao[0] == ag[0] == 0
    assert np.median(np.abs(ag[1] - ao[1]) / np.abs(ao[1])) <= 1e-6
    for i in (3, 4, 5):
        assert np.max(np.abs(ag[i] - ao[i])) <= 1e-4 * np.max(np.abs(ao[i]))
    o.free(ho)
    g.free(hg)


def test_oracle_abi_exports_every_declared_function():
    import ctypes as C
    import pathlib
    import re

    import oracle
    oracle.lib()
    header = (pathlib.Path(oracle.__file__).parent / "oracle_abi.h").read_text()
    names = set(re.findall(r"\b(oracle_[a-z_0-9]+)\s*\(", header))
    assert len(names) >= 10
    L = C.CDLL(str(oracle.LIB))
    missing = [n for n in sorted(names) if not hasattr(L, n)]
    assert not missing, missing
