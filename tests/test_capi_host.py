"""The C-ABI library on the host (no GPU): it loads, exports every declared
entry point, and reports argument and mechanism errors with the declared
codes before touching a device."""
import ctypes as C
import pathlib
import re

import pytest

from workloads import mech_path, tiny

ROOT = pathlib.Path(__file__).resolve().parents[1]


@pytest.fixture(scope="module")
def L():
    from paper_2508_16105_amd import _lib
    return _lib.lib()


def test_exports_every_declared_function(L):
    header = (ROOT / "include" / "chem.h").read_text()
    declared = set(re.findall(r"^\s*(?:int|void|const char \*)\s*\*?(chem_\w+)\s*\(", header, re.M))
    assert {"chem_load_mechanism", "chem_integrate", "chem_integrate_adjoint",
            "chem_integrate_batched"} <= declared
    for name in declared:
        assert hasattr(L, name), name
    from paper_2508_16105_amd import _lib
    assert declared == set(_lib.EXPORTS)


def test_version(L):
    assert b"gfx950" in L.chem_version()


def _load(L, path):
    h = C.c_void_p()
    rc = L.chem_load_mechanism(str(path).encode(), C.byref(h))
    return rc, h


def test_load_errors(L, write_mech):
    assert _load(L, "/nonexistent.mech")[0] == -1
    assert _load(L, write_mech("not a mechanism\n", "bad1.mech"))[0] == -2
    txt = tiny.isomer_pair().replace("species B H=1,O=1", "species B H=2,O=1")
    rc, _ = _load(L, write_mech(txt, "bad2.mech"))
    assert rc == -3 and b"balanced" in L.chem_last_error()
    txt = tiny.isomer_pair().replace("end\n", "")
    assert _load(L, write_mech(txt, "bad3.mech"))[0] == -2


def test_load_generates_and_caches_device_code(L):
    from paper_2508_16105_amd import _lib
    h = _lib.load_mechanism_handle(mech_path("m9"))
    ns, nr = C.c_int(), C.c_int()
    assert L.chem_mechanism_info(h, C.byref(ns), C.byref(nr)) == 0
    assert (ns.value, nr.value) == (9, 21)
    L.chem_free_mechanism(h)


def test_params_roundtrip_and_argument_errors(L):
    import numpy as np
    from paper_2508_16105_amd import _lib
    import oracle
    h = _lib.load_mechanism_handle(mech_path("m9"))
    a, b, e = (np.zeros(21) for _ in range(3))
    assert L.chem_get_params(h, a.ctypes.data, b.ctypes.data, e.ctypes.data) == 0
    oa, ob, oe = oracle.Mechanism(mech_path("m9")).params()
    assert np.allclose(a, oa, rtol=1e-15) and np.allclose(b, ob) and np.allclose(e, oe, rtol=1e-14)
    e[3] = np.nan
    assert L.chem_set_params(h, a.ctypes.data, b.ctypes.data, e.ctypes.data) == -1
    # argument checks come before any device work
    assert L.chem_integrate(h, 10, None, None, None, -1.0, 1e-8, 1e-12, None, None, None, None,
                            None, None) == -1
    assert L.chem_integrate(h, 10, None, None, None, 1e-8, 0.0, 1e-12, None, None, None, None,
                            None, None) == -1
    assert L.chem_integrate(h, 0, None, None, None, 1e-8, 1e-8, 1e-12, None, None, None, None,
                            None, None) == 0
    assert L.chem_integrate(None, 10, None, None, None, 1e-8, 1e-8, 1e-12, None, None, None, None,
                            None, None) == -1
    # the coupled step: the same checks, and host pointers refused before any launch
    host = np.zeros(10)
    assert L.chem_integrate_source(h, 10, None, None, None, -1.0, 1e-8, 1e-12, None, None, None, None,
                                   None, None) == -1
    assert L.chem_integrate_source(h, 0, None, None, None, 1e-8, 1e-8, 1e-12, None, None, None, None,
                                   None, None) == 0
    assert L.chem_integrate_source(h, 10, host.ctypes.data, host.ctypes.data, host.ctypes.data, 1e-8, 1e-8,
                                   1e-12, host.ctypes.data, host.ctypes.data, None, None, None, None) == -1
    assert L.chem_integrate_source(None, 10, None, None, None, 1e-8, 1e-8, 1e-12, None, None, None, None,
                                   None, None) == -1
    # the 1D driver: the same checks before any launch
    assert L.chem_euler1d_step(h, 0, 1e-4, 1e-9, None, None, None, 1e-8, 1e-12, None, None, None, None) == -1
    assert L.chem_euler1d_step(h, 8, 0.0, 1e-9, None, None, None, 1e-8, 1e-12, None, None, None, None) == -1
    assert L.chem_euler1d_step(h, 8, 1e-4, -1.0, None, None, None, 1e-8, 1e-12, None, None, None, None) == -1
    assert L.chem_euler1d_step(h, 8, 1e-4, 1e-9, host.ctypes.data, host.ctypes.data, host.ctypes.data, 1e-8,
                               1e-12, None, None, None, None) == -1
    assert L.chem_euler1d_init(h, 0, None, None, None, None, None, None) == 0
    assert L.chem_euler1d_init(h, 8, host.ctypes.data, host.ctypes.data, host.ctypes.data, None,
                               host.ctypes.data, None) == -1
    L.chem_free_mechanism(h)


def test_product_path_never_reaches_the_oracle():
    """The library and its binding neither import, link nor name the oracle,
    and libchemmi.so needs no oracle symbol."""
    pkg = ROOT / "paper_2508_16105_amd"
    for f in list(pkg.rglob("*.py")) + list((pkg / "csrc").rglob("*.[ch]pp")) + list((pkg / "csrc").rglob("*.hip")):
        text = f.read_text()
        assert not re.search(r"\boracle\b|liboracle|om_\w+\(", text), f
    so = (pkg / "libchemmi.so").read_bytes()
    assert b"liboracle" not in so
    for name in set(re.findall(r"\b(om_\w+)\(", (ROOT / "oracle" / "oracle.h").read_text())):
        assert name.encode() + b"\0" not in so, name


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    """Without the built library the binding raises at once: there is no
    fallback path."""
    from paper_2508_16105_amd import _lib
    monkeypatch.setattr(_lib, "_lib", None)
    monkeypatch.setattr(_lib, "LIB_PATH", tmp_path / "libchemmi.so")
    with pytest.raises(ImportError, match="not built"):
        _lib.lib()
