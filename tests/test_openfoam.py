"""OpenFOAM chemistry dictionaries: the oracle's converter (oracle/foam.py)
against values the format fixes, the library's reader (chem_load_openfoam)
against the converter, and both against the `chemmi-mech 1` files of the same
mechanisms.  No GPU.

Fixture tests/golden/foam_small/{reactions,thermo}: nine species, made-up
rates in OpenFOAM's kmol units, one reaction of every supported type, the
older "...Reaction" type name, an equation without spaces, Lindemann with an
empty F, a single-collider efficiency list."""
import ctypes as C
import pathlib

import numpy as np
import pytest

from workloads import gen_mech, mech_path

ROOT = pathlib.Path(__file__).resolve().parents[1]
FX = ROOT / "tests" / "golden" / "foam_small"
RU = 8.314462618


@pytest.fixture(scope="module")
def L():
    from paper_2508_16105_amd import _lib
    return _lib.lib()


def test_converter_reads_the_fixture_as_the_format_defines(oracle_lib):
    from oracle import foam
    txt = foam.convert((FX / "reactions").read_text(), (FX / "thermo").read_text())
    r = [l.split() for l in txt.splitlines() if l.startswith("reaction")]
    kinds = [x[1] for x in r]
    assert kinds == ["elementary", "elementary", "elementary", "thirdbody", "troe", "sri", "elementary",
                     "lindemann"]
    # A: (m^3/kmol)^(n-1)/s -> (cm^3/mol)^(n-1)/s is x 1e3 per order above one
    assert float(r[0][4]) == pytest.approx(2e11 * 1e3, rel=1e-15)
    assert float(r[1][4]) == pytest.approx(50.0 * 1e3, rel=1e-15)
    assert float(r[3][4]) == pytest.approx(1e12 * 1e6, rel=1e-15)              # 2H + M: order 3
    assert float(r[4][4]) == pytest.approx(4.5e9 * 1e3, rel=1e-15)             # k_inf: order 2
    assert float(r[4][7]) == pytest.approx(6e13 * 1e6, rel=1e-15)              # k0: order 3
    # Ta = Ea / R
    assert float(r[0][6]) == pytest.approx(8050.0 * RU / 1e3, rel=1e-15)
    assert float(r[2][6]) == pytest.approx(-1057.0 * RU / 1e3, rel=1e-15)
    assert r[2][2:4] == ["O=1,H2O=1", "OH=2"] and r[3][2:4] == ["H=2", "H2=1"]
    assert [float(x) for x in r[4][10:14]] == [0.5, 1e-30, 1e30, 1e30]           # alpha T*** T* T**
    assert [float(x) for x in r[5][10:15]] == [0.45, 797.0, 979.0, 1.0, 0.0]
    assert r[6][-1] == "irrev" and r[5][2:4] == ["H=1,OH=1", "H2O=1"]
    w = {l.split()[1]: l.split()[3] for l in txt.splitlines() if l.startswith("species")}
    assert w["H2O"] == "W=18.015" and w["AR"] == "W=39.95"


def test_library_reader_matches_the_converter(L, oracle_lib):
    from paper_2508_16105_amd import _lib
    om = oracle_lib.openfoam_mechanism(FX / "reactions", FX / "thermo")
    h = _lib.load_mechanism_handle(str(FX / "reactions"), str(FX / "thermo"), "openfoam")
    ns, nr = C.c_int(), C.c_int()
    L.chem_mechanism_info(h, C.byref(ns), C.byref(nr))
    assert (ns.value, nr.value) == (om.ns, om.nr) == (9, 8)
    a, b, e = (np.zeros(8) for _ in range(3))
    L.chem_get_params(h, a.ctypes.data, b.ctypes.data, e.ctypes.data)
    oa, ob, oe = om.params()
    assert np.allclose(a, oa, rtol=0, atol=1e-13) and np.array_equal(b, ob)
    assert np.allclose(e, oe, rtol=1e-14, atol=1e-12)
    assert e[0] == pytest.approx(8050.0 * RU, rel=1e-15)
    L.chem_free_mechanism(h)


@pytest.mark.parametrize("name,library", [("m9", True), ("m13", False), ("m32", False), ("m32s", True)])
def test_generated_mechanisms_read_back(L, oracle_lib, tmp_path, name, library):
    """The seeded mechanisms written as OpenFOAM dictionaries read back to the
    native files' parameters and weights (A through the kmol conversion to
    round-off; the library side for m9 and m32s, whose device code is
    prebuilt)."""
    from paper_2508_16105_amd import _lib
    rtext, ttext = gen_mech.to_openfoam(gen_mech.build_mechanism(name))
    rp, tp = tmp_path / f"{name}.foam", tmp_path / "thermo"
    rp.write_text(rtext)
    tp.write_text(ttext)
    ref = oracle_lib.Mechanism(mech_path(name))
    ra, rb, re_ = ref.params()
    o = oracle_lib.openfoam_mechanism(rp, tp)
    oa, ob, oe = o.params()
    assert np.allclose(oa, ra, rtol=0, atol=1e-13) and np.array_equal(ob, rb)
    assert np.allclose(oe, re_, rtol=1e-14, atol=1e-9)
    assert np.allclose(o.weights(), ref.weights(), rtol=1e-15, atol=0)
    for T in (300.0, 1000.0, 2500.0):
        for x, y in zip(o.thermo(T), ref.thermo(T)):
            assert np.array_equal(x, y)
    if not library:
        return
    h = _lib.load_mechanism_handle(str(rp), str(tp), "openfoam")
    a, b, e = (np.zeros(len(ra)) for _ in range(3))
    L.chem_get_params(h, a.ctypes.data, b.ctypes.data, e.ctypes.data)
    assert np.allclose(a, ra, rtol=0, atol=1e-13) and np.array_equal(b, rb)
    assert np.allclose(e, re_, rtol=1e-14, atol=1e-9)
    L.chem_free_mechanism(h)


REACTIONS = (FX / "reactions").read_text()
THERMO = (FX / "thermo").read_text()


@pytest.mark.parametrize("which,old,new,code,what", [
    ("r", "type     irreversibleArrhenius;", "type     irreversibleArrheniusPLOG;", -8, "not supported"),
    ("r", '"HO2 + H = H2 + O2"', '"HO2 + H^1.5 = H2 + O2"', -8, "orders"),
    ("r", '"HO2 + H = H2 + O2"', '"HO2 + H = H2 + O"', -3, "balanced"),
    ("r", '"O + H2 = H + OH"', '"O + H2 = H + OX"', -2, "OX"),
    ("r", "        Ta       3170;\n", "", -2, "Ta"),
    ("t", "AR\n{", "ARGON\n{", -3, "AR"),
    ("r", "species 9 ( H2 O2 H O OH H2O HO2 N2 AR );", "species 9 ( H2 O2 H O OH H2O HO2 N2 AR ;", -2, "species"),
])
def test_library_reader_errors(L, tmp_path, which, old, new, code, what):
    r, t = REACTIONS, THERMO
    if which == "r":
        assert old in r
        r = r.replace(old, new, 1)
    else:
        assert old in t
        t = t.replace(old, new, 1)
    (tmp_path / "reactions").write_text(r)
    (tmp_path / "thermo").write_text(t)
    h = C.c_void_p()
    rc = L.chem_load_openfoam(str(tmp_path / "reactions").encode(), str(tmp_path / "thermo").encode(), C.byref(h))
    msg = L.chem_last_error().decode()
    assert rc == code and what in msg, (rc, msg)
