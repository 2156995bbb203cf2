"""The seeded input generators: reproducible, element-balanced, right sizes."""
import numpy as np
import pytest

from workloads import WORKLOADS, gen_mech, mech_path, mech_text
from workloads import states


@pytest.mark.parametrize("name", ["m9", "m13", "m32", "m13x", "m32x", "m32s", "m16"])
def test_committed_mechanisms_regenerate_exactly(name):
    assert gen_mech.build(name) == mech_text(name)


@pytest.mark.parametrize("name,ns,nr,ntroe,ntb", [("m9", 9, 21, 0, 0), ("m13", 13, 27, 3, 4),
                                                  ("m32", 32, 150, 15, 0)])
def test_mechanism_shape_and_balance(name, ns, nr, ntroe, ntb):
    txt = mech_text(name)
    lines = [l.split() for l in txt.splitlines() if l.strip()]
    sp = {l[1]: dict((kv.split("=")[0], int(kv.split("=")[1])) for kv in l[2].split(","))
          for l in lines if l[0] == "species"}
    rx = [l for l in lines if l[0] == "reaction"]
    assert len(sp) == ns and len(rx) == nr
    assert sum(1 for l in rx if l[1] == "troe") == ntroe
    assert sum(1 for l in rx if l[1] == "thirdbody") == ntb
    used = set()
    for l in rx:
        bal = {}
        for side, sgn in ((l[2], -1), (l[3], 1)):
            for kv in side.split(","):
                s, nu = kv.split("=")
                used.add(s)
                for e, c in sp[s].items():
                    bal[e] = bal.get(e, 0) + sgn * int(nu) * c
        assert all(v == 0 for v in bal.values()), l
        A, b, Ea = float(l[4]), float(l[5]), float(l[6])
        assert 8.0 <= np.log10(A) <= 17.0 and -1.5 <= b <= 2.0 and 0.0 <= Ea <= 200.0
    inert = {"N2"} if name == "m9" else {"AR", "HE"}
    assert set(sp) - inert <= used


def test_uniform_cells_distribution():
    T, p, Y = states.uniform_cells(mech_text("m9"), 4096, 100)
    assert T.shape == (4096,) and Y.shape == (4096, 9)
    assert T.min() >= 300 and T.max() <= 3000
    assert p.min() >= 101325 * 0.999 and p.max() <= 30 * 101325 * 1.001
    assert np.allclose(Y.sum(1), 1.0, atol=1e-14) and Y.min() > 0
    names, _ = states.parse_species(mech_text("m9"))
    m = Y.mean(0)
    assert abs(m[names.index("H2")] - 0.0285) < 2e-3 and abs(m[names.index("N2")] - 0.745) < 5e-3
    T2, _, _ = states.uniform_cells(mech_text("m9"), 4096, 100)
    assert np.array_equal(T, T2)


def test_rde_field_regions():
    T, p, Y, reg = states.rde_field(mech_text("m9"), 1024, 1024, 101)
    n = 1024 * 1024
    assert (reg == 1).sum() == 52429 and (reg == 2).sum() == 52429
    assert (reg == 0).sum() == n - 2 * 52429
    assert np.all(T[reg == 0] == 300.0) and np.all(p[reg == 0] == 101325.0)
    assert T[reg == 2].min() >= 2500 and T[reg == 1].max() <= 3500
    assert np.allclose(Y.sum(1), 1.0, atol=1e-13)
    # the front is a band: every row holds a contiguous run of front cells
    r = reg.reshape(1024, 1024)
    for row in (0, 511, 1023):
        idx = np.where(r[row] == 1)[0]
        assert idx.size > 0 and idx.max() - idx.min() + 1 == idx.size


def test_stoichiometric_mix():
    names, w = states.parse_species(mech_text("m9"))
    y = states.stoich_air(names, w)
    assert abs(y[names.index("H2")] - 0.028522) < 2e-6
    assert abs(y[names.index("O2")] - 0.226354) < 2e-6
    assert abs(y[names.index("N2")] - 0.745124) < 2e-6


def test_workload_table():
    assert WORKLOADS["rde1m"]["width"] * WORKLOADS["rde1m"]["height"] == 1048576
    sizes = states.amr_field_sizes(WORKLOADS["amr64"]["seed"])
    assert len(sizes) == 64 and min(sizes) >= 10000 and max(sizes) <= 2000000


@pytest.mark.parametrize("name,base,nsri,nlind,nplog,nirrev", [("m13x", "m13", 1, 1, 4, 6),
                                                               ("m32x", "m32", 5, 3, 12, 30),
                                                               ("m32s", "m32", 5, 3, 0, 30)])
def test_variant_mechanisms_use_every_form(name, base, nsri, nlind, nplog, nirrev):
    rx = [l.split() for l in mech_text(name).splitlines() if l.startswith("reaction")]
    rb = [l.split() for l in mech_text(base).splitlines() if l.startswith("reaction")]
    assert len(rx) == len(rb)
    kinds = [l[1] for l in rx]
    assert kinds.count("sri") == nsri and kinds.count("lindemann") == nlind
    assert kinds.count("plog") == nplog and sum(l[-1] == "irrev" for l in rx) == nirrev
    for l, b in zip(rx, rb):
        assert l[2:4] == b[2:4]                 # same species and coefficients
        if l[1] == "plog":
            ps = [float(e.split(":")[0]) for e in next(t for t in l if t.startswith("plog="))[5:].split(",")]
            assert ps == sorted(ps) and len(set(ps)) == len(ps)
