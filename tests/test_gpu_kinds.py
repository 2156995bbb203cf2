"""GPU parity for every reaction form: irreversible reactions, Lindemann, Troe
and SRI falloff, and pressure-tabulated (PLOG) rates, in both kernel families.
m13x (13 species, lane form and forced into the wave-cooperative form) and
m32x (32 species, wave-cooperative) are m13 and m32 with those forms mixed in;
their PLOG tables put the cells' pressures below, inside and above the
tabulated range.  Bars as in the other parity tests: source terms to 1e-11 of
the row scale, Jacobians to 1e-10 (plus the oracle's own analytic-vs-complex-
step gap near equilibrium), |dT| <= 1e-6 T and |dY_k| <= 1e-8 for integrated
states at rtol 1e-8, atol 1e-12, persistent and plain forms bitwise, adjoint
gradients to 1e-5 relative."""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from workloads import mech_path, mech_text  # noqa: E402
from workloads.states import parse_species, uniform_cells  # noqa: E402

RTOL, ATOL = 1e-8, 1e-12
PATM = 101325.0


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch.device("cuda:0")


@pytest.fixture(scope="module")
def chem():
    import paper_2508_16105_amd as chem
    return chem


def _load_wide(chem, name):
    old = os.environ.get("CHEM_LANE_MAX_SPECIES")
    os.environ["CHEM_LANE_MAX_SPECIES"] = "0"
    try:
        return chem.Mechanism(mech_path(name))
    finally:
        if old is None:
            del os.environ["CHEM_LANE_MAX_SPECIES"]
        else:
            os.environ["CHEM_LANE_MAX_SPECIES"] = old


@pytest.fixture(scope="module")
def mechs(chem, oracle_lib):
    return {"m13x": (chem.Mechanism(mech_path("m13x")), oracle_lib.Mechanism(mech_path("m13x"))),
            "m13xw": (_load_wide(chem, "m13x"), oracle_lib.Mechanism(mech_path("m13x"))),
            "m32x": (chem.Mechanism(mech_path("m32x")), oracle_lib.Mechanism(mech_path("m32x")))}


def _g(a, dev):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)


def _cells(name, n, seed, wide_p=False):
    T, p, Y = uniform_cells(mech_text(name), n, seed)
    if wide_p:   # 0.005 - 2000 atm: below, inside and above every PLOG table
        p = PATM * np.exp(np.random.default_rng(seed + 1).uniform(np.log(0.005), np.log(2000.0), n))
    return T, p, Y


@pytest.mark.parametrize("key", ["m13x", "m13xw", "m32x"])
@pytest.mark.parametrize("wide_p", [False, True])
def test_source_terms_and_jacobian(chem, mechs, dev, key, wide_p):
    gm, om = mechs[key]
    name = key.rstrip("w")
    T, p, Y = _cells(name, 96, 81, wide_p)
    f, J = chem.eval_source(gm, _g(T, dev), _g(p, dev), _g(Y, dev))
    f, J = f.cpu().numpy(), J.cpu().numpy()
    for i in range(len(T)):
        y = np.concatenate([[T[i]], Y[i]])
        fo = om.rhs(p[i], y)
        assert np.all(np.abs(f[i] - fo) <= 1e-11 * np.abs(fo).max() + 1e-300), (key, i, p[i])
        Jo = om.jac_cs(p[i], y)
        Ja = om.jac(p[i], y)
        sc = np.abs(Jo).max(axis=1, keepdims=True) * np.maximum(np.abs(y), 1e-3)[None, :] \
            / np.maximum(np.abs(y), 1e-3).max()
        tol = 1e-10 * (np.abs(Jo) + sc) + 4.0 * np.abs(Ja - Jo)
        off = np.argwhere(~(np.abs(J[i] - Jo) <= tol))
        assert len(off) == 0, (key, i, p[i], [(int(r), int(c), J[i][r, c], Jo[r, c]) for r, c in off[:6]])


def _assert_state_parity(Tg, Yg, To, Yo, what):
    dT = np.abs(Tg - To)
    dY = np.abs(Yg - Yo)
    bad = (dT > 1e-6 * To) | np.any(dY > 1e-8, axis=1)
    assert not bad.any(), (f"{what}: {bad.sum()} cells out of tolerance; max |dT|/T "
                           f"{(dT / To).max():.3e}, max |dY| {dY.max():.3e}")


# dt: m32's reactions are slower; 1e-5 s gives its cells 10 substeps on median, 124 at most
DT = {"m13x": 1e-8, "m13xw": 1e-8, "m32x": 1e-5}


@pytest.mark.parametrize("key,n", [("m13x", 1031), ("m13xw", 515), ("m32x", 259)])
def test_integrate_matches_oracle(chem, mechs, dev, key, n):
    gm, om = mechs[key]
    T, p, Y = _cells(key.rstrip("w"), n, 82, wide_p=True)
    Tg, Yg, stats = chem.integrate(gm, _g(T, dev), _g(p, dev), _g(Y, dev), DT[key], RTOL, ATOL)
    To, Yo, _, _, sto = om.integrate(T, p, Y, DT[key], RTOL, ATOL)
    assert stats["failed"] == 0 and np.all(sto == 0)
    _assert_state_parity(Tg.cpu().numpy(), Yg.cpu().numpy(), To, Yo, key)


@pytest.mark.parametrize("key", ["m13x", "m32x"])
def test_persistent_is_bitwise_equal_to_plain(chem, mechs, dev, key):
    gm, _ = mechs[key]
    T, p, Y = _cells(key, 700, 83, wide_p=True)
    a = chem.integrate(gm, _g(T, dev), _g(p, dev), _g(Y, dev), DT[key], RTOL, ATOL, return_counts=True)
    b = chem.integrate(gm, _g(T, dev), _g(p, dev), _g(Y, dev), DT[key], RTOL, ATOL, form=chem.FORM_PERSISTENT,
                       return_counts=True)
    for x, y in ((a[0], b[0]), (a[1], b[1]), (a[4], b[4]), (a[5], b[5])):
        assert torch.equal(x, y)


def _oracle_adjoint(om, T, p, Y, dt, gT, gY):
    ref = om.adjoint(T, p, Y, dt, RTOL, ATOL, gT, gY)
    spread = [np.zeros(len(T)), np.zeros(len(T)), 0.0, 0.0, 0.0]
    for f in (1.0 + 2.0**-52, 1.0 - 2.0**-52):
        alt = om.adjoint(T * f, p, Y, dt, RTOL, ATOL, gT, gY)
        spread[0] = np.maximum(spread[0], np.abs(alt[0] - ref[0]))
        spread[1] = np.maximum(spread[1], np.max(np.abs(alt[1] - ref[1]), axis=1))
        for i in (2, 3, 4):
            spread[i] = max(spread[i], np.max(np.abs(alt[i] - ref[i])))
    return ref, spread


@pytest.mark.parametrize("key", ["m13x", "m13xw"])
def test_adjoint_matches_oracle(chem, mechs, dev, key):
    """Gradients with respect to the initial state and to every reaction's
    (ln A, b, Ea), including the PLOG reactions' main-rate factor and the
    irreversible reactions, against the oracle's complex-step adjoint."""
    gm, om = mechs[key]
    T, p, Y = _cells("m13x", 40, 84, wide_p=True)
    species = parse_species(mech_text("m13x"))[0]
    gT = np.full(len(T), 1.0 / 1000.0)
    gY = np.random.default_rng(85).standard_normal((len(T), len(species)))
    out = chem.integrate_adjoint(gm, _g(T, dev), _g(p, dev), _g(Y, dev), 1e-8, RTOL, ATOL, _g(gT, dev), _g(gY, dev))
    gT0, gY0, ga, gb, ge = [x.cpu().numpy() for x in out[:5]]
    assert out[7]["failed"] == 0
    (oT0, oY0, oa, ob, oe), spread = _oracle_adjoint(om, T, p, Y, 1e-8, gT, gY)
    assert np.all(np.abs(gT0 - oT0) <= np.maximum(1e-5 * np.abs(oT0), 4 * spread[0]))
    sc = np.max(np.abs(oY0), axis=1)
    assert np.all(np.max(np.abs(gY0 - oY0), axis=1) <= np.maximum(1e-5 * sc, 4 * spread[1]))
    for i, g, o in ((2, ga, oa), (3, gb, ob), (4, ge, oe)):
        assert np.max(np.abs(g - o)) <= max(1e-5 * np.max(np.abs(o)), 4 * spread[i]), i


# ---------------- mechanisms read from CHEMKIN files and OpenFOAM dictionaries ----------------

@pytest.fixture(scope="module")
def ck(chem, oracle_lib, tmp_path_factory):
    """The hand-written CHEMKIN and OpenFOAM fixtures (9 species, every
    reaction form each format has, lane form), m32x written as CHEMKIN with
    its thermo in a separate file and m32s as OpenFOAM dictionaries
    (wave-cooperative form), each with the oracle's reading of the same files
    and the `chemmi-mech 1` text of that reading."""
    import pathlib
    from oracle import chemkin
    from workloads import gen_mech
    fixture = pathlib.Path(__file__).resolve().parent / "golden" / "ck_small.inp"
    d = tmp_path_factory.mktemp("ck")
    m = gen_mech.build_mechanism("m32x")
    bare, thermo = d / "m32x.inp", d / "therm.dat"
    bare.write_text(gen_mech.to_chemkin(m, inline_thermo=False))
    thermo.write_text(gen_mech.thermo_chemkin(m))
    from oracle import foam
    fx = pathlib.Path(__file__).resolve().parent / "golden" / "foam_small"
    fr, ft = fx / "reactions", fx / "thermo"
    sr, st = d / "m32s.foam", d / "thermo"
    r, t = gen_mech.to_openfoam(gen_mech.build_mechanism("m32s"))
    sr.write_text(r)
    st.write_text(t)
    return {"ck_small": (chem.Mechanism(fixture), oracle_lib.chemkin_mechanism(fixture),
                         chemkin.convert(fixture.read_text())),
            "m32x_ck": (chem.Mechanism(bare, thermo=thermo), oracle_lib.chemkin_mechanism(bare, thermo),
                        chemkin.convert(bare.read_text(), thermo.read_text())),
            "foam_small": (chem.Mechanism(fr, thermo=ft, fmt="openfoam"), oracle_lib.openfoam_mechanism(fr, ft),
                           foam.convert(fr.read_text(), ft.read_text())),
            "m32s_foam": (chem.Mechanism(sr, thermo=st, fmt="openfoam"), oracle_lib.openfoam_mechanism(sr, st),
                          foam.convert(sr.read_text(), st.read_text()))}


@pytest.mark.parametrize("key,n,dt", [("ck_small", 777, 1e-7), ("m32x_ck", 130, 1e-5), ("foam_small", 777, 1e-7),
                                      ("m32s_foam", 130, 1e-5)])
def test_chemkin_mechanisms_match_oracle(chem, ck, dev, key, n, dt):
    gm, om, text = ck[key]
    T, p, Y = uniform_cells(text, n, 86)
    p = PATM * np.exp(np.random.default_rng(87).uniform(np.log(0.005), np.log(2000.0), n))
    f, J = chem.eval_source(gm, _g(T, dev), _g(p, dev), _g(Y, dev))
    f, J = f.cpu().numpy(), J.cpu().numpy()
    for i in range(0, n, 7):
        y = np.concatenate([[T[i]], Y[i]])
        fo = om.rhs(p[i], y)
        assert np.all(np.abs(f[i] - fo) <= 1e-11 * np.abs(fo).max() + 1e-300), (key, i)
        Jo, Ja = om.jac_cs(p[i], y), om.jac(p[i], y)
        sc = np.abs(Jo).max(axis=1, keepdims=True) * np.maximum(np.abs(y), 1e-3)[None, :] \
            / np.maximum(np.abs(y), 1e-3).max()
        assert np.all(np.abs(J[i] - Jo) <= 1e-10 * (np.abs(Jo) + sc) + 4.0 * np.abs(Ja - Jo)), (key, i)
    Tg, Yg, stats = chem.integrate(gm, _g(T, dev), _g(p, dev), _g(Y, dev), dt, RTOL, ATOL)
    To, Yo, _, _, sto = om.integrate(T, p, Y, dt, RTOL, ATOL)
    assert stats["failed"] == 0 and np.all(sto == 0)
    _assert_state_parity(Tg.cpu().numpy(), Yg.cpu().numpy(), To, Yo, key)


@pytest.mark.parametrize("key,form", [("m13x", "persistent"), ("m32x", "plain")])
def test_source_mode_with_every_form(chem, mechs, dev, key, form):
    """chem_integrate_source on mechanisms with SRI, PLOG and irreversible
    reactions: the end state equals chem_integrate's and the rates agree with
    the oracle's end state to the parity bar carried through the formulas."""
    gm, om = mechs[key]
    f = chem.FORM_PERSISTENT if form == "persistent" else chem.FORM_PLAIN
    T, p, Y = _cells(key, 300, 88, wide_p=True)
    Tg, Yg, wg, qg, stats = chem.integrate_source(gm, _g(T, dev), _g(p, dev), _g(Y, dev), DT[key], RTOL, ATOL,
                                                   form=f)
    Ti, Yi, _ = chem.integrate(gm, _g(T, dev), _g(p, dev), _g(Y, dev), DT[key], RTOL, ATOL, form=f)
    assert torch.equal(Tg, Ti) and torch.equal(Yg, Yi) and stats["failed"] == 0
    To, Yo, _, _, sto = om.integrate(T, p, Y, DT[key], RTOL, ATOL)
    assert np.all(sto == 0)
    W = om.weights()
    rho0 = p / (8.314462618 * T * (Y / W).sum(axis=1))
    wo = rho0[:, None] * (Yo - Y) / DT[key]
    _, hrt, _ = om.thermo(298.15)
    hf = 8.314462618 * 298.15 * hrt / W
    qo = -(wo @ hf)
    bar = rho0 * 1e-8 / DT[key]
    assert np.all(np.abs(wg.cpu().numpy() - wo) <= 1.01 * bar[:, None])
    assert np.all(np.abs(qg.cpu().numpy() - qo) <= 1.01 * bar * np.abs(hf).sum())


def test_batched_fields_with_every_form(chem, mechs, dev):
    """Three m13x fields of different sizes in one persistent launch equal
    their per-field plain integrations bitwise."""
    gm, _ = mechs["m13x"]
    fields = [_cells("m13x", n, 89 + n, wide_p=True) for n in (1, 130, 517)]
    Ts = [_g(T, dev) for T, _, _ in fields]
    ps = [_g(p, dev) for _, p, _ in fields]
    Ys = [_g(Y, dev) for _, _, Y in fields]
    stats = chem.integrate_batched(gm, Ts, ps, Ys, DT["m13x"], RTOL, ATOL)
    assert stats["failed"] == 0 and stats["cells"] == 648
    for (T, p, Y), Tb, Yb in zip(fields, Ts, Ys):
        Tp, Yp, _ = chem.integrate(gm, _g(T, dev), _g(p, dev), _g(Y, dev), DT["m13x"], RTOL, ATOL)
        assert torch.equal(Tp, Tb) and torch.equal(Yp, Yb)


@pytest.mark.parametrize("key,side", [("m13x", 512), ("m32x", 256)])
def test_rde_field_with_every_form_sampled(chem, mechs, dev, key, side):
    """A whole RDE-shaped field (fresh, front and burnt regions; 1-30 atm, so
    inside the PLOG tables) in the persistent form at dt = 5 ns, with 32 cells
    of every region against the oracle."""
    from workloads.states import rde_field
    gm, om = mechs[key]
    T, p, Y, reg = rde_field(mech_text(key), side, side, 107)
    Tg, Yg, stats = chem.integrate(gm, _g(T, dev), _g(p, dev), _g(Y, dev), 5e-9, RTOL, ATOL,
                                   form=chem.FORM_PERSISTENT)
    assert stats["failed"] == 0 and stats["cells"] == side * side
    rng = np.random.default_rng(108)
    idx = np.concatenate([rng.choice(np.nonzero(reg == r)[0], 32, replace=False) for r in (0, 1, 2)])
    To, Yo, _, _, sto = om.integrate(T[idx], p[idx], Y[idx], 5e-9, RTOL, ATOL)
    assert np.all(sto == 0)
    _assert_state_parity(Tg.cpu().numpy()[idx], Yg.cpu().numpy()[idx], To, Yo, key)
