"""GPU parity of the wave-cooperative form (G lanes per cell) against the
CPU oracle: the 32-species / 150-reaction mechanism (third-body + Troe on 15
reactions; n = 33, one cell per wave), and the 9- and 13-species mechanisms
forced into the same form (n = 10 and 14, four cells per 16-lane groups of a
wave) so both group sizes and the padding lanes are exercised.

Tolerances are those of the one-cell-per-lane parity tests: |dT| <= 1e-6 T and
|dY_k| <= 1e-8 at rtol 1e-8, atol 1e-12 for integrated states; source terms
to 1e-11 and the Jacobian to 1e-10 of the row scale; persistent and plain
forms bitwise."""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from workloads import WORKLOADS, mech_path, mech_text  # noqa: E402
from workloads.states import rde_field, rde_field_n, uniform_cells  # noqa: E402

from errnorm_ref import errnorm_bar, errnorm_with_spread  # noqa: E402

RTOL, ATOL = 1e-8, 1e-12


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch.device("cuda:0")


@pytest.fixture(scope="module")
def chem():
    import paper_2508_16105_amd as chem
    return chem


def _load_wide(chem, name):
    """Load `name` in the wave-cooperative form (the lane form's species limit
    lowered to 0 for this load only)."""
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
    out = {"m32": (chem.Mechanism(mech_path("m32")), oracle_lib.Mechanism(mech_path("m32")))}
    for name in ("m9", "m13"):
        out[name + "w"] = (_load_wide(chem, name), oracle_lib.Mechanism(mech_path(name)))
    return out


def _g(a, dev):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)


def _assert_state_parity(Tg, Yg, To, Yo, what):
    dT = np.abs(Tg - To)
    dY = np.abs(Yg - Yo)
    bad = (dT > 1e-6 * To) | np.any(dY > 1e-8, axis=1)
    assert not bad.any(), (f"{what}: {bad.sum()} cells out of tolerance; max |dT|/T "
                           f"{(dT / To).max():.3e}, max |dY| {dY.max():.3e}")


@pytest.mark.parametrize("key", ["m32", "m9w", "m13w"])
def test_wide_source_terms_and_jacobian(chem, mechs, dev, key):
    gm, om = mechs[key]
    name = key.rstrip("w")
    T, p, Y = uniform_cells(mech_text(name), 100, 71)
    f, J = chem.eval_source(gm, _g(T, dev), _g(p, dev), _g(Y, dev))
    f2, _ = chem.eval_source(gm, _g(T, dev), _g(p, dev), _g(Y, dev), jacobian=False)
    assert torch.equal(f, f2)
    f, J = f.cpu().numpy(), J.cpu().numpy()
    for i in range(len(T)):
        y = np.concatenate([[T[i]], Y[i]])
        fo = om.rhs(p[i], y)
        Jo = om.jac_cs(p[i], y)
        assert np.all(np.abs(f[i] - fo) <= 1e-11 * np.abs(fo).max() + 1e-300), (key, i)
        sc = np.abs(Jo).max(axis=1, keepdims=True) * np.maximum(np.abs(y), 1e-3)[None, :] \
            / np.maximum(np.abs(y), 1e-3).max()
        # Entries near equilibrium are small differences of large forward and
        # reverse terms; an analytic Jacobian carries an absolute error set by
        # those terms, which complex step does not.  The oracle's own analytic
        # Jacobian measures that conditioning, so its gap to complex step
        # (4x) is allowed on top of the relative bound.
        Ja = om.jac(p[i], y)
        tol = 1e-10 * (np.abs(Jo) + sc) + 4.0 * np.abs(Ja - Jo)
        off = np.argwhere(~(np.abs(J[i] - Jo) <= tol))
        assert len(off) == 0, (key, i, [(int(r), int(c), J[i][r, c], Jo[r, c], tol[r, c]) for r, c in off[:6]])


@pytest.mark.parametrize("key", ["m32", "m9w", "m13w"])
def test_wide_integrate_uniform_matches_oracle(chem, mechs, dev, key):
    gm, om = mechs[key]
    name = key.rstrip("w")
    n = 515                                              # not a multiple of the cells per wave
    T, p, Y = uniform_cells(mech_text(name), n, 72)
    Tg, Yg, stats, st, na, nr = chem.integrate(gm, _g(T, dev), _g(p, dev), _g(Y, dev), 1e-8, RTOL, ATOL,
                                               return_counts=True)
    To, Yo, nao, nro, sto = om.integrate(T, p, Y, 1e-8, RTOL, ATOL)
    assert stats["failed"] == 0 and np.all(sto == 0) and stats["cells"] == n
    _assert_state_parity(Tg.cpu().numpy(), Yg.cpu().numpy(), To, Yo, key)
    differ = np.sum((na.cpu().numpy() != nao) | (nr.cpu().numpy() != nro))
    assert differ <= max(2, 0.01 * n), f"{differ} cells took a different step sequence"


def test_wide_big4m_field_sample(chem, mechs, dev):
    """The 2048 x 2048 RDE-shaped field with the 32-species mechanism at full
    size: sampled cells of every region against the oracle, and properties
    that hold for every cell; plain and persistent forms bitwise equal."""
    w = WORKLOADS["big4m"]
    gm, om = mechs["m32"]
    T, p, Y, reg = rde_field(mech_text("m32"), w["width"], w["height"], w["seed"])
    rng = np.random.default_rng(3)
    idx = np.concatenate([rng.choice(np.where(reg == r)[0], 200, replace=False) for r in (0, 1, 2)])
    To, Yo, _, _, _ = om.integrate(T[idx], p[idx], Y[idx], w["dt"], w["rtol"], w["atol"])
    out = {}
    for form in (chem.FORM_PLAIN, chem.FORM_PERSISTENT):
        Tg, Yg, stats, st, na, nr = chem.integrate(gm, _g(T, dev), _g(p, dev), _g(Y, dev), w["dt"], w["rtol"],
                                                   w["atol"], form=form, return_counts=True)
        assert stats["failed"] == 0 and stats["cells"] == len(T)
        Tn, Yn = Tg.cpu().numpy(), Yg.cpu().numpy()
        _assert_state_parity(Tn[idx], Yn[idx], To, Yo, f"big4m form {form}")
        nsub = (na + nr).cpu().numpy()
        assert np.all(np.abs(Yn.sum(1) - 1.0) <= 1e-13 * np.maximum(nsub, 1) + 1e-14)
        out[form] = (Tg, Yg, na, nr)
    for a, b in zip(out[chem.FORM_PLAIN], out[chem.FORM_PERSISTENT]):
        assert torch.equal(a, b)


def test_wide_batched_fields(chem, mechs, dev):
    """Several fields of different sizes (ragged, tiny, empty) in one
    persistent launch equal per-field plain launches bitwise."""
    gm, om = mechs["m32"]
    sizes = [700, 1, 0, 3001, 64, 17]
    fields = [rde_field_n(mech_text("m32"), n, 900 + i)[:3] for i, n in enumerate(sizes)]
    Ts = [_g(f[0], dev) for f in fields]
    ps = [_g(f[1], dev) for f in fields]
    Ys = [_g(f[2].reshape(-1, gm.ns), dev) for f in fields]
    stats = chem.integrate_batched(gm, Ts, ps, Ys, 5e-9, RTOL, ATOL)
    assert stats["cells"] == sum(sizes) and stats["failed"] == 0
    for (T, p, Y), Tb, Yb in zip(fields, Ts, Ys):
        if len(T) == 0:
            continue
        Tr, Yr, _ = chem.integrate(gm, _g(T, dev), _g(p, dev), _g(Y, dev), 5e-9, RTOL, ATOL)
        assert torch.equal(Tr, Tb) and torch.equal(Yr, Yb)
        To, Yo, _, _, _ = om.integrate(T, p, Y, 5e-9, RTOL, ATOL)
        _assert_state_parity(Tb.cpu().numpy(), Yb.cpu().numpy(), To, Yo, "batched m32")


def test_wide_bad_cells_and_limits(chem, mechs, dev):
    gm, om = mechs["m13w"]
    T, p, Y = uniform_cells(mech_text("m13"), 9, 73)
    T[2] = -10.0
    Y[3, 4] = np.nan
    p[5] = 0.0
    Tg, Yg, stats, st, na, nr = chem.integrate(gm, _g(T, dev), _g(p, dev), _g(Y, dev), 1e-8, RTOL, ATOL,
                                               return_counts=True, allow_failed=True)
    st = st.cpu().numpy()
    assert list(np.where(st == 4)[0]) == [2, 3, 5] and stats["failed"] == 3
    assert Tg[2].item() == -10.0 and np.isnan(Yg[3, 4].item())
    ok = [i for i in range(9) if i not in (2, 3, 5)]
    To, Yo, _, _, _ = om.integrate(T[ok], p[ok], Y[ok], 1e-8, RTOL, ATOL)
    _assert_state_parity(Tg.cpu().numpy()[ok], Yg.cpu().numpy()[ok], To, Yo, "good cells")
    # max_substeps = 1 as in the oracle
    T2, p2, Y2 = uniform_cells(mech_text("m13"), 64, 74)
    _, _, _, st2, na2, nr2 = chem.integrate(gm, _g(T2, dev), _g(p2, dev), _g(Y2, dev), 1e-8, RTOL, ATOL,
                                            max_substeps=1, return_counts=True, allow_failed=True)
    _, _, _, _, sto = om.integrate(T2, p2, Y2, 1e-8, RTOL, ATOL, max_substeps=1)
    assert np.array_equal(st2.cpu().numpy(), sto)


@pytest.mark.parametrize("key", ["m32", "m9w", "m13w"])
def test_wide_fixed_step_matches_oracle(chem, mechs, dev, key):
    """chem_step_fixed in the wave-cooperative form: one RODAS4 step of given
    size per cell, the new state to the lane form's bars (T to 1e-10
    relative, Y to 1e-12)."""
    gm, om = mechs[key]
    name = key.rstrip("w")
    T, p, Y = uniform_cells(mech_text(name), 67, 75)
    # m13's hot cells are stiffer: at h = 1e-9 a third of its step matrices
    # are too ill-conditioned for the comparison, so it takes smaller steps
    for h in ((1e-12, 1e-11) if name == "m13" else (1e-11, 1e-9)):
        yn, en, ok = chem.step_fixed(gm, _g(T, dev), _g(p, dev), _g(Y, dev), h, RTOL, ATOL)
        yn, ok, en = yn.cpu().numpy(), ok.cpu().numpy(), en.cpu().numpy()
        skipped = 0
        for i in range(len(T)):
            yo, eo = om.step(p[i], np.concatenate([[T[i]], Y[i]]), h)
            # a step whose stages leave the finite range (one m13 cell at
            # h = 1e-11) is reported as not ok, as the oracle's result is not finite
            finite = bool(np.all(np.isfinite(yo)) and np.all(np.isfinite(eo)))
            assert bool(ok[i]) == finite, (key, i, h)
            if not finite:
                continue
            # a cell whose step matrix is ill-conditioned (cond up to 1e19 on
            # 3000 K m13 cells) gives a step result that a 1-ulp change of T
            # moves by more than the bar (by up to 1e4 K for a step far too
            # large for it, which the controller would reject); two correct
            # results differ by as much, so such cells are not compared
            y0 = np.concatenate([[T[i]], Y[i]])
            spread = np.zeros(len(y0))
            for f in (1.0 + 2.0**-52, 1.0 - 2.0**-52):
                y1 = y0.copy()
                y1[0] *= f
                spread = np.maximum(spread, np.abs(om.step(p[i], y1, h)[0] - yo))
            if spread[0] > 2.5e-11 * yo[0] or np.any(spread[1:] > 2.5e-13):
                skipped += 1
                continue
            assert abs(yn[i, 0] - yo[0]) <= 1e-10 * yo[0], (key, i)
            assert np.all(np.abs(yn[i, 1:] - yo[1:]) <= 1e-12), (key, i)
            # the embedded error estimate that decides acceptance
            eno, espread, _, _ = errnorm_with_spread(om, p[i], y0, h, RTOL, ATOL)
            assert abs(en[i] - eno) <= errnorm_bar(eno, espread), (key, i, h, en[i], eno, espread)
        assert skipped <= len(T) // 5, (key, h, skipped)


def test_wide_source_mode(chem, mechs, dev):
    """chem_integrate_source in the wave-cooperative form (32 species): the
    same end state as chem_integrate, and rates formed from it to round-off."""
    gm, om = mechs["m32"]
    T, p, Y, _ = rde_field_n(mech_text("m32"), 3000, 930)
    Tg, Yg, wg, qg, stats = chem.integrate_source(gm, _g(T, dev), _g(p, dev), _g(Y, dev), 5e-9, RTOL, ATOL,
                                                  form=chem.FORM_PERSISTENT)
    Ti, Yi, _ = chem.integrate(gm, _g(T, dev), _g(p, dev), _g(Y, dev), 5e-9, RTOL, ATOL,
                               form=chem.FORM_PERSISTENT)
    assert torch.equal(Tg, Ti) and torch.equal(Yg, Yi) and stats["failed"] == 0
    W = om.weights()
    rho0 = p / (8.314462618 * T * (Y / W).sum(axis=1))
    ws = rho0[:, None] * (Yg.cpu().numpy() - Y) / 5e-9
    _, hrt, _ = om.thermo(298.15)
    hf = 8.314462618 * 298.15 * hrt / W
    wg, qg = wg.cpu().numpy(), qg.cpu().numpy()
    assert np.all(np.abs(wg - ws) <= 1e-12 * np.abs(ws) + 1e-300)
    assert np.all(np.abs(qg + (ws * hf).sum(axis=1)) <= 1e-12 * np.abs(ws * hf).sum(axis=1) + 1e-300)


def test_mid_size_mechanism_runs_wave_cooperatively_at_parity(chem, oracle_lib, dev):
    """A 16-species mechanism (above the one-cell-per-lane limit) loads in the
    wave-cooperative form by default (G = 32: two cells per wave) and matches
    the oracle on uniform cells and on every region of an RDE-shaped field,
    plain and persistent."""
    import ctypes as C
    gm = chem.Mechanism(mech_path("m16"))
    om = oracle_lib.Mechanism(mech_path("m16"))
    T, p, Y = uniform_cells(mech_text("m16"), 301, 76)
    Tg, Yg, stats = chem.integrate(gm, _g(T, dev), _g(p, dev), _g(Y, dev), 1e-8, RTOL, ATOL)
    To, Yo, _, _, sto = om.integrate(T, p, Y, 1e-8, RTOL, ATOL)
    assert stats["failed"] == 0 and np.all(sto == 0)
    _assert_state_parity(Tg.cpu().numpy(), Yg.cpu().numpy(), To, Yo, "m16 uniform")
    T, p, Y, reg = rde_field(mech_text("m16"), 128, 128, 77)
    Tp, Yp, sp = chem.integrate(gm, _g(T, dev), _g(p, dev), _g(Y, dev), 5e-9, RTOL, ATOL, form=chem.FORM_PERSISTENT)
    Tq, Yq, sq = chem.integrate(gm, _g(T, dev), _g(p, dev), _g(Y, dev), 5e-9, RTOL, ATOL)
    assert torch.equal(Tp, Tq) and torch.equal(Yp, Yq) and sp["failed"] == 0
    rng = np.random.default_rng(78)
    idx = np.concatenate([rng.choice(np.nonzero(reg == r)[0], 16, replace=False) for r in (0, 1, 2)])
    To, Yo, _, _, sto = om.integrate(T[idx], p[idx], Y[idx], 5e-9, RTOL, ATOL)
    assert np.all(sto == 0)
    _assert_state_parity(Tp.cpu().numpy()[idx], Yp.cpu().numpy()[idx], To, Yo, "m16 field")
