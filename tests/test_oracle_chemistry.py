"""Pins of the oracle's chemistry (thermo, rates, source terms, Jacobian)
against mathematics and physics that do not depend on its code."""
import math

import numpy as np
import pytest

from workloads import mech_path, mech_text, tiny
from workloads.states import uniform_cells

RU = 8.314462618
PATM = 101325.0


def _y(T, Y):
    return np.concatenate([[T], Y])


@pytest.fixture(scope="module")
def m9(oracle_lib):
    return oracle_lib.Mechanism(mech_path("m9"))


@pytest.fixture(scope="module")
def m13(oracle_lib):
    return oracle_lib.Mechanism(mech_path("m13"))


# ---------------- thermo ----------------

@pytest.mark.parametrize("T", [350.0, 800.0, 1500.0, 2900.0])
def test_thermo_derivative_identities(m9, T):
    """dH/dT = cp and dS/dT = cp/T (H = HRT*R*T molar), by Richardson FD."""
    def H(t):
        return m9.thermo(t)[1] * t

    def Sr(t):
        return m9.thermo(t)[2]
    cp = m9.thermo(T)[0]
    for d in (1e-2,):
        dH = (8 * (H(T + d) - H(T - d)) - (H(T + 2 * d) - H(T - 2 * d))) / (12 * d)
        dS = (8 * (Sr(T + d) - Sr(T - d)) - (Sr(T + 2 * d) - Sr(T - 2 * d))) / (12 * d)
        assert np.allclose(dH, cp, rtol=1e-9)
        assert np.allclose(dS, cp / T, rtol=1e-9)


def test_thermo_continuous_at_tmid(m9):
    lo = m9.thermo(1000.0 - 1e-9)
    hi = m9.thermo(1000.0)
    for a, b in zip(lo, hi):
        assert np.allclose(a, b, rtol=1e-10, atol=1e-10)


def test_thermo_constant_cp_closed_form(oracle_lib, write_mech):
    """Only a1, a6, a7 non-zero: cp/R = a1, H/RT = a1 + a6/T, S/R = a1 ln T + a7."""
    m = oracle_lib.Mechanism(write_mech(tiny.dissociation()))
    T = 1234.5
    cp, h, s = m.thermo(T)
    # species order H2, H, N2 with (a1, a6, a7) from tiny.dissociation
    for k, (a1, a6, a7) in enumerate([(3.5, -1043.5, -3.0), (2.5, 25000.0, -1.0),
                                      (3.5, -1043.5, 4.0)]):
        assert cp[k] == pytest.approx(a1, rel=1e-15)
        assert h[k] == pytest.approx(a1 + a6 / T, rel=1e-14)
        assert s[k] == pytest.approx(a1 * math.log(T) + a7, rel=1e-14)


# ---------------- rate constants ----------------

def test_kf_reduces_to_A_in_si(oracle_lib, write_mech):
    """b = Ea = 0: k_f = A, converted from cm^3/mol to m^3/mol per order."""
    m = oracle_lib.Mechanism(write_mech(tiny.falloff(kind="elementary", A=3.0e12)))
    y = _y(1500.0, [0.2, 0.2, 0.1, 0.5])
    kf, kr, q = m.rates(PATM, y)
    assert kf[0] == pytest.approx(3.0e12 * 1e-6, rel=1e-14)       # second order
    m1 = oracle_lib.Mechanism(write_mech(tiny.isomer_pair(A=7.0e5), "iso.mech"))
    kf1, _, _ = m1.rates(PATM, _y(900.0, [0.3, 0.2, 0.5]))
    assert kf1[0] == pytest.approx(7.0e5, rel=1e-14)               # first order


def test_kf_arrhenius_temperature_dependence(oracle_lib, write_mech):
    """k(T2)/k(T1) = (T2/T1)^b exp(-Ea/R (1/T2 - 1/T1))."""
    m = oracle_lib.Mechanism(write_mech(tiny.isomer_pair(A=1e9, b=1.3, Ea=80.0)))
    k1 = m.rates(PATM, _y(800.0, [0.3, 0.2, 0.5]))[0][0]
    k2 = m.rates(PATM, _y(2100.0, [0.3, 0.2, 0.5]))[0][0]
    expect = (2100.0 / 800.0) ** 1.3 * math.exp(-80e3 / RU * (1 / 2100.0 - 1 / 800.0))
    assert k2 / k1 == pytest.approx(expect, rel=1e-12)


def test_isomer_kc_from_entropy(oracle_lib, write_mech):
    """dH = 0, dnu = 0: K_c = exp(dS/R), so k_r = k_f exp(-dS/R)."""
    m = oracle_lib.Mechanism(write_mech(tiny.isomer_pair(A=5e5, dS_R=1.7)))
    kf, kr, _ = m.rates(PATM, _y(1100.0, [0.3, 0.2, 0.5]))
    assert kr[0] / kf[0] == pytest.approx(math.exp(-1.7), rel=1e-13)


@pytest.mark.parametrize("T", [600.0, 1400.0, 2500.0])
def test_van_t_hoff(m13, T):
    """d ln K_c / dT = (dH/RT - dnu) / T with dH from the oracle's thermo
    (K_c = k_f/k_r).  Pins sign and standard-state terms of K_c."""
    y = _y(T, np.full(13, 1.0 / 13))
    d = 0.5

    def lnkc(t):
        kf, kr, _ = m13.rates(PATM, _y(t, y[1:]))
        return np.log(kf) - np.log(kr)
    dlnkc = (8 * (lnkc(T + d) - lnkc(T - d)) - (lnkc(T + 2 * d) - lnkc(T - 2 * d))) / (12 * d)
    h = m13.thermo(T)[1]
    txt = [l.split() for l in mech_text("m13").splitlines() if l.startswith("reaction")]
    names = [l.split()[1] for l in mech_text("m13").splitlines() if l.startswith("species")]
    for j, l in enumerate(txt):
        dH, dnu = 0.0, 0
        for side, sg in ((l[2], -1), (l[3], 1)):
            for kv in side.split(","):
                s, nu = kv.split("=")
                dH += sg * int(nu) * h[names.index(s)]
                dnu += sg * int(nu)
        assert dlnkc[j] == pytest.approx((dH - dnu) / T, rel=1e-8, abs=1e-12)


# ---------------- third-body and falloff ----------------

def test_third_body_unit_efficiencies_is_total_concentration(oracle_lib, write_mech):
    """All efficiencies 1: [M] = sum C_k = p/(RT) (ideal gas), so
    q = p/(RT) * (k_f C_A C_B - k_r C_AB)."""
    me = oracle_lib.Mechanism(write_mech(tiny.falloff(kind="elementary"), "e.mech"))
    mt = oracle_lib.Mechanism(write_mech(tiny.falloff(kind="thirdbody", A=1.0e13 * 1e6),
                                         "t.mech"))
    p, y = 3 * PATM, _y(1800.0, [0.1, 0.2, 0.3, 0.4])
    qe = me.rates(p, y)[2][0]
    qt = mt.rates(p, y)[2][0]
    # the third-body A carries one more cm^3/mol factor, undone by the 1e6 above
    assert qt == pytest.approx(qe * p / (RU * 1800.0), rel=1e-13)


def test_falloff_limits(oracle_lib, write_mech):
    """Lindemann/Troe: P_r -> 0 gives k -> k0 [M], P_r -> inf gives k -> k_inf;
    F_cent = 1 reduces Troe to Lindemann."""
    A, A0 = 1.0e13, 1.0e16
    y = _y(1500.0, [0.1, 0.2, 0.3, 0.4])
    for kind in ("lindemann", "troe"):
        m = oracle_lib.Mechanism(write_mech(tiny.falloff(kind=kind, A=A, A0=A0), kind + ".mech"))
        lo = m.rates(1e-6 * PATM, y)[0][0]
        Mlo = 1e-6 * PATM / (RU * 1500.0)
        kinf = A * 1e-6
        k0 = A0 * 1e-12
        if kind == "lindemann":
            assert lo == pytest.approx(k0 * Mlo, rel=1e-6)
        hi = m.rates(1e9 * PATM, y)[0][0]
        assert hi == pytest.approx(kinf, rel=1e-4 if kind == "lindemann" else 2e-2)
    # Troe with alpha = 1, T1 -> inf and no T2: F_cent = 1
    mt = oracle_lib.Mechanism(write_mech(tiny.falloff(kind="troe", troe=(1.0, 100.0, 1e300, None)),
                                         "t1.mech"))
    ml = oracle_lib.Mechanism(write_mech(tiny.falloff(kind="lindemann"), "l1.mech"))
    for p in (0.01 * PATM, PATM, 100 * PATM):
        assert mt.rates(p, y)[0][0] == pytest.approx(ml.rates(p, y)[0][0], rel=1e-13)


def test_troe_center_value(oracle_lib, write_mech):
    """At log10 P_r = -c the Troe broadening equals F_cent exactly."""
    alpha, T3, T1 = 0.6, 300.0, 3000.0
    T = 1500.0
    m = oracle_lib.Mechanism(write_mech(tiny.falloff(kind="troe", troe=(alpha, T3, T1, None))))
    Fc = (1 - alpha) * math.exp(-T / T3) + alpha * math.exp(-T / T1)
    c = -0.4 - 0.67 * math.log10(Fc)
    Pr = 10.0 ** (-c)
    kinf, k0 = 1.0e13 * 1e-6, 1.0e16 * 1e-12
    M = Pr * kinf / k0
    p = M * RU * T
    k = m.rates(p, _y(T, [0.1, 0.2, 0.3, 0.4]))[0][0]
    assert k == pytest.approx(kinf * Pr / (1 + Pr) * Fc, rel=1e-12)


# ---------------- source terms ----------------

@pytest.mark.parametrize("mech", ["m9", "m13", "m32", "m13x", "m32x"])
def test_rhs_conserves_mass_elements_enthalpy(oracle_lib, mech):
    m = oracle_lib.Mechanism(mech_path(mech))
    T, p, Y = uniform_cells(mech_text(mech), 16, 7)
    names = [l.split()[1] for l in mech_text(mech).splitlines() if l.startswith("species")]
    comps = [dict((kv.split("=")[0], int(kv.split("=")[1])) for kv in l.split()[2].split(","))
             for l in mech_text(mech).splitlines() if l.startswith("species")]
    W = m.weights()
    elems = sorted({e for c in comps for e in c})
    for i in range(16):
        y = _y(T[i], Y[i])
        f = m.rhs(p[i], y)
        scale = np.abs(f[1:]).max()
        assert abs(f[1:].sum()) <= 1e-12 * scale                       # sum dY/dt = 0
        for e in elems:
            a = np.array([c.get(e, 0) for c in comps])
            assert abs((a / W) @ f[1:]) <= 1e-12 * (np.abs(a / W) @ np.abs(f[1:]) + 1e-300)
        cpR, hRT, _ = m.thermo(T[i])
        h = hRT * RU * T[i] / W                                         # J/kg
        cp = (Y[i] * cpR * RU / W).sum()
        # adiabatic, constant p: d/dt sum Y_k h_k(T) = sum h_k dY_k/dt + cp dT/dt = 0
        assert abs(h @ f[1:] + cp * f[0]) <= 1e-11 * (np.abs(h) @ np.abs(f[1:]))


def test_rhs_zero_at_detailed_balance(oracle_lib, write_mech):
    """A <=> B at Y_B / Y_A = K_c: every rate of progress vanishes."""
    m = oracle_lib.Mechanism(write_mech(tiny.isomer_pair(A=1e6, dS_R=0.8)))
    K = math.exp(0.8)
    ya = 0.4 / (1 + K)
    f = m.rhs(PATM, _y(1000.0, [ya, 0.4 - ya, 0.6]))
    assert np.abs(f).max() <= 1e-15 * 1e6


# ---------------- Jacobian ----------------

@pytest.mark.parametrize("mech", ["m9", "m13", "m32", "m13x", "m32x"])
def test_analytic_jacobian_matches_complex_step(oracle_lib, mech):
    m = oracle_lib.Mechanism(mech_path(mech))
    T, p, Y = uniform_cells(mech_text(mech), 8, 3)
    for i in range(8):
        y = _y(T[i], Y[i])
        J = m.jac(p[i], y)
        Jc = m.jac_cs(p[i], y)
        # scale of each entry: the terms that make it up can cancel, so compare
        # against the row magnitude times the column's scale
        sc = np.abs(Jc).max(axis=1, keepdims=True) * np.maximum(np.abs(y), 1e-3)[None, :] \
            / np.maximum(np.abs(y), 1e-3).max()
        assert np.all(np.abs(J - Jc) <= 1e-11 * (np.abs(Jc) + sc)), mech


def test_complex_step_matches_finite_differences(m9):
    T, p, Y = uniform_cells(mech_text("m9"), 2, 11)
    y = _y(1800.0, Y[0])
    Jc = m9.jac_cs(p[0], y)
    for j in range(10):
        d = 1e-6 * max(abs(y[j]), 1e-4)
        yp, ym = y.copy(), y.copy()
        yp[j] += d
        ym[j] -= d
        fd = (m9.rhs(p[0], yp) - m9.rhs(p[0], ym)) / (2 * d)
        assert np.allclose(fd, Jc[:, j], rtol=1e-5, atol=1e-6 * np.abs(Jc).max())


@pytest.mark.parametrize("kind", ["thirdbody", "lindemann", "troe"])
def test_jacobian_falloff_terms(oracle_lib, write_mech, kind):
    m = oracle_lib.Mechanism(write_mech(tiny.falloff(kind=kind, eff={"N2": 2.5, "AB": 0.7},
                                                     troe=(0.4, 150.0, 2500.0, 6000.0))))
    for p in (0.05 * PATM, 3 * PATM, 300 * PATM):
        y = _y(1700.0, [0.1, 0.2, 0.3, 0.4])
        J, Jc = m.jac(p, y), m.jac_cs(p, y)
        assert np.allclose(J, Jc, rtol=1e-11, atol=1e-12 * np.abs(Jc).max())
