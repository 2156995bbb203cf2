"""Pins of the oracle's irreversible reactions, SRI falloff and pressure-
tabulated (PLOG) rates against special cases of their definitions, limits,
closed-form solutions and complex-step derivatives.  No GPU."""
import math

import numpy as np
import pytest

from workloads import tiny

RU = 8.314462618
PATM = 101325.0


def _y(T, Y):
    return np.concatenate([[T], Y])


Y4 = [0.1, 0.2, 0.3, 0.4]


# ---------------- irreversible reactions ----------------

def test_irreversible_has_no_reverse_rate(oracle_lib, write_mech):
    """'irrev': k_r = 0 and q = k_f C_A C_B, with k_f as in the reversible
    reaction of the same rate."""
    mr = oracle_lib.Mechanism(write_mech(tiny.falloff(kind="elementary"), "r.mech"))
    mi = oracle_lib.Mechanism(write_mech(tiny.falloff(kind="elementary", irrev=True), "i.mech"))
    p, y = 2 * PATM, _y(1600.0, Y4)
    kfr, krr, qr = mr.rates(p, y)
    kfi, kri, qi = mi.rates(p, y)
    assert krr[0] > 0 and kri[0] == 0.0 and kfi[0] == kfr[0]
    rho = p / (RU * 1600.0) / sum(np.array(Y4) / mi.weights())
    CA, CB = rho * Y4[0] / mi.weights()[0], rho * Y4[1] / mi.weights()[1]
    assert qi[0] == pytest.approx(kfi[0] * CA * CB, rel=1e-14)


def test_irreversible_isomerisation_closed_form(oracle_lib, write_mech):
    """A => B with K_c favouring A (dS < 0): without the reverse reaction A
    still decays as Y_A0 exp(-k t) (dH = 0, so T stays constant)."""
    k = 5.0e7
    m = oracle_lib.Mechanism(write_mech(tiny.isomer_pair(A=k, dS_R=-2.0, irrev=True)))
    for dt in (2e-9, 4e-8):
        Te, Ye, _, _, st = m.integrate([1100.0], PATM, [[0.3, 0.1, 0.6]], dt, 1e-10, 1e-15)
        assert st[0] == 0 and Te[0] == pytest.approx(1100.0, rel=1e-13)
        assert Ye[0, 0] == pytest.approx(0.3 * math.exp(-k * dt), rel=1e-8)
        assert Ye[0, 1] == pytest.approx(0.4 - 0.3 * math.exp(-k * dt), rel=1e-8)


# ---------------- SRI falloff ----------------

def _k(m, p, T=1500.0):
    return m.rates(p, _y(T, Y4))[0][0]


def test_sri_with_unit_broadening_is_lindemann(oracle_lib, write_mech):
    """a = 0, c -> inf, d = 1, e = 0 gives F = 1: the Lindemann rate."""
    ms = oracle_lib.Mechanism(write_mech(tiny.falloff(kind="sri", sri=(0.0, 500.0, 1e300, 1.0, 0.0)), "s.mech"))
    ml = oracle_lib.Mechanism(write_mech(tiny.falloff(kind="lindemann"), "l.mech"))
    for p in (0.01 * PATM, PATM, 100 * PATM):
        assert _k(ms, p) == pytest.approx(_k(ml, p), rel=1e-14)


def test_sri_d_and_e_scale_the_rate(oracle_lib, write_mech):
    """F is proportional to d and to T^e at any pressure."""
    base = (0.6, 400.0, 1200.0, 1.0, 0.0)
    m1 = oracle_lib.Mechanism(write_mech(tiny.falloff(kind="sri", sri=base), "1.mech"))
    md = oracle_lib.Mechanism(write_mech(tiny.falloff(kind="sri", sri=base[:3] + (2.5, 0.0)), "d.mech"))
    me = oracle_lib.Mechanism(write_mech(tiny.falloff(kind="sri", sri=base[:3] + (1.0, 0.7)), "e.mech"))
    for p in (0.03 * PATM, 4 * PATM):
        for T in (900.0, 2100.0):
            assert _k(md, p, T) == pytest.approx(2.5 * _k(m1, p, T), rel=1e-13)
            assert _k(me, p, T) == pytest.approx(T ** 0.7 * _k(m1, p, T), rel=1e-13)


def test_sri_at_unit_reduced_pressure(oracle_lib, write_mech):
    """At P_r = 1 the exponent X is 1: k = k_inf / 2 * d (a e^(-b/T) + e^(-T/c)) T^e."""
    a, b, c, d, e = 0.45, 797.0, 979.0, 1.3, 0.2
    T = 1500.0
    m = oracle_lib.Mechanism(write_mech(tiny.falloff(kind="sri", sri=(a, b, c, d, e))))
    kinf, k0 = 1.0e13 * 1e-6, 1.0e16 * 1e-12
    M = kinf / k0                          # P_r = k0 [M] / k_inf = 1
    k = _k(m, M * RU * T, T)
    assert k == pytest.approx(kinf / 2 * d * (a * math.exp(-b / T) + math.exp(-T / c)) * T ** e, rel=1e-12)


def test_sri_high_pressure_limit(oracle_lib, write_mech):
    """P_r -> inf: X -> 0 (like 1 / log10(P_r)^2), so k -> k_inf d T^e."""
    d, e = 1.4, -0.3
    m = oracle_lib.Mechanism(write_mech(tiny.falloff(kind="sri", sri=(0.5, 300.0, 1500.0, d, e))))
    T = 1500.0
    assert _k(m, 1e100 * PATM, T) == pytest.approx(1.0e13 * 1e-6 * d * T ** e, rel=1e-4)
    assert _k(m, 1e200 * PATM, T) == pytest.approx(1.0e13 * 1e-6 * d * T ** e, rel=3e-5)


# ---------------- PLOG ----------------

ENTRIES = [(0.1 * PATM, 1.0e12, 0.5, 20.0), (PATM, 3.0e13, 0.1, 35.0),
           (10 * PATM, 2.0e14, -0.4, 50.0)]


def _arr(A, b, Ea, T):
    """k in SI for a bimolecular rate given in cm^3/(mol s), Ea in kJ/mol."""
    return A * 1e-6 * T ** b * math.exp(-Ea * 1e3 / (RU * T))


def test_plog_at_the_tabulated_pressures(oracle_lib, write_mech):
    m = oracle_lib.Mechanism(write_mech(tiny.plog(ENTRIES)))
    for T in (800.0, 1700.0):
        for p, A, b, Ea in ENTRIES:
            assert _k(m, p, T) == pytest.approx(_arr(A, b, Ea, T), rel=1e-13)


def test_plog_between_and_outside(oracle_lib, write_mech):
    """ln k is linear in ln p: at the geometric mean of two tabulated pressures
    it is the mean of their ln k; outside the table the end rate holds."""
    m = oracle_lib.Mechanism(write_mech(tiny.plog(ENTRIES)))
    T = 1300.0
    ks = [_arr(A, b, Ea, T) for _, A, b, Ea in ENTRIES]
    for i in range(2):
        pm = math.sqrt(ENTRIES[i][0] * ENTRIES[i + 1][0])
        assert _k(m, pm, T) == pytest.approx(math.sqrt(ks[i] * ks[i + 1]), rel=1e-13)
    # a quarter of the way in ln p
    pq = ENTRIES[0][0] ** 0.75 * ENTRIES[1][0] ** 0.25
    assert _k(m, pq, T) == pytest.approx(ks[0] ** 0.75 * ks[1] ** 0.25, rel=1e-13)
    assert _k(m, 1e-3 * PATM, T) == pytest.approx(ks[0], rel=1e-13)
    assert _k(m, 1e3 * PATM, T) == pytest.approx(ks[2], rel=1e-13)


def test_plog_main_rate_multiplies_and_single_entry_is_arrhenius(oracle_lib, write_mech):
    m1 = oracle_lib.Mechanism(write_mech(tiny.plog(ENTRIES), "1.mech"))
    m2 = oracle_lib.Mechanism(write_mech(tiny.plog(ENTRIES, A=3.0, b=0.25, Ea=-4.0), "2.mech"))
    T = 1100.0
    for p in (0.05 * PATM, 2 * PATM):
        assert _k(m2, p, T) == pytest.approx(3.0 * T ** 0.25 * math.exp(4e3 / (RU * T)) * _k(m1, p, T),
                                             rel=1e-13)
    ms = oracle_lib.Mechanism(write_mech(tiny.plog([ENTRIES[1]]), "s.mech"))
    me = oracle_lib.Mechanism(write_mech(tiny.falloff(kind="elementary", A=3.0e13, b=0.1, Ea=35.0), "e.mech"))
    for p in (0.01 * PATM, 50 * PATM):
        assert _k(ms, p, T) == pytest.approx(_k(me, p, T), rel=1e-13)


def test_plog_reverse_rate_from_equilibrium(oracle_lib, write_mech):
    """The reverse rate is k_f / K_c as for any reversible reaction."""
    mp = oracle_lib.Mechanism(write_mech(tiny.plog(ENTRIES), "p.mech"))
    T, p = 1400.0, 0.4 * PATM
    kf, kr, _ = mp.rates(p, _y(T, Y4))
    me = oracle_lib.Mechanism(write_mech(tiny.falloff(kind="elementary", A=1.0e13), "e.mech"))
    kfe, kre, _ = me.rates(p, _y(T, Y4))
    assert kf[0] / kr[0] == pytest.approx(kfe[0] / kre[0], rel=1e-13)


# ---------------- Jacobians of every kind ----------------

@pytest.mark.parametrize("case", ["sri", "sri_irrev", "plog", "plog_irrev", "troe_irrev", "thirdbody_irrev"])
def test_jacobian_matches_complex_step(oracle_lib, write_mech, case):
    eff = {"N2": 2.5, "AB": 0.7}
    if case.startswith("plog"):
        txt = tiny.plog(ENTRIES, A=1.7, b=0.1, Ea=3.0, irrev=case.endswith("irrev"))
    else:
        kind = case.split("_")[0]
        txt = tiny.falloff(kind=kind, eff=eff, troe=(0.4, 150.0, 2500.0, 6000.0),
                           sri=(0.45, 797.0, 979.0, 1.2, 0.3), irrev=case.endswith("irrev"))
    m = oracle_lib.Mechanism(write_mech(txt))
    for p in (0.05 * PATM, 0.7 * PATM, 3 * PATM, 300 * PATM):
        y = _y(1700.0, Y4)
        J, Jc = m.jac(p, y), m.jac_cs(p, y)
        assert np.allclose(J, Jc, rtol=1e-11, atol=1e-12 * np.abs(Jc).max()), p
