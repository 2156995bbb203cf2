"""Pins of the oracle's 1D reactive-Euler step (oracle/euler1d.py): the flow
part against the exact Riemann solution of a calorically perfect gas (Sod's
problem, first-order convergence), a gas at rest staying at rest, and the
coupled step conserving mass, every element and the total (sensible plus
chemical) energy in a closed tube.  No GPU."""
import math

import numpy as np
import pytest

from workloads import mech_path, mech_text, tiny
from workloads.states import parse_species, stoich_air

RU = 8.314462618
PATM = 101325.0


@pytest.fixture(scope="module")
def inert(oracle_lib, tmp_path_factory):
    p = tmp_path_factory.mktemp("e") / "iso.mech"
    p.write_text(tiny.isomer_pair())
    return oracle_lib.Mechanism(str(p))


def _sod(om, n, tend=1.5e-4):
    from oracle import euler1d as E
    dx = 1.0 / n
    x = (np.arange(n) + 0.5) * dx
    Y = np.zeros((n, 3))
    Y[:, 2] = 1.0                                    # N2 only: cp/R = 3.5, gamma = 1.4
    pl, pr, Tl, Tr = 1e6, 1e5, 400.0, 300.0
    T, p = np.where(x < 0.5, Tl, Tr), np.where(x < 0.5, pl, pr)
    U = E.conserved(om, T, p, Y, np.zeros(n))
    R = RU / om.weights()[2]
    rl, rr = pl / (R * Tl), pr / (R * Tr)
    nst = int(math.ceil(tend / (0.2 * dx / math.sqrt(1.4 * pl / rl))))
    dt = tend / nst
    Tg = T.copy()
    for _ in range(nst):
        U, Tg, _, _ = E.step(om, U, dx, dt, T_guess=Tg)
    ex = E.riemann_exact(1.4, (rl, 0.0, pl), (rr, 0.0, pr), (x - 0.5) / tend)
    return U, ex


def test_sod_converges_to_the_exact_riemann_solution(inert):
    errs = []
    for n in (50, 100, 200, 400):
        U, ex = _sod(inert, n)
        errs.append(np.abs(U[:, 0] - ex[:, 0]).mean() / ex[:, 0].mean())
    # first order with a contact and a shock: L1 error ~ h^(1/2) .. h
    for a, b in zip(errs, errs[1:]):
        assert b < 0.85 * a, errs
    assert errs[-1] < 0.012, errs


def test_exact_riemann_solver_against_sod_star_state():
    """Sod's classic problem (gamma 1.4; rho, u, p = 1, 0, 1 | 0.125, 0, 0.1):
    star pressure 0.30313 and velocity 0.92745 (Toro, Table 4.3)."""
    from oracle import euler1d as E
    s = E.riemann_exact(1.4, (1.0, 0.0, 1.0), (0.125, 0.0, 0.1), [0.5, 1.2])
    assert s[0, 2] == pytest.approx(0.30313, abs=2e-5) and s[0, 1] == pytest.approx(0.92745, abs=2e-5)
    assert s[1, 0] == pytest.approx(0.26557, abs=2e-5)                 # shocked gas, right of the contact


def test_gas_at_rest_stays_at_rest(inert):
    from oracle import euler1d as E
    n = 16
    Y = np.tile([0.2, 0.3, 0.5], (n, 1))
    U = E.conserved(inert, np.full(n, 800.0), np.full(n, 2 * PATM), Y, np.zeros(n))
    U2, T, w, q = E.step(inert, U, 1e-3, 1e-7)
    # the isomerisation moves Y but not rho, momentum or the total energy
    assert np.array_equal(U2[:, 0], U[:, 0]) and np.all(U2[:, 1] == 0.0)
    assert np.allclose(T, 800.0, rtol=1e-12)


def _comps(name):
    return [dict((kv.split("=")[0], int(kv.split("=")[1])) for kv in l.split()[2].split(","))
            for l in mech_text(name).splitlines() if l.startswith("species")]


def _tube(om, name, n, hot=0.15):
    from oracle import euler1d as E
    names, W = parse_species(mech_text(name))
    Y = np.tile(stoich_air(names, W), (n, 1))
    x = (np.arange(n) + 0.5) / n
    T = np.where(x < hot, 2800.0, 300.0)
    p = np.where(x < hot, 30 * PATM, PATM)
    return E.conserved(om, T, p, Y, np.zeros(n)), T


def totals(om, U, dx, comps, elements):
    """Mass, element masses and total (sensible + chemical) energy of the tube."""
    from oracle import euler1d as E
    href, _ = E._species_h_cp(om, E.T_REF)
    W = om.weights()
    rhoY = U[:, 3:]
    el = [dx * (rhoY.sum(axis=0) @ np.array([c.get(e, 0) / w for c, w in zip(comps, W)])) for e in elements]
    return np.array([dx * U[:, 0].sum(), dx * (U[:, 2].sum() + (rhoY @ href).sum())] + el)


def test_coupled_step_conserves_mass_elements_energy(oracle_lib):
    from oracle import euler1d as E
    om = oracle_lib.Mechanism(mech_path("m9"))
    comps = _comps("m9")
    elements = sorted({e for c in comps for e in c})
    n, dx = 48, 1e-4
    U, T = _tube(om, "m9", n)
    t0 = totals(om, U, dx, comps, elements)
    for _ in range(6):
        U, T, w, q = E.step(om, U, dx, 2e-9, T_guess=T)
    t1 = totals(om, U, dx, comps, elements)
    assert np.abs(w).max() > 1e3                          # the hot gas reacts
    assert np.all(np.abs(t1 - t0) <= 1e-12 * np.abs(t0)), (t0, t1)


def test_cj_speed_matches_the_perfect_gas_closed_form(oracle_lib, write_mech):
    """Reactants and products with the same weight and cp/R = 3.5 (gamma 1.4):
    M_CJ = sqrt(H + 1) + sqrt(H), H = (gamma^2 - 1) q / (2 gamma R T0), q the
    heat of reaction per unit mass."""
    from oracle import euler1d as E
    q_mol = 80e3
    txt = tiny.text([("H", 1.008), ("O", 15.999), ("N", 14.007)],
                    [("A", "H=1,O=1"), ("B", "H=1,O=1"), ("N2", "N=2")],
                    [tiny._thermo("A", 3.5, 0.0, 5.0), tiny._thermo("B", 3.5, -q_mol / RU, 5.0),
                     tiny._thermo("N2", 3.5, 0.0, 4.0)],
                    ["reaction elementary A=1 B=1 1e6 0.0 50.0 irrev"])
    om = oracle_lib.Mechanism(write_mech(txt))
    W = om.weights()[0]
    D, T, p = E.cj_speed(om, 300.0, PATM, np.array([1.0, 0, 0]), np.array([0, 1.0, 0]))
    g, R = 1.4, RU / W
    H = (g * g - 1) * (q_mol / W) / (2 * g * R * 300.0)
    M = math.sqrt(H + 1) + math.sqrt(H)
    assert D == pytest.approx(M * math.sqrt(g * R * 300.0), rel=1e-9)
    assert p == pytest.approx(PATM * (1 + g * M * M) / (1 + g), rel=1e-6)   # p_CJ / p0 = (1 + gamma M^2)/(1 + gamma)
