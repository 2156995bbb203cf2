"""Pins of the oracle's linear algebra and Rosenbrock integrator: library
routines, order conditions, closed-form solutions, matrix exponentials,
brute-force Gibbs equilibrium and step refinement."""
import math

import numpy as np
import pytest
import scipy.linalg

from workloads import mech_path, mech_text, tiny
from workloads.states import uniform_cells, rde_field

RU = 8.314462618
PATM = 101325.0


def _y(T, Y):
    return np.concatenate([[T], Y])


# ---------------- LU ----------------

@pytest.mark.parametrize("n", [1, 3, 10, 14, 33])
def test_lu_solve_matches_lapack(oracle_lib, n):
    rng = np.random.default_rng(n)
    for trial in range(5):
        A = rng.standard_normal((n, n)) * np.exp(rng.uniform(-8, 8, (n, 1)))
        if trial == 0 and n > 1:
            A[0, 0] = 0.0                     # forces a pivot on the first column
        b = rng.standard_normal(n)
        LU, piv, rc = oracle_lib.lu(A)
        assert rc == 0
        x = oracle_lib.lu_solve(LU, piv, b)
        xr = np.linalg.solve(A, b)
        assert np.allclose(x, xr, rtol=1e-9, atol=1e-12 * np.abs(xr).max())
        P, L, U = scipy.linalg.lu(A)
        assert np.allclose(np.abs(np.diag(U)), np.abs(np.diag(np.triu(LU))), rtol=1e-10)


def test_lu_pivot_tie_takes_lowest_row_and_singular_detected(oracle_lib):
    A = np.array([[1.0, 2.0, 3.0], [-3.0, 1.0, 0.0], [3.0, 5.0, 1.0]])
    _, piv, rc = oracle_lib.lu(A)
    assert rc == 0 and piv[0] == 1                 # |-3| == |3|: row 1 wins the tie
    _, _, rc = oracle_lib.lu(np.array([[1.0, 2.0], [2.0, 4.0]]))
    assert rc != 0


# ---------------- tableau ----------------

def _original_form(t):
    """Recover (alpha, Gamma, b, b_hat) of the untransformed method from the
    u-form coefficients: Gamma^-1 = diag(1/gamma) - C, alpha = A Gamma,
    b = m Gamma (Hairer & Wanner, Sec. IV.7)."""
    s = t["s"]
    G = np.linalg.inv(np.diag(np.full(s, 1.0 / t["gamma"])) - t["c"])
    return t["a"] @ G, G, t["m"] @ G, (t["m"] - t["e"]) @ G


@pytest.mark.parametrize("method", ["RODAS4", "ROS4"])
def test_rosenbrock_order_conditions(oracle_lib, method):
    """Both tableaux the oracle carries: the eight order-4 conditions of a
    Rosenbrock method (Hairer & Wanner, Sec. IV.7, Table 7.1), the embedded
    solution of order 3 (and not 4), stiff accuracy (RODAS4 only), and
    stability: |R(iw)| <= 1 and R(-inf) = 0 for RODAS4; for ROS4 the
    published coefficients are rounded (gamma = 0.57282), so R(-inf) is
    small, not zero."""
    t = oracle_lib.tableau(getattr(oracle_lib, method))
    alpha, G, b, bh = _original_form(t)
    g = t["gamma"]
    s = t["s"]
    assert s == (6 if method == "RODAS4" else 4)
    assert np.allclose(np.diag(G), g, atol=1e-14)
    bp = alpha + G - np.diag(np.diag(G))
    a_i, be_i = alpha.sum(1), bp.sum(1)

    def conds(w):
        return np.array([w.sum() - 1, w @ be_i - (0.5 - g), w @ a_i**2 - 1 / 3,
                         w @ (bp @ be_i) - (1 / 6 - g + g * g), w @ a_i**3 - 1 / 4,
                         w @ (a_i * (alpha @ be_i)) - (1 / 8 - g / 3),
                         w @ (bp @ a_i**2) - (1 / 12 - g / 3),
                         w @ (bp @ (bp @ be_i)) - (1 / 24 - g / 2 + 1.5 * g * g - g**3)])
    assert np.abs(conds(b)).max() < 1e-13               # order 4
    assert np.abs(conds(bh)[:4]).max() < 1e-13          # embedded order 3
    assert abs(conds(bh)[4:]).max() > 1e-6              # ... and not 4
    if method == "RODAS4":
        assert np.allclose(b, alpha[-1] + G[-1], atol=1e-14)   # stiffly accurate
    # stability function R(z) = 1 + z b^T (I - z B)^-1 1
    B = alpha + G
    R = lambda z: 1 + z * b @ np.linalg.solve(np.eye(s) - z * B, np.ones(s))
    assert abs(R(-1e12)) < (1e-9 if method == "RODAS4" else 1e-4)
    assert max(abs(R(1j * w)) for w in np.logspace(-3, 4, 200)) <= 1 + 1e-12
    # a plausible mistake in any stored coefficient (a, c or the weights m,
    # off by 0.1 %) breaks an order condition
    for key in ("a", "c", "m"):
        arr = t[key]
        for ix in zip(*np.nonzero(arr)):
            t2 = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in t.items()}
            t2[key][ix] *= 1.001
            a2, G2, b2, _ = _original_form(t2)
            bp2 = a2 + G2 - np.diag(np.diag(G2))
            ai2, bei2 = a2.sum(1), bp2.sum(1)
            r = [b2.sum() - 1, b2 @ bei2 - (0.5 - g), b2 @ ai2**2 - 1 / 3,
                 b2 @ (bp2 @ bei2) - (1 / 6 - g + g * g), b2 @ ai2**3 - 1 / 4,
                 b2 @ (ai2 * (a2 @ bei2)) - (1 / 8 - g / 3), b2 @ (bp2 @ ai2**2) - (1 / 12 - g / 3),
                 b2 @ (bp2 @ (bp2 @ bei2)) - (1 / 24 - g / 2 + 1.5 * g * g - g**3)]
            assert max(abs(x) for x in r) > 1e-8, (method, key, ix)


def test_ros4_integrates_like_rodas4(oracle_lib):
    """ROS4 is a second, independent order-4 method: an adaptive solve of a
    reacting front cell with it lands within the tolerance of RODAS4's."""
    m = oracle_lib.Mechanism(mech_path("m9"))
    T, p, Y, reg = rde_field(mech_text("m9"), 64, 64, 101)
    idx = np.concatenate([np.where(reg == r)[0][:4] for r in (0, 1, 2)])
    Ta, Ya, na, _, sa = m.integrate(T[idx], p[idx], Y[idx], 5e-9, 1e-10, 1e-14)
    Tb, Yb, nb, _, sb = m.integrate(T[idx], p[idx], Y[idx], 5e-9, 1e-10, 1e-14, method=oracle_lib.ROS4)
    assert np.all(sa == 0) and np.all(sb == 0)
    assert np.all(np.abs(Ta - Tb) <= 1e-7 * Ta), np.abs(Ta - Tb).max()
    assert np.abs(Ya - Yb).max() <= 1e-9


def test_observed_order_on_nonlinear_problem(oracle_lib):
    """Fixed-step global error on a reacting stretch of a detonation-front cell
    (M9, the middle of its adaptive solve) falls like h^4."""
    m = oracle_lib.Mechanism(mech_path("m9"))
    T, p, Y, reg = rde_field(mech_text("m9"), 64, 64, 101)
    i = int(np.where(reg == 1)[0][0])
    hs = m.step_sizes(T[i], p[i], Y[i], 5e-9, 1e-8, 1e-12)
    k = len(hs) // 2
    ystart = m.replay(p[i], _y(T[i], Y[i]), hs[:k])
    H = hs[k:k + 20].sum()

    def solve(nsteps):
        y = ystart.copy()
        for _ in range(nsteps):
            y, _ = m.step(p[i], y, H / nsteps)
        return y
    ref = solve(4096)
    assert np.abs(ref - ystart)[1:].max() > 1e-3          # the state really moves
    errs = [np.abs(solve(n) - ref)[1:].max() for n in (10, 20, 40)]
    rates = [math.log2(errs[k] / errs[k + 1]) for k in range(2)]
    assert min(rates) > 3.8, (errs, rates)


# ---------------- closed forms ----------------

def test_reversible_isomerisation_closed_form(oracle_lib, write_mech):
    """A <=> B, dH = 0: T constant, Y_A = Y_eq + (Y_A0 - Y_eq) exp(-(kf + kr) t)."""
    kf, dS = 2.0e8, 1.3
    m = oracle_lib.Mechanism(write_mech(tiny.isomer_pair(A=kf, dS_R=dS)))
    kr = kf * math.exp(-dS)
    s = 0.5
    T, Y = np.array([1300.0]), np.array([[0.45, 0.05, 0.5]])
    for dt in (1e-9, 5e-9, 3e-8):
        Te, Ye, na, nj, st = m.integrate(T, PATM, Y, dt, 1e-10, 1e-14)
        yeq = kr * s / (kf + kr)
        ya = yeq + (0.45 - yeq) * math.exp(-(kf + kr) * dt)
        assert st[0] == 0 and Te[0] == pytest.approx(1300.0, rel=1e-13)
        assert Ye[0, 0] == pytest.approx(ya, rel=1e-8, abs=1e-12)
        assert Ye[0, 1] == pytest.approx(s - ya, rel=1e-8, abs=1e-12)


def test_irreversible_limit_closed_form(oracle_lib, write_mech):
    """K_c = e^60: the reverse rate is negligible and Y_A = Y_A0 exp(-k t)."""
    k = 7.0e7
    m = oracle_lib.Mechanism(write_mech(tiny.isomer_pair(A=k, dS_R=60.0)))
    Te, Ye, _, _, st = m.integrate([900.0], PATM, [[0.3, 0.0, 0.7]], 4e-8, 1e-10, 1e-15)
    assert st[0] == 0
    assert Ye[0, 0] == pytest.approx(0.3 * math.exp(-k * 4e-8), rel=1e-8)


def _network():
    rates = [(0, 1, 3.0e7), (1, 2, 1.0e8), (0, 2, 5.0e6), (2, 3, 4.0e7), (3, 0, 2.0e6)]
    dS = [0.0, 0.7, -0.4, 1.1]
    return rates, dS


def _network_matrix(rates, dS):
    """dY/dt = K Y for the isomer network (all W equal, b = Ea = 0)."""
    n = len(dS)
    Ks = []
    for i, j, A in rates:
        kr = A * math.exp(-(dS[j] - dS[i]))
        Kj = np.zeros((n, n))
        Kj[i, i] -= A
        Kj[j, i] += A
        Kj[j, j] -= kr
        Kj[i, j] += kr
        Ks.append(Kj)
    return sum(Ks), Ks


def test_isomer_network_matches_expm(oracle_lib, write_mech):
    rates, dS = _network()
    m = oracle_lib.Mechanism(write_mech(tiny.isomer_network(rates, dS)))
    K, _ = _network_matrix(rates, dS)
    y0 = np.array([0.25, 0.05, 0.1, 0.2])
    dt = 2e-8
    Te, Ye, _, _, st = m.integrate([1000.0], 2 * PATM, [np.append(y0, 0.4)], dt, 1e-11, 1e-16)
    ref = scipy.linalg.expm(K * dt) @ y0
    assert st[0] == 0 and Te[0] == pytest.approx(1000.0, rel=1e-14)
    assert np.allclose(Ye[0, :4], ref, rtol=1e-9, atol=1e-13)
    assert Ye[0, 4] == pytest.approx(0.4, rel=1e-14)


def _hp_equilibrium(T0, Y0, p, W, a1, a6, a7):
    """Brute-force constant-(h, p) equilibrium of H2 <=> 2H with inert N2 by
    Gibbs minimisation over the extent, using the constant-cp thermo
    cp/R = a1, H/RT = a1 + a6/T, S/R = a1 ln T + a7 (species H2, H, N2)."""
    n0 = Y0 / W                                 # mol per kg
    nu = np.array([-1.0, 2.0, 0.0])

    def h_mass(T, n):
        return (n * RU * (a1 * T + a6)).sum()

    def mu_over_rt(T, n):
        x = n / n.sum()
        g = a1 + a6 / T - (a1 * math.log(T) + a7)
        return g + np.log(np.maximum(x, 1e-300) * p / PATM)

    def extent(T):
        lo, hi = -n0[1] / 2 * (1 - 1e-15), n0[0] * (1 - 1e-15)
        grid = np.linspace(lo, hi, 2001)[1:-1]
        G = [(lambda n: (n * mu_over_rt(T, n)).sum())(n0 + nu * x) for x in grid]
        k = int(np.argmin(G))
        a, b = grid[max(k - 1, 0)], grid[min(k + 1, len(grid) - 1)]
        for _ in range(200):                  # bisection on dG/dxi
            c = 0.5 * (a + b)
            if nu @ mu_over_rt(T, n0 + nu * c) > 0:
                b = c
            else:
                a = c
        return n0 + nu * 0.5 * (a + b)

    h0 = h_mass(T0, n0)
    Ta, Tb = 500.0, T0
    for _ in range(100):                        # bisection on h(T, n_eq(T)) = h0
        Tc = 0.5 * (Ta + Tb)
        if h_mass(Tc, extent(Tc)) > h0:
            Tb = Tc
        else:
            Ta = Tc
    T = 0.5 * (Ta + Tb)
    return T, extent(T) * W


def test_hp_equilibrium_matches_gibbs_minimisation(oracle_lib, write_mech):
    m = oracle_lib.Mechanism(write_mech(tiny.dissociation(A=1e13, Ea=150.0)))
    W = m.weights()
    a1, a6, a7 = np.array([3.5, 2.5, 3.5]), np.array([-1043.5, 25000.0, -1043.5]), \
        np.array([-3.0, -1.0, 4.0])
    Y0 = np.array([0.06, 0.0, 0.94])
    for T0, p in ((3400.0, PATM), (3600.0, 5 * PATM)):
        Te, Ye, _, _, st = m.integrate([T0], p, [Y0], 1e-3, 1e-10, 1e-16)
        Teq, Yeq = _hp_equilibrium(T0, Y0, p, W, a1, a6, a7)
        assert st[0] == 0
        assert Te[0] == pytest.approx(Teq, rel=1e-6)
        assert np.allclose(Ye[0], Yeq, atol=1e-8)
        assert Ye[0, 1] > 1e-4                     # a real dissociation equilibrium


# ---------------- tolerance behaviour ----------------

def test_refinement_and_tolerance_convergence(oracle_lib):
    m = oracle_lib.Mechanism(mech_path("m9"))
    T, p, Y, reg = rde_field(mech_text("m9"), 64, 64, 101)
    idx = np.concatenate([np.where(reg == 1)[0][:6], np.where(reg == 2)[0][:6]])
    T, p, Y = T[idx], p[idx], Y[idx]
    dt = 5e-9
    ref = m.integrate(T, p, Y, dt, 1e-13, 1e-18)
    errs = []
    for rtol in (1e-6, 1e-8):
        r = m.integrate(T, p, Y, dt, rtol, rtol * 1e-4)
        errs.append(max(np.abs(r[1] - ref[1]).max(), (np.abs(r[0] - ref[0]) / ref[0]).max()))
        half = m.integrate(*m.integrate(T, p, Y, dt / 2, rtol, rtol * 1e-4)[:1], p,
                           m.integrate(T, p, Y, dt / 2, rtol, rtol * 1e-4)[1], dt / 2, rtol,
                           rtol * 1e-4)
        assert np.abs(half[1] - r[1]).max() < 100 * rtol
    assert errs[0] < 100 * 1e-6 and errs[1] < 100 * 1e-8
    assert errs[1] < errs[0] / 10


def test_invariants_over_a_step(oracle_lib):
    m = oracle_lib.Mechanism(mech_path("m9"))
    T, p, Y = uniform_cells(mech_text("m9"), 256, 100)
    Te, Ye, na, nj, st = m.integrate(T, p, Y, 1e-8, 1e-8, 1e-12)
    assert np.all(st == 0)
    assert np.abs(Ye.sum(1) - 1.0).max() < 1e-13 * max(na.max(), 1)
    W = m.weights()
    comps = [dict((kv.split("=")[0], int(kv.split("=")[1])) for kv in l.split()[2].split(","))
             for l in mech_text("m9").splitlines() if l.startswith("species")]
    for e in ("H", "O", "N"):
        a = np.array([c.get(e, 0) for c in comps]) / W
        assert np.abs(Ye @ a - Y @ a).max() < 1e-12 * (Y @ a).max()

    def h(Tv, Yv):
        return np.array([(Yv[i] * m.thermo(Tv[i])[1] * RU * Tv[i] / W).sum() for i in range(len(Tv))])
    cp = np.array([(Y[i] * m.thermo(T[i])[0] * RU / W).sum() for i in range(len(T))])
    dh = np.abs(h(Te, Ye) - h(T, Y))
    assert np.all(dh <= 10 * 1e-8 * cp * Te + 1e-9)


# ---------------- failure handling ----------------

def test_cell_status_codes(oracle_lib):
    m = oracle_lib.Mechanism(mech_path("m9"))
    T, p, Y = uniform_cells(mech_text("m9"), 4, 100)
    T = T.copy()
    T[2] = -5.0
    Yn = Y.copy()
    Yn[3, 0] = np.nan
    Te, Ye, na, nj, st = m.integrate(T, p, Yn, 1e-8, 1e-8, 1e-12, max_substeps=1)
    assert st[2] == oracle_lib.CELL_BADINPUT and Te[2] == -5.0
    assert st[3] == oracle_lib.CELL_BADINPUT
    hot = int(np.argmax(T[:2]))
    assert st[hot] == oracle_lib.CELL_MAXSTEPS and na[hot] + nj[hot] == 1
    Te, Ye, na, nj, st = m.integrate(T[:2], p[:2], Y[:2], 1e-8, 1e-8, 1e-12, hmin_rel=0.5)
    assert st[hot] == oracle_lib.CELL_HMIN


def _flops_per_substep_formula(ns, nr, s=6):
    """The method's algorithmic work per substep attempt used for the roofline:
    Jacobian 50 nr + 4 n^2, LU (2/3) n^3, per stage a source evaluation
    40 ns + 30 nr, two triangular solves 2 n^2 and the stage combinations 2 s n."""
    n = ns + 1
    return (50 * nr + 4 * n * n) + (2.0 / 3.0) * n**3 + s * (40 * ns + 30 * nr + 2 * n * n + 2 * s * n)


@pytest.mark.parametrize("name", ["m9", "m13", "m32"])
def test_counted_mode(oracle_lib, name):
    """The oracle's counted instantiation of one RODAS4 step attempt: for m9
    the source terms are evaluated exactly six times (two exponentials per
    reaction each time) and the counts do not depend on the state; for every
    mechanism a plain implementation's flop count is at or above the method's
    minimal per-substep work (the roofline's figure) and within 3x of it."""
    om = oracle_lib.Mechanism(mech_path(name))
    T, p, Y = uniform_cells(mech_text(name), 3, 17)
    counts = []
    for i in range(3):
        y = np.concatenate([[T[i]], Y[i]])
        c = om.count_step(p[i], y, 1e-9)
        counts.append(c)
    nr = om.nr
    if name == "m9":
        assert counts[0] == counts[1] == counts[2]
    f = _flops_per_substep_formula(om.ns, nr)
    for c in counts:
        assert f <= c["flop"] <= 3.0 * f, (name, c, f)
    if name == "m9":
        assert counts[0]["exp"] == 6 * 2 * nr
