"""Pins of the oracle's discrete adjoint of the frozen-step map: dot-product
test against forward-mode complex step, central finite differences, and the
Frechet derivative of the matrix exponential on a linear network."""
import math

import numpy as np
import pytest
import scipy.linalg

from workloads import mech_path, mech_text, tiny
from workloads.states import uniform_cells

PATM = 101325.0
RU = 8.314462618


@pytest.fixture(scope="module")
def m9(oracle_lib):
    return oracle_lib.Mechanism(mech_path("m9"))


def _cells(m9, k=3):
    T, p, Y = uniform_cells(mech_text("m9"), 64, 100)
    _, _, na, _, _ = m9.integrate(T, p, Y, 1e-8, 1e-8, 1e-12)
    # reacting cells with a modest number of steps keep the test quick
    idx = [i for i in np.argsort(na) if 8 <= na[i] <= 40][:k]
    return T[idx], p[idx], Y[idx]


def test_adjoint_dot_product_with_forward_complex_step(m9):
    T, p, Y = _cells(m9)
    rng = np.random.default_rng(0)
    nr = m9.nr
    for i in range(len(T)):
        gT, gY = rng.standard_normal(), rng.standard_normal(9)
        gT0, gY0, ga, gb, ge = m9.adjoint([T[i]], [p[i]], [Y[i]], 1e-8, 1e-8, 1e-12, [gT], [gY])
        hs = m9.step_sizes(T[i], p[i], Y[i], 1e-8, 1e-8, 1e-12)
        dy0 = rng.standard_normal(10) * np.concatenate([[T[i]], np.abs(Y[i])]) * 1e-3
        dpar = rng.standard_normal(3 * nr) * np.concatenate([np.ones(nr), np.ones(nr), np.full(nr, 1e4)])
        dyend = m9.replay_dir(p[i], np.concatenate([[T[i]], Y[i]]), hs, dy0, dpar)
        lhs = gT * dyend[0] + gY @ dyend[1:]
        rhs = gT0[0] * dy0[0] + gY0[0] @ dy0[1:] + ga @ dpar[:nr] + gb @ dpar[nr:2 * nr] \
            + ge @ dpar[2 * nr:]
        assert lhs == pytest.approx(rhs, rel=1e-11, abs=1e-14)


def test_adjoint_matches_central_differences(m9):
    T, p, Y = _cells(m9, 2)
    nr = m9.nr
    lnA, b, Ea = m9.params()
    par0 = np.concatenate([lnA, b, Ea])
    for i in range(len(T)):
        gT, gY = 1.0 / 1000.0, np.eye(9)[2]              # L = T_end / 1000 + Y_H2O,end
        gT0, gY0, ga, gb, ge = m9.adjoint([T[i]], [p[i]], [Y[i]], 1e-8, 1e-8, 1e-12, [gT], [gY])
        hs = m9.step_sizes(T[i], p[i], Y[i], 1e-8, 1e-8, 1e-12)
        y0 = np.concatenate([[T[i]], Y[i]])

        def L(y, par):
            e = m9.replay(p[i], y, hs, par=par)
            return e[0] / 1000.0 + e[3]
        fd = []
        for k in range(10):
            d = 1e-6 * max(abs(y0[k]), 1.0) if k == 0 else 1e-6
            yp, ym = y0.copy(), y0.copy()
            yp[k] += d
            ym[k] -= d
            fd.append((L(yp, par0) - L(ym, par0)) / (2 * d))
        for q in range(3 * nr):
            d = 1e-6 * max(abs(par0[q]), 1.0)
            pp, pm = par0.copy(), par0.copy()
            pp[q] += d
            pm[q] -= d
            fd.append((L(y0, pp) - L(y0, pm)) / (2 * d))
        fd = np.array(fd)
        ad = np.concatenate([gT0, gY0[0], ga, gb, ge])
        # relative to the gradient's own scale per block
        for sl in (slice(0, 1), slice(1, 10), slice(10, 10 + nr), slice(10 + nr, 10 + 2 * nr),
                   slice(10 + 2 * nr, 10 + 3 * nr)):
            scale = np.abs(ad[sl]).max()
            if scale > 0:
                assert np.abs(ad[sl] - fd[sl]).max() <= 1e-5 * scale, (sl, ad[sl], fd[sl])


def test_adjoint_linear_network_matches_expm_frechet(oracle_lib, write_mech):
    rates = [(0, 1, 3.0e7), (1, 2, 1.0e8), (0, 2, 5.0e6), (2, 3, 4.0e7), (3, 0, 2.0e6)]
    dS = [0.0, 0.7, -0.4, 1.1]
    m = oracle_lib.Mechanism(write_mech(tiny.isomer_network(rates, dS)))
    n = 4
    Ks = []
    for i, j, A in rates:
        kr = A * math.exp(-(dS[j] - dS[i]))
        Kj = np.zeros((n, n))
        Kj[i, i] -= A
        Kj[j, i] += A
        Kj[j, j] -= kr
        Kj[i, j] += kr
        Ks.append(Kj)
    K = sum(Ks)
    y0 = np.array([0.25, 0.05, 0.1, 0.2])
    w = np.array([0.3, -1.0, 0.5, 2.0])
    T, dt = 1000.0, 2e-8
    gT0, gY0, ga, gb, ge = m.adjoint([T], [2 * PATM], [np.append(y0, 0.4)], dt, 1e-11, 1e-16,
                                     [0.0], [np.append(w, 0.0)])
    E = scipy.linalg.expm(K * dt)
    assert np.allclose(gY0[0, :4], E.T @ w, rtol=1e-8)
    for j, Kj in enumerate(Ks):
        _, dE = scipy.linalg.expm_frechet(K * dt, Kj * dt)
        exact = w @ dE @ y0                          # dL/d ln A_j
        assert ga[j] == pytest.approx(exact, rel=1e-7, abs=1e-12)
        assert gb[j] == pytest.approx(exact * math.log(T), rel=1e-7, abs=1e-12)
        assert ge[j] == pytest.approx(-exact / (RU * T), rel=1e-7, abs=1e-16)
    assert abs(gT0[0]) < 1e-12                       # rates do not depend on T here
