"""The 1D reactive-Euler step of the library's driver, written plainly.

TEST INFRASTRUCTURE ONLY.  Conserved state per cell (rho, rho u, rho E_s,
rho Y_k) with E_s = e_s + u^2/2 and e_s = sum_k Y_k (h_k(T) - h_k(298.15 K))
- p/rho; ideal gas; reflecting ends; the local Lax-Friedrichs (Rusanov) flux
F = (F_L + F_R)/2 - s (U_R - U_L)/2 with s the larger |u| + c of the two
sides, c the frozen sound speed; forward Euler in time; the chemistry over
the same dt at constant pressure (the oracle's integrator), entering as
wdot_k = rho (Y_k(dt) - Y_k(0))/dt in the species equations and
qdot = -sum_k h_k(298.15 K) wdot_k in the sensible-energy equation
(the coupling terms of eqs. (20)-(21)).  Also an exact Riemann solver for a
calorically perfect gas (Toro, Riemann Solvers and Numerical Methods for
Fluid Dynamics, ch. 4) to pin the flow part.
"""
from __future__ import annotations

import math

import numpy as np

RU = 8.314462618
T_REF = 298.15


def _species_h_cp(om, T):
    """h_k (J/kg) and cp_k (J/(kg K)) at T."""
    cpR, hRT, _ = om.thermo(T)
    W = om.weights()
    return hRT * RU * T / W, cpR * RU / W


def primitives(om, U, T_guess=None):
    """(T, p, Y, u, c) of every cell; T by Newton's method on e_s(T)."""
    W = om.weights()
    href, _ = _species_h_cp(om, T_REF)
    n = U.shape[0]
    T = np.full(n, 1000.0) if T_guess is None else np.where(T_guess > 0, T_guess, 1000.0).astype(float)
    rho = U[:, 0]
    u = U[:, 1] / rho
    Y = U[:, 3:] / rho[:, None]
    es = U[:, 2] / rho - 0.5 * u * u
    Rm = RU * (Y / W).sum(axis=1)
    p = np.empty(n)
    c = np.empty(n)
    for i in range(n):
        t = T[i]
        for _ in range(100):
            h, cp = _species_h_cp(om, t)
            f = Y[i] @ (h - href) - Rm[i] * t - es[i]
            cv = Y[i] @ cp - Rm[i]
            tn = t - f / cv
            done = abs(tn - t) <= 1e-13 * t
            t = tn
            if done:
                break
        else:
            raise ValueError(f"cell {i}: no temperature")
        h, cp = _species_h_cp(om, t)
        cpm = Y[i] @ cp
        T[i] = t
        p[i] = rho[i] * Rm[i] * t
        c[i] = math.sqrt(cpm / (cpm - Rm[i]) * p[i] / rho[i])
    return T, p, Y, u, c


def physical_flux(U, p, u):
    F = U * u[:, None]
    F[:, 1] += p
    F[:, 2] += p * u
    return F


def step(om, U, dx, dt, rtol=1e-8, atol=1e-12, T_guess=None):
    """One step; returns (U_new, T of U, wdot, qdot)."""
    T, p, Y, u, c = primitives(om, U, T_guess)
    Te, Ye, _, _, st = om.integrate(T, p, Y, dt, rtol, atol)
    if np.any(st != 0):
        raise ValueError("chemistry failed")
    rho = U[:, 0]
    wdot = rho[:, None] * (Ye - Y) / dt
    href, _ = _species_h_cp(om, T_REF)
    qdot = -(wdot @ href)
    # ghost cells: mirror states with the velocity reversed
    Ug = np.vstack([U[:1], U, U[-1:]]).copy()
    Ug[0, 1] *= -1.0
    Ug[-1, 1] *= -1.0
    pg = np.concatenate([p[:1], p, p[-1:]])
    ug = np.concatenate([-u[:1], u, -u[-1:]])
    cg = np.concatenate([c[:1], c, c[-1:]])
    F = physical_flux(Ug, pg, ug)
    s = np.maximum(np.abs(ug[:-1]) + cg[:-1], np.abs(ug[1:]) + cg[1:])
    Fface = 0.5 * (F[:-1] + F[1:]) - 0.5 * s[:, None] * (Ug[1:] - Ug[:-1])
    S = np.zeros_like(U)
    S[:, 2] = qdot
    S[:, 3:] = wdot
    return U - dt / dx * (Fface[1:] - Fface[:-1]) + dt * S, T, wdot, qdot


def conserved(om, T, p, Y, u):
    """The conserved state of cells given (T, p, Y, u)."""
    W = om.weights()
    href, _ = _species_h_cp(om, T_REF)
    n = len(T)
    U = np.empty((n, 3 + om.ns))
    for i in range(n):
        Rm = RU * (Y[i] / W).sum()
        rho = p[i] / (Rm * T[i])
        h, _ = _species_h_cp(om, T[i])
        es = Y[i] @ (h - href) - Rm * T[i]
        U[i, 0] = rho
        U[i, 1] = rho * u[i]
        U[i, 2] = rho * (es + 0.5 * u[i] ** 2)
        U[i, 3:] = rho * Y[i]
    return U


def riemann_exact(gamma, left, right, xi):
    """Exact solution (rho, u, p) of the Riemann problem of a calorically
    perfect gas at similarity coordinates xi = x/t (Toro, ch. 4)."""
    rl, ul, pl = left
    rr, ur, pr = right
    cl, cr = math.sqrt(gamma * pl / rl), math.sqrt(gamma * pr / rr)

    def f(pk, rk, pk0, ck):
        if pk > pk0:                                    # shock
            A = 2.0 / ((gamma + 1.0) * rk)
            B = (gamma - 1.0) / (gamma + 1.0) * pk0
            return (pk - pk0) * math.sqrt(A / (pk + B))
        return 2.0 * ck / (gamma - 1.0) * ((pk / pk0) ** ((gamma - 1.0) / (2.0 * gamma)) - 1.0)

    lo, hi = 1e-12 * min(pl, pr), 10.0 * max(pl, pr)
    for _ in range(200):                                # bisection on the star pressure
        mid = 0.5 * (lo + hi)
        if f(mid, rl, pl, cl) + f(mid, rr, pr, cr) + ur - ul > 0:
            hi = mid
        else:
            lo = mid
    ps = 0.5 * (lo + hi)
    us = 0.5 * (ul + ur) + 0.5 * (f(ps, rr, pr, cr) - f(ps, rl, pl, cl))
    g1 = (gamma - 1.0) / (gamma + 1.0)
    out = []
    for x in xi:
        if x <= us:                                     # left of the contact
            if ps > pl:
                rs = rl * (ps / pl + g1) / (g1 * ps / pl + 1.0)
                S = ul - cl * math.sqrt((gamma + 1.0) / (2.0 * gamma) * ps / pl + (gamma - 1.0) / (2.0 * gamma))
                out.append((rl, ul, pl) if x < S else (rs, us, ps))
            else:
                rs = rl * (ps / pl) ** (1.0 / gamma)
                cs = cl * (ps / pl) ** ((gamma - 1.0) / (2.0 * gamma))
                if x < ul - cl:
                    out.append((rl, ul, pl))
                elif x > us - cs:
                    out.append((rs, us, ps))
                else:
                    r = rl * (2.0 / (gamma + 1.0) + g1 / cl * (ul - x)) ** (2.0 / (gamma - 1.0))
                    uu = 2.0 / (gamma + 1.0) * (cl + (gamma - 1.0) / 2.0 * ul + x)
                    pp = pl * (2.0 / (gamma + 1.0) + g1 / cl * (ul - x)) ** (2.0 * gamma / (gamma - 1.0))
                    out.append((r, uu, pp))
        else:                                           # right of the contact
            if ps > pr:
                rs = rr * (ps / pr + g1) / (g1 * ps / pr + 1.0)
                S = ur + cr * math.sqrt((gamma + 1.0) / (2.0 * gamma) * ps / pr + (gamma - 1.0) / (2.0 * gamma))
                out.append((rr, ur, pr) if x > S else (rs, us, ps))
            else:
                rs = rr * (ps / pr) ** (1.0 / gamma)
                cs = cr * (ps / pr) ** ((gamma - 1.0) / (2.0 * gamma))
                if x > ur + cr:
                    out.append((rr, ur, pr))
                elif x < us + cs:
                    out.append((rs, us, ps))
                else:
                    r = rr * (2.0 / (gamma + 1.0) - g1 / cr * (ur - x)) ** (2.0 / (gamma - 1.0))
                    uu = 2.0 / (gamma + 1.0) * (-cr + (gamma - 1.0) / 2.0 * ur + x)
                    pp = pr * (2.0 / (gamma + 1.0) - g1 / cr * (ur - x)) ** (2.0 * gamma / (gamma - 1.0))
                    out.append((r, uu, pp))
    return np.array(out)


def cj_speed(om, T0, p0, Y0, Yb):
    """Chapman-Jouguet speed of a detonation that takes the fresh state
    (T0, p0, Y0) to the complete-reaction composition Yb: the least D for
    which the Rayleigh line p = p0 + (rho0 D)^2 (v0 - v) meets the reactive
    Hugoniot h_b(T) - h_0 = (p - p0)(v0 + v)/2 (h with formation enthalpies,
    T = p v / R_b), i.e. where the two are tangent.  Returns (D, T, p) of the
    CJ state."""
    W = om.weights()
    R0 = RU * float(np.sum(Y0 / W))
    Rb = RU * float(np.sum(Yb / W))
    v0 = R0 * T0 / p0

    def h(Y, T):
        hk, _ = _species_h_cp(om, T)
        return float(Y @ hk)

    h0 = h(Y0, T0)

    def F(D, v):
        p = p0 + (D / v0) ** 2 * (v0 - v)
        T = p * v / Rb
        return h(Yb, T) - h0 - 0.5 * (p - p0) * (v0 + v), T, p

    def fmax(D):
        vs = np.linspace(0.02 * v0, v0, 400)
        vals = [F(D, v)[0] for v in vs]
        k = int(np.argmax(vals))
        a, b = vs[max(k - 1, 0)], vs[min(k + 1, len(vs) - 1)]
        for _ in range(60):                      # golden section on the bracket
            m1, m2 = a + 0.382 * (b - a), a + 0.618 * (b - a)
            if F(D, m1)[0] > F(D, m2)[0]:
                b = m2
            else:
                a = m1
        v = 0.5 * (a + b)
        return F(D, v)[0], v

    lo, hi = 100.0, 10000.0
    for _ in range(80):
        mid = 0.5 * (lo + hi)
        if fmax(mid)[0] >= 0.0:
            hi = mid
        else:
            lo = mid
    D = hi
    _, v = fmax(D)
    _, T, p = F(D, v)
    return D, T, p
