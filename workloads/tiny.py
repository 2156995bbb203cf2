"""Tiny hand-made mechanisms (text) whose solutions have closed forms or can be
found by brute force.  Input construction only.

Thermo here is either constant-cp (only a1, a6, a7 non-zero, so cp/R = a1,
H/RT = a1 + a6/T, S/R = a1 ln T + a7) or copied from a generated mechanism.
"""
from __future__ import annotations


def _fmt(x):
    return repr(float(x))


def _thermo(name, a1, a6, a7, tmid=1000.0, hi=None):
    lo = [a1, 0.0, 0.0, 0.0, 0.0, a6, a7]
    hi = lo if hi is None else hi
    return (f"thermo {name} 200.0 {_fmt(tmid)} 6000.0 " + " ".join(_fmt(x) for x in lo) + " "
            + " ".join(_fmt(x) for x in hi))


def text(elements, species, thermo, reactions):
    lines = ["chemmi-mech 1", "name tiny"]
    lines += [f"element {e} {_fmt(w)}" for e, w in elements]
    lines += [f"species {s} {c}" for s, c in species]
    lines += thermo
    lines += reactions
    lines.append("end")
    return "\n".join(lines) + "\n"


def isomer_pair(A=1.0e6, dS_R=1.0, b=0.0, Ea=0.0, irrev=False):
    """A <=> B + inert N2; A and B are isomers (same weight) with identical
    cp and H, differing only in S by dS_R (so K_c = exp(dS_R), dH = 0).
    irrev: A => B only."""
    return text([("H", 1.008), ("O", 15.999), ("N", 14.007)],
                [("A", "H=1,O=1"), ("B", "H=1,O=1"), ("N2", "N=2")],
                [_thermo("A", 3.5, -1000.0, 5.0), _thermo("B", 3.5, -1000.0, 5.0 + dS_R),
                 _thermo("N2", 3.5, -1000.0, 4.0)],
                [f"reaction elementary A=1 B=1 {_fmt(A)} {_fmt(b)} {_fmt(Ea)}" + (" irrev" if irrev else "")])


def isomer_network(rates, dS):
    """n isomers X0..X{n-1} (same weight, same cp and H, S differing by dS[i])
    linked by unimolecular reversible reactions rates = [(i, j, A)];
    b = Ea = 0, so the system is linear with constant coefficients."""
    n = len(dS)
    species = [(f"X{i}", "H=2,O=1") for i in range(n)] + [("N2", "N=2")]
    thermo = [_thermo(f"X{i}", 4.0, -2000.0, 10.0 + dS[i]) for i in range(n)]
    thermo.append(_thermo("N2", 3.5, -1000.0, 4.0))
    rx = [f"reaction elementary X{i}=1 X{j}=1 {_fmt(A)} 0.0 0.0" for i, j, A in rates]
    return text([("H", 1.008), ("O", 15.999), ("N", 14.007)], species, thermo, rx)


def dissociation(A=1.0e14, b=0.0, Ea=100.0, a6_H=25000.0, a7_H=-1.0, a7_H2=-3.0):
    """H2 <=> H + H with inert N2, constant-cp thermo (cp/R: H2 3.5, H 2.5,
    N2 3.5).  H carries formation enthalpy a6_H * R."""
    return text([("H", 1.008), ("N", 14.007)],
                [("H2", "H=2"), ("H", "H=1"), ("N2", "N=2")],
                [_thermo("H2", 3.5, -1043.5, a7_H2), _thermo("H", 2.5, a6_H, a7_H),
                 _thermo("N2", 3.5, -1043.5, 4.0)],
                [f"reaction elementary H2=1 H=2 {_fmt(A)} {_fmt(b)} {_fmt(Ea)}"])


def falloff(kind="troe", A=1.0e13, b=0.0, Ea=0.0, A0=1.0e16, b0=0.0, Ea0=0.0,
            troe=(0.5, 200.0, 2000.0, None), eff=None, sri=(0.5, 300.0, 1500.0, 1.0, 0.0),
            irrev=False):
    """A + B (+M) <=> AB (+M) with inert N2 and constant-cp thermo."""
    line = f"reaction {kind} A=1,B=1 AB=1 {_fmt(A)} {_fmt(b)} {_fmt(Ea)}"
    if kind in ("troe", "lindemann", "sri"):
        line += f" {_fmt(A0)} {_fmt(b0)} {_fmt(Ea0)}"
    if kind == "troe":
        a, t3, t1, t2 = troe
        line += f" {_fmt(a)} {_fmt(t3)} {_fmt(t1)} " + ("-" if t2 is None else _fmt(t2))
    if kind == "sri":
        line += " " + " ".join(_fmt(x) for x in sri)
    if eff:
        line += " eff=" + ",".join(f"{s}:{_fmt(v)}" for s, v in eff.items())
    if irrev:
        line += " irrev"
    return _abn2([line])


def plog(entries, A=1.0, b=0.0, Ea=0.0, irrev=False):
    """A + B <=> AB with a pressure-tabulated rate: entries = [(p Pa, A, b, Ea
    kJ/mol)], the main rate (A, b, Ea) a factor on it."""
    line = f"reaction plog A=1,B=1 AB=1 {_fmt(A)} {_fmt(b)} {_fmt(Ea)} plog=" + ",".join(
        ":".join(_fmt(x) for x in e) for e in entries)
    if irrev:
        line += " irrev"
    return _abn2([line])


def _abn2(reactions):
    return text([("H", 1.008), ("O", 15.999), ("N", 14.007)],
                [("A", "H=1"), ("B", "O=1"), ("AB", "H=1,O=1"), ("N2", "N=2")],
                [_thermo("A", 2.5, 20000.0, 2.0), _thermo("B", 2.5, 25000.0, 3.0),
                 _thermo("AB", 3.5, 4000.0, 4.0), _thermo("N2", 3.5, -1043.5, 4.0)],
                reactions)


def global_h2_air(A=3.6e18, b=0.0, Ea=120.0):
    """One irreversible global reaction 2 H2 + O2 => 2 H2O with inert N2, for
    the 1D driver's detonation run: constant-cp thermo (cp/R: H2 3.5, O2 3.7,
    H2O 4.5, N2 3.6) with H2O's standard formation enthalpy -241.8 kJ/mol at
    298.15 K (a6 = h_f/R - a1 298.15), the others zero.  A in cm^6/(mol^2 s),
    Ea in kJ/mol."""
    R = 8.314462618
    hf = -241.8e3 / R
    return text([("H", 1.008), ("O", 15.999), ("N", 14.007)],
                [("H2", "H=2"), ("O2", "O=2"), ("H2O", "H=2,O=1"), ("N2", "N=2")],
                [_thermo("H2", 3.5, -3.5 * 298.15, 0.0), _thermo("O2", 3.7, -3.7 * 298.15, 0.0),
                 _thermo("H2O", 4.5, hf - 4.5 * 298.15, 0.0), _thermo("N2", 3.6, -3.6 * 298.15, 0.0)],
                [f"reaction elementary H2=2,O2=1 H2O=2 {_fmt(A)} {_fmt(b)} {_fmt(Ea)} irrev"])
