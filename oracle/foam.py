"""OpenFOAM chemistry dictionaries -> `chemmi-mech 1` text, for the oracle.

TEST INFRASTRUCTURE ONLY: the oracle reads only its own text format, so an
OpenFOAM reactions/thermo pair reaches it through this converter; the GPU
library has its own reader, and the two are checked against each other and
against values the format fixes.

OpenFOAM's conventions followed: rates per kmol, A in (m^3/kmol)^(n-1)/s for a
reaction of order n (+1 for a third body and for k0), Ta = Ea/R in K; Troe F
as alpha, Tsss (T***), Ts (T*), Tss (T**); SRI F as a b c d e; third-body
efficiencies as coeffs ((species value) ...); species weights from molWeight
(kg/kmol); NASA-7 coefficients as highCpCoeffs / lowCpCoeffs.  The converter
writes A in cm-mol-s and Ea in kJ/mol, which its reader converts back.
"""
from __future__ import annotations

import re

RU = 8.314462618                  # J/(mol K)


def _tokens(text):
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return re.findall(r'"[^"]*"|[{}();]|[^\s{}();"]+', text)


def _parse(tokens, i=0, top=True):
    """Nested dict; a primitive entry is its list of tokens (parentheses kept)."""
    d = {}
    while i < len(tokens):
        t = tokens[i]
        if t == "}":
            return d, i + 1
        if t == ";":
            i += 1
            continue
        key = tokens[i + 1]
        if key == "{":
            d[t], i = _parse(tokens, i + 2, False)
            continue
        j = i + 1
        depth = 0
        while not (tokens[j] == ";" and depth == 0):
            depth += tokens[j] == "("
            depth -= tokens[j] == ")"
            j += 1
        d[t] = tokens[i + 1:j]
        i = j + 1
    return d, i


def _words(v):
    w = [x for x in v if x not in "()"]
    if len(w) > 0 and re.fullmatch(r"\d+", w[0]) and len(v) > 1 and v[1] == "(":
        w = w[1:]
    return w


def _side(txt):
    terms = {}
    for t in [x.strip() for x in txt.split("+")]:
        m = re.fullmatch(r"(\d*)(\S+)", t)
        n = int(m.group(1)) if m.group(1) else 1
        terms[m.group(2)] = terms.get(m.group(2), 0) + n
    return terms


def convert(reactions_text: str, thermo_text: str, name: str = "foam") -> str:
    R, _ = _parse(_tokens(reactions_text))
    T, _ = _parse(_tokens(thermo_text))
    species = _words(R["species"])
    elements = _words(R["elements"]) if "elements" in R else []
    comps = {}
    for s in species:
        comps[s] = {e: int(float(v[0])) for e, v in T[s]["elements"].items() if float(v[0]) > 0}
        for e in comps[s]:
            if e not in elements:
                elements.append(e)
    out = ["chemmi-mech 1", f"name {name}"]
    # element weights are not used: every species states its own molar mass
    out += [f"element {e} 1.0" for e in elements]
    for s in species:
        W = float(T[s]["specie"]["molWeight"][0])
        out.append(f"species {s} " + ",".join(f"{e}={n}" for e, n in comps[s].items()) + f" W={W!r}")
    for s in species:
        th = T[s]["thermodynamics"]
        lo = [float(x) for x in _words(th["lowCpCoeffs"])]
        hi = [float(x) for x in _words(th["highCpCoeffs"])]
        out.append(f"thermo {s} {float(th['Tlow'][0])!r} {float(th['Tcommon'][0])!r} {float(th['Thigh'][0])!r} "
                   + " ".join(repr(x) for x in lo) + " " + " ".join(repr(x) for x in hi))

    def arr(d, order):
        """(A in cm-mol-s, b, Ea in kJ/mol) from OpenFOAM's kmol-based values."""
        A = float(d["A"][0]) * 1e3 ** (order - 1)
        return A, float(d["beta"][0]), float(d["Ta"][0]) * RU / 1e3

    for rname, r in R["reactions"].items():
        typ = r["type"][0]
        typ = typ[:-len("Reaction")] if typ.endswith("Reaction") else typ
        irrev = typ.startswith("irreversible")
        kind = typ[len("irreversible"):] if irrev else typ[len("reversible"):]
        lhs, rhs = r["reaction"][0].strip('"').split("=")
        reac, prod = _side(lhs), _side(rhs)
        order = sum(reac.values())
        sides = ",".join(f"{s}={n}" for s, n in reac.items()) + " " + ",".join(f"{s}={n}" for s, n in prod.items())
        if kind == "Arrhenius":
            A, b, E = arr(r, order)
            line = f"reaction elementary {sides} {A!r} {b!r} {E!r}"
        elif kind == "ThirdBodyArrhenius":
            A, b, E = arr(r, order + 1)
            line = f"reaction thirdbody {sides} {A!r} {b!r} {E!r}"
        else:
            A, b, E = arr(r["kInf"], order)
            A0, b0, E0 = arr(r["k0"], order + 1)
            F = r["F"]
            head = f"{sides} {A!r} {b!r} {E!r} {A0!r} {b0!r} {E0!r}"
            if kind == "ArrheniusLindemannFallOff":
                line = f"reaction lindemann {head}"
            elif kind == "ArrheniusTroeFallOff":
                vals = [float(F[k][0]) for k in ("alpha", "Tsss", "Ts", "Tss")]
                line = f"reaction troe {head} " + " ".join(repr(v) for v in vals)
            elif kind == "ArrheniusSRIFallOff":
                line = f"reaction sri {head} " + " ".join(repr(float(F[k][0])) for k in "abcde")
            else:
                raise ValueError(f"{rname}: type {typ} not supported")
        if kind != "Arrhenius":
            w = _words(r["thirdBodyEfficiencies"]["coeffs"])
            line += " eff=" + ",".join(f"{w[k]}:{float(w[k + 1])!r}" for k in range(0, len(w), 2))
        if irrev:
            line += " irrev"
        out.append(line)
    out.append("end")
    return "\n".join(out) + "\n"
