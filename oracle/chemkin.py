"""CHEMKIN-format mechanism -> `chemmi-mech 1` text, for the oracle.

TEST INFRASTRUCTURE ONLY: the oracle reads only its own text format, so a
CHEMKIN file reaches it through this converter; the GPU library has its own
CHEMKIN reader, and the two are checked against each other and against
values the format fixes.

The CHEMKIN conventions followed (as described in the CHEMKIN-II manual):
ELEMENTS with optional /weight/; SPECIES; THERMO [ALL] with an optional line
of default temperatures and four-line NASA-7 records in fixed columns
(upper-range coefficients first); REACTIONS with unit keywords for the
activation energy (cal/mol by default) and A in cm-mol-s; "=", "<=>",
"=>"; "+M" and "(+M)" / "(+species)"; auxiliary LOW, TROE, SRI, PLOG (p in
atm), DUPLICATE and species/efficiency/ pairs.  Anything else raises
ValueError.
"""
from __future__ import annotations

import re

# Standard atomic weights, g/mol (IUPAC abridged values).
WEIGHTS = {"H": 1.008, "D": 2.014, "HE": 4.0026, "C": 12.011, "N": 14.007, "O": 15.999,
           "F": 18.998, "NE": 20.180, "SI": 28.085, "S": 32.06, "CL": 35.45, "AR": 39.95,
           "KR": 83.798, "XE": 131.29}

RU = 8.314462618                  # J/(mol K)
PATM = 101325.0                   # Pa
# activation-energy units -> J/mol
E_UNITS = {"CAL/MOLE": 4.184, "KCAL/MOLE": 4184.0, "JOULES/MOLE": 1.0, "KJOULES/MOLE": 1000.0,
           "EVOLTS": 96485.33212}
SECTIONS = {"ELEMENTS": "ELEM", "ELEM": "ELEM", "SPECIES": "SPEC", "SPEC": "SPEC",
            "THERMO": "THERMO", "THER": "THERMO", "REACTIONS": "REAC", "REAC": "REAC"}


def _num(s):
    return float(s.strip().replace("D", "E").replace("d", "e"))


def _lines(text):
    return [l.split("!", 1)[0].rstrip() for l in text.splitlines()]


def _thermo_records(lines, default_tmid=1000.0):
    """{name: (composition, tmid, low[7], high[7])} from four-line records;
    the first record of a name wins."""
    out = {}
    i = 0
    # a line of three numbers sets the default temperatures
    while i < len(lines) and not lines[i].strip():
        i += 1
    if i < len(lines):
        try:
            t = [float(x) for x in lines[i].split()]
            if len(t) == 3:
                default_tmid = t[1]
                i += 1
        except ValueError:
            pass
    while i < len(lines):
        if not lines[i].strip():
            i += 1
            continue
        if lines[i].split()[0].upper() == "END":
            break
        l1, l2, l3, l4 = (l.ljust(80) for l in lines[i:i + 4])
        name = l1[:18].split()[0]
        comp = {}
        for f in [l1[24 + 5 * k: 29 + 5 * k] for k in range(4)] + [l1[73:78]]:
            sym, cnt = f[:2].strip().upper(), f[2:].strip()
            if sym and cnt and float(cnt) > 0:
                comp[sym] = comp.get(sym, 0) + int(float(cnt))
        tmid = _num(l1[65:73]) if l1[65:73].strip() else default_tmid
        a = [_num(row[15 * k: 15 * k + 15]) for row, n in ((l2, 5), (l3, 5), (l4, 4)) for k in range(n)]
        if name not in out:
            out[name] = (comp, tmid, a[7:14], a[0:7])
        i += 4
    return out


def _side(txt, species):
    m = re.search(r"\(\+([^)]*)\)", txt)
    fo = None
    if m:
        fo = m.group(1)
        txt = txt[:m.start()] + txt[m.end():]
    third = False
    terms = {}
    for t in [x for x in txt.split("+") if x]:
        if t.upper() == "M":
            third = True
            continue
        if t in species:
            nu, name = 1, t
        else:
            m2 = re.match(r"^(\d+)(.+)$", t)
            if not m2 or m2.group(2) not in species:
                raise ValueError(f"unknown species {t}")
            nu, name = int(m2.group(1)), m2.group(2)
        terms[name] = terms.get(name, 0) + nu
    return terms, third, fo


def convert(mech_text: str, thermo_text: str | None = None, name: str = "ck") -> str:
    """The mechanism as `chemmi-mech 1` text."""
    lines = _lines(mech_text)
    elements, species, thermo, rxn_lines, e_mult, kelvin = [], [], {}, [], 4.184, False
    i = 0
    while i < len(lines):
        words = lines[i].split()
        if not words:
            i += 1
            continue
        sec = SECTIONS.get(words[0].upper())
        if sec is None:
            raise ValueError(f"line {i + 1}: expected a section keyword")
        i += 1
        if sec == "THERMO":
            j = i
            while j < len(lines) and not (lines[j].split() and lines[j].split()[0].upper() in ("END",) + tuple(SECTIONS)):
                j += 1
            for k, v in _thermo_records(lines[i:j]).items():
                thermo.setdefault(k, v)
            i = j + 1 if j < len(lines) and lines[j].split()[0].upper() == "END" else j
            continue
        if sec == "REAC":
            for u in words[1:]:
                uu = u.upper()
                if uu in E_UNITS:
                    e_mult = E_UNITS[uu]
                elif uu == "KELVINS":
                    kelvin = True
                elif uu != "MOLES":
                    raise ValueError(f"unit {u} not supported")
            while i < len(lines) and lines[i].strip().upper() != "END":
                rxn_lines.append(lines[i])
                i += 1
            i += 1
            continue
        body = " ".join(words[1:])
        while i < len(lines):
            w = lines[i].split()
            if w and w[0].upper() == "END":
                i += 1
                break
            if w and w[0].upper() in SECTIONS:
                break
            body += " " + lines[i]
            i += 1
        if sec == "ELEM":
            for m in re.finditer(r"([A-Za-z]+)\s*(/\s*([^/]*)/)?", body):
                sym = m.group(1).upper()
                elements.append((sym, _num(m.group(3)) if m.group(3) else WEIGHTS[sym]))
        else:
            species += body.split()
    if thermo_text is not None:
        tl = _lines(thermo_text)
        while tl and not tl[0].strip():
            tl.pop(0)
        if tl and tl[0].split()[0].upper() in ("THERMO", "THER"):
            tl = tl[1:]
        for k, v in _thermo_records(tl).items():
            thermo.setdefault(k, v)

    def to_kj(E):
        return E * RU / 1000.0 if kelvin else E * e_mult / 1000.0

    out = ["chemmi-mech 1", f"name {name}"]
    out += [f"element {s} {w!r}" for s, w in elements]
    for s in species:
        comp = thermo[s][0]
        out.append(f"species {s} " + ",".join(f"{e}={comp[e]}" for e, _ in elements if comp.get(e, 0)))
    for s in species:
        comp, tmid, lo, hi = thermo[s]
        out.append(f"thermo {s} 200.0 {tmid!r} 6000.0 " + " ".join(repr(x) for x in lo) + " "
                   + " ".join(repr(x) for x in hi))

    # group each reaction line with its auxiliary lines
    rx = []
    for l in rxn_lines:
        if not l.strip():
            continue
        if "=" in l:
            t = l.split()
            rx.append({"eq": "".join(t[:-3]), "abe": [_num(x) for x in t[-3:]], "aux": []})
        else:
            rx[-1]["aux"].append(l)
    for r in rx:
        eq = r["eq"]
        if "<=>" in eq:
            lhs, rhs, irrev = *eq.split("<=>"), False
        elif "=>" in eq:
            lhs, rhs, irrev = *eq.split("=>"), True
        else:
            lhs, rhs, irrev = *eq.split("="), False
        reac, third, fo = _side(lhs, species)
        prod, _, _ = _side(rhs, species)
        A, b, E = r["abe"]
        low = troe = sri = None
        eff, plog = {}, []
        for l in r["aux"]:
            for m in re.finditer(r"([^\s/]+)\s*(/([^/]*)/)?", l):
                key, vals = m.group(1), m.group(3)
                v = [_num(x) for x in vals.split()] if vals is not None else []
                k = key.upper()
                if k in ("DUP", "DUPLICATE"):
                    continue
                if k == "LOW":
                    low = v
                elif k == "TROE":
                    troe = v
                elif k == "SRI":
                    sri = v if len(v) == 5 else v + [1.0, 0.0]
                elif k == "PLOG":
                    plog.append(v)
                elif key in species:
                    eff[key] = v[0]
                else:
                    raise ValueError(f"keyword {key} not supported")
        sides = ",".join(f"{s}={n}" for s, n in reac.items()) + " " + ",".join(f"{s}={n}" for s, n in prod.items())
        if plog:
            entries = ",".join(f"{p * PATM!r}:{a!r}:{bb!r}:{to_kj(e)!r}" for p, a, bb, e in plog)
            line = f"reaction plog {sides} 1.0 0.0 0.0 plog={entries}"
        elif fo is not None:
            kind = "troe" if troe else "sri" if sri else "lindemann"
            line = f"reaction {kind} {sides} {A!r} {b!r} {to_kj(E)!r} {low[0]!r} {low[1]!r} {to_kj(low[2])!r}"
            if troe:
                line += " " + " ".join(repr(x) for x in troe[:3]) + " " + (repr(troe[3]) if len(troe) == 4 else "-")
            if sri:
                line += " " + " ".join(repr(x) for x in sri)
            if fo.upper() != "M":
                eff = {s: (1.0 if s == fo else 0.0) for s in species}
        else:
            line = f"reaction {'thirdbody' if third else 'elementary'} {sides} {A!r} {b!r} {to_kj(E)!r}"
        if eff:
            line += " eff=" + ",".join(f"{s}:{v!r}" for s, v in eff.items())
        if irrev:
            line += " irrev"
        out.append(line)
    out.append("end")
    return "\n".join(out) + "\n"
