"""Seeded synthetic reaction mechanisms in the `chemmi-mech 1` text format.

The paper (Sec. 2.1) runs a detailed H2/air mechanism with its own reaction
and thermo data; that data is not reproduced here.  Instead this module draws
element-balanced mechanisms of the same kind from a seed:

* species: an H/O/N set (9 species), the same plus AR, HE, N, NO (13), and
  that plus 19 C1/C2 C-H-O species (32);
* reactions: element-balanced reversible reactions with at most two species on
  each side, every reacting species used at least once;
* modified-Arrhenius parameters: log10 A ~ U(8, 17) in cm-mol-s units of the
  reaction's order, b ~ U(-1.5, 2), Ea ~ U(0, 200) kJ/mol;
* third-body efficiencies and Troe falloff on the chosen reactions;
* NASA-7 two-range polynomials least-squares fitted to a smooth, seeded
  cp(T)/R curve, continuous in cp, H and S at T_mid = 1000 K.

This is input generation only: nothing here evaluates rates, equilibrium
constants or any other part of the integration.  The format is documented in
`format_doc()`; both the CPU oracle and the GPU library parse it with their own
readers.
"""
from __future__ import annotations

import itertools
import math
from dataclasses import dataclass, field

import numpy as np

FORMAT_TAG = "chemmi-mech 1"

# Standard atomic weights, g/mol (IUPAC abridged values).
ATOMIC_WEIGHTS = {"H": 1.008, "O": 15.999, "N": 14.007, "C": 12.011,
                  "AR": 39.95, "HE": 4.0026}

R_J = 8.314462618          # J/(mol K), used only to turn drawn H and S into the
T_REF = 298.15             # NASA-7 integration constants a6, a7.
T_LOW, T_MID, T_HIGH = 200.0, 1000.0, 6000.0

SPECIES_H_O_N = [
    ("H2", {"H": 2}), ("O2", {"O": 2}), ("H2O", {"H": 2, "O": 1}),
    ("H", {"H": 1}), ("O", {"O": 1}), ("OH", {"O": 1, "H": 1}),
    ("HO2", {"H": 1, "O": 2}), ("H2O2", {"H": 2, "O": 2}), ("N2", {"N": 2}),
]
SPECIES_EXTRA_13 = [("AR", {"AR": 1}), ("HE", {"HE": 1}), ("N", {"N": 1}),
                    ("NO", {"N": 1, "O": 1})]
SPECIES_EXTRA_32 = [
    ("CH4", {"C": 1, "H": 4}), ("CH3", {"C": 1, "H": 3}), ("CH2", {"C": 1, "H": 2}),
    ("CH", {"C": 1, "H": 1}), ("C", {"C": 1}), ("CO", {"C": 1, "O": 1}),
    ("CO2", {"C": 1, "O": 2}), ("HCO", {"H": 1, "C": 1, "O": 1}),
    ("CH2O", {"C": 1, "H": 2, "O": 1}), ("CH3O", {"C": 1, "H": 3, "O": 1}),
    ("CH2OH", {"C": 1, "H": 3, "O": 1}), ("CH3OH", {"C": 1, "H": 4, "O": 1}),
    ("C2H6", {"C": 2, "H": 6}), ("C2H5", {"C": 2, "H": 5}), ("C2H4", {"C": 2, "H": 4}),
    ("C2H3", {"C": 2, "H": 3}), ("C2H2", {"C": 2, "H": 2}), ("C2H", {"C": 2, "H": 1}),
    ("HCCO", {"H": 1, "C": 2, "O": 1}),
]
# Species whose standard formation enthalpy is zero (elements in their
# reference state, as far as they appear in these sets).
REFERENCE_SPECIES = {"H2", "O2", "N2", "AR", "HE"}
INERT_SPECIES = {"AR", "HE"}


@dataclass
class Reaction:
    kind: str                      # elementary | thirdbody | troe | lindemann | sri | plog
    reac: dict                     # species -> stoichiometric coefficient
    prod: dict
    A: float                       # cm-mol-s units of the reaction's order
    b: float
    Ea: float                      # kJ/mol
    low: tuple | None = None       # (A0, b0, Ea0) for falloff
    troe: tuple | None = None      # (alpha, T3, T1, T2 or None)
    eff: dict = field(default_factory=dict)
    sri: tuple | None = None       # (a, b, c, d, e)
    plog: list | None = None       # [(p Pa, A, b, Ea kJ/mol)], increasing p
    irrev: bool = False


@dataclass
class Mechanism:
    name: str
    elements: list
    species: list                  # [(name, composition)]
    thermo: dict                   # name -> (low[7], high[7])
    reactions: list


# --------------------------------------------------------------------------
# thermo: smooth cp(T)/R curve and its NASA-7 fit
# --------------------------------------------------------------------------

def _cp_curve(rng, n_atoms):
    """Seeded logistic cp/R(T): a low-T plateau rising smoothly by `rise`."""
    if n_atoms == 1:
        c0, rise = 2.5, rng.uniform(0.0, 0.3)
    else:
        c0 = 3.5 + rng.uniform(-0.1, 0.3) + 0.5 * (n_atoms - 2) * rng.uniform(0.8, 1.2)
        rise = rng.uniform(0.2, 1.5) * (n_atoms - 1)
    tc = rng.uniform(700.0, 1800.0)
    w = rng.uniform(200.0, 600.0)
    return lambda T: c0 + rise / (1.0 + np.exp(-(T - tc) / w))


def _fit_nasa(cp):
    """Two-range quartic fit of cp/R with equal values at T_MID (KKT system)."""
    tl = np.linspace(T_LOW, T_MID, 161)
    th = np.linspace(T_MID, T_HIGH, 201)
    s = 1000.0                                   # powers of T/1000 for conditioning
    Vl = np.vander(tl / s, 5, increasing=True)
    Vh = np.vander(th / s, 5, increasing=True)
    vm = np.vander(np.array([T_MID / s]), 5, increasing=True)[0]
    n = 10
    K = np.zeros((n + 1, n + 1))
    rhs = np.zeros(n + 1)
    K[:5, :5] = Vl.T @ Vl
    K[5:10, 5:10] = Vh.T @ Vh
    rhs[:5] = Vl.T @ cp(tl)
    rhs[5:10] = Vh.T @ cp(th)
    K[10, :5], K[10, 5:10] = vm, -vm
    K[:5, 10], K[5:10, 10] = vm, -vm
    sol = np.linalg.solve(K, rhs)
    scale = s ** np.arange(5)
    return sol[:5] / scale, sol[5:10] / scale


def _h_over_r(a, T):
    return (a[0] * T + a[1] * T**2 / 2 + a[2] * T**3 / 3 + a[3] * T**4 / 4
            + a[4] * T**5 / 5)


def _s_over_r(a, T):
    return (a[0] * math.log(T) + a[1] * T + a[2] * T**2 / 2 + a[3] * T**3 / 3
            + a[4] * T**4 / 4)


def _nasa7(rng, name, comp, hf_kj):
    n_atoms = sum(comp.values())
    lo5, hi5 = _fit_nasa(_cp_curve(rng, n_atoms))
    if n_atoms == 1:
        s298 = rng.uniform(14.0, 20.0)
    elif n_atoms == 2:
        s298 = rng.uniform(18.0, 27.0)
    else:
        s298 = rng.uniform(22.0, 28.0) + 1.5 * (n_atoms - 3)
    a6l = hf_kj * 1e3 / R_J - _h_over_r(lo5, T_REF)
    a7l = s298 - _s_over_r(lo5, T_REF)
    # integration constants of the high range from H, S continuity at T_MID
    a6h = _h_over_r(lo5, T_MID) + a6l - _h_over_r(hi5, T_MID)
    a7h = _s_over_r(lo5, T_MID) + a7l - _s_over_r(hi5, T_MID)
    low = [float(x) for x in lo5] + [float(a6l), float(a7l)]
    high = [float(x) for x in hi5] + [float(a6h), float(a7h)]
    return low, high


def _formation_enthalpy(rng, name, comp):
    if name in REFERENCE_SPECIES:
        return 0.0
    if sum(comp.values()) == 1:                 # free atoms: strongly endothermic
        return rng.uniform(150.0, 250.0)
    return rng.uniform(-150.0, 150.0)


# --------------------------------------------------------------------------
# reactions
# --------------------------------------------------------------------------

def _side_key(side):
    return tuple(sorted(side))


def _elem_vector(side, comps, elements):
    v = np.zeros(len(elements), dtype=np.int64)
    for sp in side:
        for e, c in comps[sp].items():
            v[elements.index(e)] += c
    return tuple(v)


def _candidates(reacting, comps, elements):
    """All element-balanced reactions with 1-2 species per side, each listed once."""
    sides = [(a,) for a in reacting] + [tuple(p) for p in
                                         itertools.combinations_with_replacement(reacting, 2)]
    groups = {}
    for s in sides:
        groups.setdefault(_elem_vector(s, comps, elements), []).append(_side_key(s))
    out = []
    for grp in groups.values():
        for l, r in itertools.combinations(sorted(set(grp)), 2):
            out.append((l, r))
    return out


def _to_dict(side):
    d = {}
    for s in side:
        d[s] = d.get(s, 0) + 1
    return d


def _dh(l, r, hf):
    return sum(hf[s] for s in r) - sum(hf[s] for s in l)


def _draw_arrhenius(rng):
    return 10.0 ** rng.uniform(8.0, 17.0), rng.uniform(-1.5, 2.0), rng.uniform(0.0, 200.0)


def _pick(rng, cands, n, must_cover, taken):
    """Choose n reactions from cands (not in taken), first covering must_cover."""
    chosen = []
    uncovered = set(must_cover)
    order = list(rng.permutation(len(cands)))
    while uncovered:
        sp = sorted(uncovered)[0]
        opts = [i for i in order if sp in cands[i][0] + cands[i][1]
                and cands[i] not in taken and i not in chosen]
        if not opts:
            raise RuntimeError(f"no reaction can use species {sp}")
        i = opts[int(rng.integers(len(opts)))]
        chosen.append(i)
        uncovered -= set(cands[i][0] + cands[i][1])
    for i in order:
        if len(chosen) >= n:
            break
        if i not in chosen and cands[i] not in taken:
            chosen.append(i)
    if len(chosen) < n:
        raise RuntimeError("not enough candidate reactions")
    return [cands[i] for i in chosen[:n]]


def generate(name, species, n_reactions, seed, n_troe=0, n_thirdbody=0,
             inert=(), max_dh_kj=400.0):
    rng = np.random.default_rng(seed)
    comps = dict(species)
    names = [s for s, _ in species]
    elements = []
    for _, c in species:
        for e in c:
            if e not in elements:
                elements.append(e)
    hf = {s: _formation_enthalpy(rng, s, comps[s]) for s in names}
    thermo = {s: _nasa7(rng, s, comps[s], hf[s]) for s in names}

    reacting = [s for s in names if s not in inert]
    cands = [c for c in _candidates(reacting, comps, elements)
             if abs(_dh(c[0], c[1], hf)) <= max_dh_kj]
    # falloff / third-body reactions need one side made of a single species
    assoc = [c for c in cands if (len(c[0]) == 1) != (len(c[1]) == 1)]
    taken = []
    special = []
    if n_troe + n_thirdbody:
        idx = rng.permutation(len(assoc))[: n_troe + n_thirdbody]
        special = [assoc[i] for i in idx]
        taken = list(special)
    elem_reactions = _pick(rng, cands, n_reactions - len(special), reacting, taken)

    eff_pool = [s for s in ("H2O", "H2", "AR", "HE", "CO2", "CO", "N2") if s in names]
    reactions = []
    for k, (l, r) in enumerate(special + elem_reactions):
        # The drawn Arrhenius parameters belong to the exothermic direction, so
        # the reverse rate k_f / K_c carries an activation energy of at least
        # Ea + |dH|.  (Drawn for the endothermic direction, the reverse rate
        # would grow like exp(|dH|/RT) as T falls, which no real mechanism does.)
        if _dh(l, r, hf) > 0.0:
            l, r = r, l
        A, b, Ea = _draw_arrhenius(rng)
        rx = Reaction("elementary", _to_dict(l), _to_dict(r), A, b, Ea)
        if k < len(special):
            picks = rng.permutation(len(eff_pool))[: int(rng.integers(2, 4))]
            rx.eff = {eff_pool[i]: float(rng.uniform(0.4, 12.0)) for i in sorted(picks)}
            if k < n_troe:
                rx.kind = "troe"
                rx.low = (10.0 ** rng.uniform(14.0, 19.0), rng.uniform(-2.5, 0.0),
                          rng.uniform(0.0, 100.0))
                t2 = float(rng.uniform(2000.0, 10000.0)) if rng.random() < 0.5 else None
                rx.troe = (float(rng.uniform(0.1, 0.9)), float(rng.uniform(50.0, 1000.0)),
                           float(rng.uniform(500.0, 5000.0)), t2)
            else:
                rx.kind = "thirdbody"
        reactions.append(rx)
    return Mechanism(name, elements, species, thermo, reactions)


# --------------------------------------------------------------------------
# text format
# --------------------------------------------------------------------------

def _fmt(x):
    return repr(float(x))


def _side(d):
    return ",".join(f"{s}={c}" for s, c in d.items())


def to_text(m: Mechanism) -> str:
    out = [FORMAT_TAG, f"name {m.name}"]
    for e in m.elements:
        out.append(f"element {e} {_fmt(ATOMIC_WEIGHTS[e])}")
    for s, c in m.species:
        out.append(f"species {s} " + ",".join(f"{e}={n}" for e, n in c.items()))
    for s, _ in m.species:
        lo, hi = m.thermo[s]
        out.append(f"thermo {s} {_fmt(T_LOW)} {_fmt(T_MID)} {_fmt(T_HIGH)} "
                   + " ".join(_fmt(x) for x in lo) + " " + " ".join(_fmt(x) for x in hi))
    for rx in m.reactions:
        line = f"reaction {rx.kind} {_side(rx.reac)} {_side(rx.prod)} " \
               f"{_fmt(rx.A)} {_fmt(rx.b)} {_fmt(rx.Ea)}"
        if rx.kind in ("troe", "lindemann", "sri"):
            line += " " + " ".join(_fmt(x) for x in rx.low)
        if rx.kind == "troe":
            a, t3, t1, t2 = rx.troe
            line += f" {_fmt(a)} {_fmt(t3)} {_fmt(t1)} " + ("-" if t2 is None else _fmt(t2))
        if rx.kind == "sri":
            line += " " + " ".join(_fmt(x) for x in rx.sri)
        if rx.kind not in ("elementary", "plog") and rx.eff:
            line += " eff=" + ",".join(f"{s}:{_fmt(v)}" for s, v in rx.eff.items())
        if rx.kind == "plog":
            line += " plog=" + ",".join(":".join(_fmt(x) for x in e) for e in rx.plog)
        if rx.irrev:
            line += " irrev"
        out.append(line)
    out.append("end")
    return "\n".join(out) + "\n"


# --------------------------------------------------------------------------
# the same mechanisms in the CHEMKIN text format
# --------------------------------------------------------------------------

def _e15(x):
    return f"{x:15.8E}"


def thermo_chemkin(m: Mechanism) -> str:
    """THERMO ALL section: four-line NASA-7 records in the fixed columns
    (coefficients to nine significant digits, as the format holds them)."""
    out = ["THERMO ALL", f"   {T_LOW:.3f}  {T_MID:.3f}  {T_HIGH:.3f}"]
    for s, comp in m.species:
        lo, hi = m.thermo[s]
        fields = "".join(f"{e:<2}{n:>3d}" for e, n in comp.items()).ljust(20)
        out.append(f"{s:<18}{'':6}{fields}G{T_LOW:10.3f}{T_HIGH:10.3f}{T_MID:8.2f}{'':6}1")
        out.append("".join(_e15(x) for x in hi[:5]) + "    2")
        out.append("".join(_e15(x) for x in list(hi[5:7]) + list(lo[:3])) + "    3")
        out.append("".join(_e15(x) for x in lo[3:7]) + " " * 15 + "    4")
    out.append("END")
    return "\n".join(out) + "\n"


def _ck_side(d, m_mark=""):
    return "+".join((f"{c}{s}" if c > 1 else s) for s, c in d.items()) + m_mark


def to_chemkin(m: Mechanism, inline_thermo=True) -> str:
    """The mechanism as a CHEMKIN file: energies in kJ/mol (KJOULES/MOLE),
    PLOG pressures in atm; thermo inline (THERMO ALL) or left to a separate
    file (thermo_chemkin)."""
    out = [f"! {m.name}: seeded synthetic mechanism", "ELEMENTS"]
    out.append(" ".join(f"{e}/{_fmt(ATOMIC_WEIGHTS[e])}/" for e in m.elements))
    out += ["END", "SPECIES", " ".join(s for s, _ in m.species), "END"]
    if inline_thermo:
        out.append(thermo_chemkin(m).rstrip("\n"))
    out.append("REACTIONS KJOULES/MOLE MOLES")
    for rx in m.reactions:
        mark = {"thirdbody": "+M", "troe": "(+M)", "lindemann": "(+M)", "sri": "(+M)"}.get(rx.kind, "")
        arrow = "=>" if rx.irrev else "<=>"
        A, b, Ea = (rx.plog[0][1:] if rx.kind == "plog" else (rx.A, rx.b, rx.Ea))
        out.append(f"{_ck_side(rx.reac, mark)}{arrow}{_ck_side(rx.prod, mark)}   {_fmt(A)} {_fmt(b)} {_fmt(Ea)}")
        if rx.kind in ("troe", "lindemann", "sri"):
            out.append("    LOW / " + " ".join(_fmt(x) for x in rx.low) + " /")
        if rx.kind == "troe":
            a, t3, t1, t2 = rx.troe
            out.append(f"    TROE / {_fmt(a)} {_fmt(t3)} {_fmt(t1)}" + ("" if t2 is None else f" {_fmt(t2)}") + " /")
        if rx.kind == "sri":
            out.append("    SRI / " + " ".join(_fmt(x) for x in rx.sri) + " /")
        if rx.kind == "plog":
            for p, Ap, bp, Ep in rx.plog:
                out.append(f"    PLOG / {_fmt(p / 101325.0)} {_fmt(Ap)} {_fmt(bp)} {_fmt(Ep)} /")
        if rx.kind not in ("elementary", "plog") and rx.eff:
            out.append("    " + " ".join(f"{s}/{_fmt(v)}/" for s, v in rx.eff.items()))
    out.append("END")
    return "\n".join(out) + "\n"


# --------------------------------------------------------------------------
# the same mechanisms as OpenFOAM chemistry dictionaries
# --------------------------------------------------------------------------

FOAM_TYPES = {"elementary": "Arrhenius", "thirdbody": "ThirdBodyArrhenius",
              "lindemann": "ArrheniusLindemannFallOff", "troe": "ArrheniusTroeFallOff",
              "sri": "ArrheniusSRIFallOff"}


def _foam_side(d):
    return " + ".join((f"{c}{s}" if c > 1 else s) for s, c in d.items())


def to_openfoam(m: Mechanism) -> tuple[str, str]:
    """(reactions, thermo) dictionary texts: A in (m^3/kmol)^(order-1)/s, Ta =
    Ea/R in K, molWeight in kg/kmol.  PLOG has no OpenFOAM form here."""
    names = [s for s, _ in m.species]
    out = ["FoamFile { version 2.0; format ascii; class dictionary; object reactions; }",
           f"elements {len(m.elements)} ( {' '.join(m.elements)} );",
           f"species {len(names)} ( {' '.join(names)} );", "reactions", "{"]

    def arr(indent, A, b, Ea, order):
        return [f"{indent}A {_fmt(A * 1e-3 ** (order - 1))};", f"{indent}beta {_fmt(b)};",
                f"{indent}Ta {_fmt(Ea * 1e3 / R_J)};"]

    for i, rx in enumerate(m.reactions):
        if rx.kind == "plog":
            raise ValueError("PLOG reactions have no OpenFOAM form")
        order = sum(rx.reac.values())
        kind = ("irreversible" if rx.irrev else "reversible") + FOAM_TYPES[rx.kind]
        out += [f"    un-named-reaction-{i}", "    {", f"        type {kind};",
                f'        reaction "{_foam_side(rx.reac)} = {_foam_side(rx.prod)}";']
        if rx.kind in ("elementary", "thirdbody"):
            out += arr("        ", rx.A, rx.b, rx.Ea, order + (rx.kind == "thirdbody"))
        else:
            A0, b0, Ea0 = rx.low
            out += ["        k0", "        {"] + arr("            ", A0, b0, Ea0, order + 1) + ["        }"]
            out += ["        kInf", "        {"] + arr("            ", rx.A, rx.b, rx.Ea, order) + ["        }"]
            out += ["        F", "        {"]
            if rx.kind == "troe":
                a, t3, t1, t2 = rx.troe
                out += [f"            alpha {_fmt(a)};", f"            Tsss {_fmt(t3)};", f"            Ts {_fmt(t1)};",
                        f"            Tss {_fmt(1e30 if t2 is None else t2)};"]
            elif rx.kind == "sri":
                out += [f"            {k} {_fmt(v)};" for k, v in zip("abcde", rx.sri)]
            out += ["        }"]
        if rx.kind != "elementary":
            coeffs = " ".join(f"({s} {_fmt(rx.eff.get(s, 1.0))})" for s in names)
            out += ["        thirdBodyEfficiencies", "        {", f"            coeffs {len(names)} ( {coeffs} );",
                    "        }"]
        out += ["    }"]
    out += ["}", f"Tlow {_fmt(T_LOW)};", f"Thigh {_fmt(T_HIGH)};"]
    th = ["FoamFile { version 2.0; format ascii; class dictionary; object thermo; }"]
    for s, comp in m.species:
        lo, hi = m.thermo[s]
        W = sum(ATOMIC_WEIGHTS[e] * n for e, n in comp.items())
        th += [s, "{", f"    specie {{ molWeight {_fmt(W)}; }}", "    thermodynamics", "    {",
               f"        Tlow {_fmt(T_LOW)};", f"        Thigh {_fmt(T_HIGH)};", f"        Tcommon {_fmt(T_MID)};",
               "        highCpCoeffs ( " + " ".join(_fmt(x) for x in hi) + " );",
               "        lowCpCoeffs ( " + " ".join(_fmt(x) for x in lo) + " );", "    }",
               "    transport { As 1.67212e-06; Ts 170.672; }",
               "    elements { " + " ".join(f"{e} {n};" for e, n in comp.items()) + " }", "}"]
    return "\n".join(out) + "\n", "\n".join(th) + "\n"


def build_mechanism(name: str) -> Mechanism:
    if name in VARIANTS:
        kw = dict(VARIANTS[name])
        base = kw.pop("base")
        return variant(generate(base, **MECHS[base]), name, **kw)
    return generate(name, **MECHS[name])


def format_doc() -> str:
    return """chemmi-mech 1 -- one record per line, '#' starts a comment
  name <id>
  element <symbol> <atomic weight g/mol>
  species <name> <element>=<count>[,<element>=<count>...] [W=<molar mass g/mol>]
      (without W the molar mass is the sum of the element weights)
  thermo <name> <Tlow> <Tmid> <Thigh> <a1..a7 for T<Tmid> <a1..a7 for T>=Tmid>
      NASA-7: cp/R = a1 + a2 T + a3 T^2 + a4 T^3 + a5 T^4,
              H/RT = a1 + a2 T/2 + a3 T^2/3 + a4 T^3/4 + a5 T^4/5 + a6/T,
              S/R  = a1 ln T + a2 T + a3 T^2/2 + a4 T^3/3 + a5 T^4/4 + a7
  reaction elementary <reac> <prod> A b Ea
  reaction thirdbody  <reac> <prod> A b Ea [eff=<sp>:<e>,...]
  reaction lindemann  <reac> <prod> A b Ea A0 b0 Ea0 [eff=...]
  reaction troe       <reac> <prod> A b Ea A0 b0 Ea0 alpha T3 T1 T2|- [eff=...]
  reaction sri        <reac> <prod> A b Ea A0 b0 Ea0 a b c d e [eff=...]
  reaction plog       <reac> <prod> A b Ea plog=<p>:<A>:<b>:<Ea>[,...]
      <reac>/<prod>: <species>=<nu>[,...].  A trailing 'irrev' drops the
      reverse reaction; otherwise it runs at k_f / K_c.
      A in cm-mol-s units of the reaction's order (+1 for third-body and for
      the low-pressure A0), Ea in kJ/mol; unlisted efficiencies are 1.
      SRI: F = d [a exp(-b/T) + exp(-T/c)]^X T^e, X = 1 / (1 + log10(P_r)^2).
      plog: pressures in Pa, increasing; ln k linear in ln p between them,
      the end rates outside; the main A (plain factor), b, Ea multiply it.
  end
"""


# The three mechanisms used by the workloads (seeds fixed here).
MECHS = {
    "m9": dict(species=SPECIES_H_O_N, n_reactions=21, seed=9001, inert=("N2",)),
    "m13": dict(species=SPECIES_H_O_N + SPECIES_EXTRA_13, n_reactions=27, seed=9002,
                n_troe=3, n_thirdbody=4, inert=tuple(INERT_SPECIES)),
    "m32": dict(species=SPECIES_H_O_N + SPECIES_EXTRA_13 + SPECIES_EXTRA_32,
                n_reactions=150, seed=9003, n_troe=15, inert=tuple(INERT_SPECIES)),
    # a mid-sized mechanism (above the one-cell-per-lane limit of 13 species)
    "m16": dict(species=SPECIES_H_O_N + SPECIES_EXTRA_13 + SPECIES_EXTRA_32[:3],
                n_reactions=48, seed=9016, n_troe=4, n_thirdbody=4, inert=tuple(INERT_SPECIES)),
}


# Variants that exercise every reaction form: some Troe reactions become SRI
# or Lindemann, some elementary ones pressure-tabulated, some irreversible.
VARIANTS = {
    "m13x": dict(base="m13", seed=9012, n_sri=1, n_lindemann=1, n_plog=4, n_irrev=6),
    "m32x": dict(base="m32", seed=9013, n_sri=5, n_lindemann=3, n_plog=12, n_irrev=30),
    # the same forms without PLOG, which OpenFOAM's dictionaries do not have
    "m32s": dict(base="m32", seed=9014, n_sri=5, n_lindemann=3, n_plog=0, n_irrev=30),
}

# PLOG pressure sets (atm): around, inside and outside the 1-30 atm of the fields
PLOG_PRESSURES = [(0.1, 1.0, 10.0, 100.0), (2.0, 5.0), (1.0,), (0.01, 0.3, 3.0, 8.0, 20.0, 300.0)]
P_ATM = 101325.0


def variant(m: Mechanism, name, seed, n_sri, n_lindemann, n_plog, n_irrev) -> Mechanism:
    rng = np.random.default_rng(seed)
    rx = [Reaction(**{k: getattr(r, k) for k in r.__dataclass_fields__}) for r in m.reactions]
    troe = [i for i, r in enumerate(rx) if r.kind == "troe"]
    for i in troe[:n_sri]:
        rx[i].kind, rx[i].troe = "sri", None
        rx[i].sri = (float(rng.uniform(0.3, 1.5)), float(rng.uniform(100.0, 1000.0)),
                     float(rng.uniform(200.0, 2000.0)), float(rng.uniform(0.8, 1.3)),
                     float(rng.uniform(-0.4, 0.4)))
    for i in troe[n_sri:n_sri + n_lindemann]:
        rx[i].kind, rx[i].troe = "lindemann", None
    elem = [i for i, r in enumerate(rx) if r.kind == "elementary"]
    for n, i in enumerate(rng.permutation(elem)[:n_plog]):
        r = rx[i]
        entries = []
        for p in PLOG_PRESSURES[n % len(PLOG_PRESSURES)]:
            entries.append((p * P_ATM, float(r.A * 10.0 ** rng.uniform(-0.7, 0.7)),
                            float(r.b + rng.uniform(-0.3, 0.3)), float(max(0.0, r.Ea + rng.uniform(-10.0, 10.0)))))
        r.kind, r.plog, r.A, r.b, r.Ea = "plog", entries, 1.0, 0.0, 0.0
    for i in rng.permutation(len(rx))[:n_irrev]:
        rx[i].irrev = True
    return Mechanism(name, m.elements, m.species, m.thermo, rx)


def build(name: str) -> str:
    return to_text(build_mechanism(name))


if __name__ == "__main__":
    import pathlib
    import sys
    outdir = pathlib.Path(__file__).parent / "mech"
    outdir.mkdir(exist_ok=True)
    for nm in (sys.argv[1:] or list(MECHS) + list(VARIANTS)):
        (outdir / f"{nm}.mech").write_text(build(nm))
        print("wrote", outdir / f"{nm}.mech")
