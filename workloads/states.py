"""Seeded synthetic thermochemical state fields (T, p, Y) for the workloads.

The paper's rotating-detonation-engine field (Sec. 3.2.1, Fig. 6-8) has a thin
detonation front with fresh premixed H2/air ahead of it and hot products (H2O
and N2) behind.  These generators draw fields with that structure and the
sizes of the workloads; no data from the paper is used.

Everything here is input preparation: mass fractions, temperatures and
pressures are drawn, never evolved.
"""
from __future__ import annotations

import math

import numpy as np

P_ATM = 101325.0
RADICALS = ("H2O", "H", "O", "OH", "HO2", "H2O2")
FRONT_RADICALS = ("H", "O", "OH", "HO2", "H2O2")
H_O_N = ("H2", "O2", "H2O", "H", "O", "OH", "HO2", "H2O2", "N2")
FRONT_ANGLE_DEG = 7.57          # front tilt measured in the paper (Sec. 3.2.3, Table 6)


def parse_species(mech_text: str):
    """(names, molar masses in g/mol) from a `chemmi-mech 1` text."""
    aw, names, w = {}, [], []
    for line in mech_text.splitlines():
        tok = line.split("#")[0].split()
        if not tok:
            continue
        if tok[0] == "element":
            aw[tok[1]] = float(tok[2])
        elif tok[0] == "species":
            names.append(tok[1])
            comp = dict(kv.split("=") for kv in tok[2].split(","))
            w.append(sum(aw[e] * int(n) for e, n in comp.items()))
    return names, np.array(w)


def _mix(names, wts, moles):
    """Mass fractions of a mixture given in moles per species name."""
    y = np.zeros(len(names))
    for s, n in moles.items():
        y[names.index(s)] = n * wts[names.index(s)]
    return y / y.sum()


def stoich_air(names, wts):
    """2 H2 + O2 + 3.76 N2."""
    return _mix(names, wts, {"H2": 2.0, "O2": 1.0, "N2": 3.76})


def products(names, wts):
    """Complete-combustion products 2 H2O + 3.76 N2 (the product gas of Sec. 3.2.1)."""
    return _mix(names, wts, {"H2O": 2.0, "N2": 3.76})


def _dirichlet_around(rng, names, mean, n, kappa=1000.0, floor=1e-4):
    """Dirichlet(kappa * m) over the H/O/N species, m = mean with a radical floor."""
    idx = [names.index(s) for s in H_O_N if s in names]
    m = mean[idx].copy()
    for j, i in enumerate(idx):
        if names[i] in RADICALS:
            m[j] = max(m[j], floor)
    m /= m.sum()
    y = np.zeros((n, len(names)))
    y[:, idx] = rng.dirichlet(kappa * m, size=n)
    return y


def uniform_cells(mech_text, n, seed):
    """Independent cells: T ~ U(300, 3000) K, p ~ log-U(1, 30) atm, Y Dirichlet
    (kappa = 1000) around stoichiometric H2-air with a 1e-4 radical floor."""
    names, wts = parse_species(mech_text)
    rng = np.random.default_rng(seed)
    T = rng.uniform(300.0, 3000.0, n)
    p = P_ATM * np.exp(rng.uniform(0.0, math.log(30.0), n))
    Y = _dirichlet_around(rng, names, stoich_air(names, wts), n)
    return T, p, Y


def region_masks(width, height, frac_front=0.05, frac_burnt=0.05):
    """Rank cells of a width x height grid (x fastest) by signed distance to a
    front line tilted by FRONT_ANGLE_DEG.  The cells farthest ahead are fresh;
    the band just behind the line is the front; the rest are burnt."""
    n = width * height
    a = math.radians(FRONT_ANGLE_DEG)
    y, x = np.divmod(np.arange(n), width)
    d = (x + 0.5) / width * math.cos(a) + (y + 0.5) / height * math.sin(a)
    order = np.argsort(-d, kind="stable")
    n_front = int(math.floor(frac_front * n + 0.5))
    n_burnt = int(math.floor(frac_burnt * n + 0.5))
    n_fresh = n - n_front - n_burnt
    region = np.empty(n, dtype=np.int8)                 # 0 fresh, 1 front, 2 burnt
    region[order[:n_fresh]] = 0
    region[order[n_fresh:n_fresh + n_front]] = 1
    region[order[n_fresh + n_front:]] = 2
    return region


def rde_field(mech_text, width, height, seed, shuffle=False):
    """RDE-shaped field: 90 % fresh stoichiometric H2-air at 300 K / 1 atm,
    5 % burnt products at 2500-3000 K / 10-20 atm, and a 5 % detonation-front
    band at 1500-3500 K / 15-30 atm with a seeded partially reacted mixture."""
    names, wts = parse_species(mech_text)
    rng = np.random.default_rng(seed)
    region = region_masks(width, height)
    n = width * height
    fresh_y = stoich_air(names, wts)
    T = np.empty(n)
    p = np.empty(n)
    Y = np.empty((n, len(names)))

    f = region == 0
    T[f] = 300.0
    p[f] = P_ATM
    Y[f] = fresh_y

    b = region == 2
    nb = int(b.sum())
    T[b] = rng.uniform(2500.0, 3000.0, nb)
    p[b] = P_ATM * rng.uniform(10.0, 20.0, nb)
    Y[b] = _dirichlet_around(rng, names, products(names, wts), nb)

    fr = region == 1
    nf = int(fr.sum())
    T[fr] = rng.uniform(1500.0, 3500.0, nf)
    p[fr] = P_ATM * rng.uniform(15.0, 30.0, nf)
    lam = rng.uniform(0.0, 1.0, (nf, 1))
    burnt = _dirichlet_around(rng, names, products(names, wts), nf)
    yf = (1.0 - lam) * fresh_y + lam * burnt
    for s in FRONT_RADICALS:
        if s in names:
            yf[:, names.index(s)] += np.exp(rng.uniform(math.log(1e-6), math.log(1e-2), nf))
    Y[fr] = yf / yf.sum(axis=1, keepdims=True)

    if shuffle:
        perm = rng.permutation(n)
        T, p, Y, region = T[perm], p[perm], Y[perm], region[perm]
    return T, p, np.ascontiguousarray(Y), region


def amr_field_sizes(seed, n_fields=64, lo=1e4, hi=2e6):
    """Field sizes drawn log-uniform in [lo, hi] (refinement-level-like counts)."""
    rng = np.random.default_rng(seed)
    return [int(math.floor(math.exp(rng.uniform(math.log(lo), math.log(hi)))))
            for _ in range(n_fields)]


def rde_field_n(mech_text, n, seed):
    """An RDE-shaped field of exactly n cells: the first n cells (row-major) of
    a square grid of width 2**ceil(log2(sqrt(n)))."""
    w = 1 << max(0, math.ceil(math.log2(math.sqrt(max(n, 1)))))
    h = max(1, -(-n // w))
    T, p, Y, reg = rde_field(mech_text, w, h, seed)
    return T[:n].copy(), p[:n].copy(), np.ascontiguousarray(Y[:n]), reg[:n].copy()
