"""The device exp (csrc/device/math.hip, exp_poly) on the host: its constants are
the ones the generator prints, and its sequence of operations, emulated here
with exactly rounded FMAs, stays within 2 ulp of exp over the double range
(checked against 30-digit exp) with the documented special values.  No GPU."""
import math
import pathlib
import re
from fractions import Fraction

import numpy as np
import pytest

ROOT = pathlib.Path(__file__).resolve().parents[1]
SRC = (ROOT / "paper_2508_16105_amd" / "csrc" / "device" / "math.hip").read_text()


def _body():
    i = SRC.index("double exp_poly(double x)")
    return SRC[i:SRC.index("\n}\n", i)]


def _constants():
    body = _body()
    named = {k: float(v) for k, v in re.findall(r"constexpr double (k\w+) = ([-+0-9.e]+);", body)}
    first = re.search(r"double q = fma\(([-+0-9.e]+), r, ([-+0-9.e]+)\);", body)
    rest = re.findall(r"q = fma\(q, r, ([-+0-9.e]+)\);", body)
    poly = [float(first.group(1)), float(first.group(2))] + [float(c) for c in rest]
    return named, poly


def _fma(a, b, c):
    if not all(math.isfinite(v) for v in (a, b, c)):
        return a * b + c
    return float(Fraction(a) * Fraction(b) + Fraction(c))


def _exp_poly(x, named, poly):
    """The device sequence: rint, the exponent converted to int as the
    hardware does (saturating at the int range, NaN to 0; the clamped
    conversion the generator may choose instead gives the same results),
    two-part reduction, Horner, ldexp."""
    nd = float(np.rint(x * named["kLog2e"]))
    n = 0 if math.isnan(nd) else int(min(max(nd, -2.0**31), 2.0**31 - 1))
    r = _fma(-nd, named["kLn2Hi"], x)
    r = _fma(-nd, named["kLn2Lo"], r)
    q = _fma(poly[0], r, poly[1])
    for c in poly[2:]:
        q = _fma(q, r, c)
    if math.isnan(q) or math.isinf(q):
        return q
    if n < -2000:
        return 0.0
    try:
        return math.ldexp(q, n)
    except OverflowError:                       # the device's ldexp gives inf
        return math.copysign(math.inf, q)


def test_constants_are_the_generator_output():
    mp = pytest.importorskip("mpmath")
    import sys
    sys.path.insert(0, str(ROOT / "paper_2508_16105_amd"))
    from exp_poly_coeffs import coefficients
    named, poly = _constants()
    want, err, _ = coefficients()
    assert poly == want and err < 1e-17
    mp.mp.dps = 40
    ln2 = mp.log(2)
    assert named["kLn2Hi"] == float(ln2)
    assert named["kLn2Lo"] == float(ln2 - mp.mpf(named["kLn2Hi"]))
    assert named["kLog2e"] == float(1 / ln2)


def test_emulated_accuracy_over_the_double_range():
    mp = pytest.importorskip("mpmath")
    mp.mp.dps = 30
    named, poly = _constants()
    rng = np.random.default_rng(11)
    xs = np.concatenate([rng.uniform(-745.0, 709.7, 1500), rng.uniform(-2.0, 2.0, 500),
                         [0.0, -0.0, 1e-300, -1e-300, 0.5 * math.log(2), -0.5 * math.log(2), 1.0, -1.0]])
    worst = 0.0
    for x in xs:
        got = _exp_poly(float(x), named, poly)
        ref = mp.exp(mp.mpf(float(x)))
        if ref < mp.mpf(2.0) ** -1022:          # subnormal results: absolute bound
            assert abs(mp.mpf(got) - ref) <= mp.mpf(2.0) ** -1073
            continue
        ulp = math.ulp(float(ref))
        worst = max(worst, float(abs(mp.mpf(got) - ref) / ulp))
    assert worst <= 2.0, worst


def test_special_values():
    named, poly = _constants()
    assert _exp_poly(0.0, named, poly) == 1.0
    assert _exp_poly(-800.0, named, poly) == 0.0
    assert _exp_poly(-1e5, named, poly) == 0.0
    assert _exp_poly(710.0, named, poly) == math.inf
    assert math.isnan(_exp_poly(math.nan, named, poly))
    assert math.isnan(_exp_poly(math.inf, named, poly))
    assert math.isnan(_exp_poly(-math.inf, named, poly))
