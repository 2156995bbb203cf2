"""Coefficients of the device exp polynomial (csrc/device/math.hip, exp_poly).

exp(r) on [-ln2/2, ln2/2] by the degree-11 polynomial that interpolates it at
the 12 Chebyshev nodes of that interval, computed in 40-digit arithmetic and
rounded to double.  Prints the coefficients (highest degree first) and the
worst relative error over a dense grid, in exact arithmetic and with Horner
evaluation in double.  Needs mpmath; not used at run time.
"""
import mpmath as mp
import numpy as np


def coefficients(degree=11, digits=40):
    mp.mp.dps = digits
    a = mp.log(2) / 2
    poly, err = mp.chebyfit(mp.exp, [-a, a], degree + 1, error=True)
    return [float(c) for c in poly], float(err), float(a)


def main():
    coef, err, a = coefficients()
    r = np.linspace(-a, a, 400001)
    v = np.zeros_like(r)
    for c in coef:
        v = v * r + c
    ref = np.exp(r.astype(np.longdouble))
    horner = float(np.max(np.abs((v.astype(np.longdouble) - ref) / ref)))
    print("coefficients, highest degree first:")
    for c in coef:
        print(f"  {c!r}")
    print(f"interpolation error {err:.2e}; double Horner max relative error {horner:.2e}")


if __name__ == "__main__":
    main()
