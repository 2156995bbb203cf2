// math.hip -- device math used by the generated source terms.
//
// exp(x) without tables or branches (Cody & Waite argument reduction followed
// by a polynomial; W. J. Cody and W. Waite, "Software Manual for the
// Elementary Functions", 1980):
//     x = n ln2 + r,  n = rint(x / ln2),  |r| <= ln2/2,
//     exp(x) = 2^n * P(r),
// with ln2 split in two parts so r = x - n ln2 is exact to working precision
// through two fused multiply-adds, and P the degree-11 polynomial that
// interpolates exp at the 12 Chebyshev nodes of [-ln2/2, ln2/2] (computed in
// 40-digit arithmetic and rounded to double; interpolation error 3e-18,
// 1.5 ulp overall with Horner evaluation in double; printed by
// exp_poly_coeffs.py in the package directory).  No lookup table, so no LDS read
// whose latency a single wave per SIMD would have to wait out.  NaN
// propagates, arguments beyond the double range give 0 or inf through ldexp
// (the exponent's conversion to int saturates or is clamped), +-inf give NaN
// (a failed step for the caller).

namespace chem_math {

__device__ __forceinline__ double exp_poly(double x)
{
    constexpr double kLog2e = 1.4426950408889634;           // 1 / ln 2
    constexpr double kLn2Hi = 0.6931471805599453;           // ln 2 rounded to double
    constexpr double kLn2Lo = 2.3190468138462996e-17;       // ln 2 - kLn2Hi
    const double nd = __builtin_rint(x * kLog2e);
    // The exponent as an int.  A C++ conversion is undefined behaviour for NaN
    // and out-of-range values (LLVM turns it into poison, which the optimiser
    // may propagate anywhere), so either the hardware conversion, which is
    // defined for every input (beyond the int range INT_MIN or INT_MAX, NaN 0),
    // or a clamp to [-2100, 2100] first (two more instructions); either way
    // ldexp then gives 0 or inf where the result needs it, and a NaN x still
    // gives NaN through r.  The choice is the generator's (chem_config).
    int n;
    if constexpr (chem_config::kExpSaturatingConvert)
        asm("v_cvt_i32_f64 %0, %1" : "=v"(n) : "v"(nd));
    else
        n = (int)fmin(fmax(nd, -2100.0), 2100.0);
    double r = fma(-nd, kLn2Hi, x);
    r = fma(-nd, kLn2Lo, r);
    double q = fma(2.5110037605963777e-08, r, 2.763263963904103e-07);
    q = fma(q, r, 2.755724091857897e-06);
    q = fma(q, r, 2.4801485482328494e-05);
    q = fma(q, r, 0.00019841269890047113);
    q = fma(q, r, 0.0013888888952314775);
    q = fma(q, r, 0.008333333333319601);
    q = fma(q, r, 0.0416666666664881);
    q = fma(q, r, 0.1666666666666668);
    q = fma(q, r, 0.5000000000000019);
    q = fma(q, r, 1.0);
    q = fma(q, r, 1.0);
    return ldexp(q, n);
}

// 1/x: the hardware reciprocal estimate refined by two Newton steps
// (e = 1 - x r, r <- r + r e; each step doubles the correct bits), within an
// ulp of the quotient for normal x whose reciprocal is normal (0 and inf give
// NaN, which the integrator treats as a failed stage).
__device__ __forceinline__ double recip(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}

}  // namespace chem_math

// ---- forward-mode dual numbers (value, derivative along one direction) ----
// Used by the discrete adjoint for the second-order terms of a Rosenbrock
// step: D_u [J(y)^T w] and D_u [f_theta(y)^T w] come from evaluating the
// generated Jacobian and parameter products at y + eps u.
namespace chem_math {

struct Dual {
    double v, d;
    Dual() = default;
    __device__ constexpr Dual(double x) : v(x), d(0.0) {}
    __device__ constexpr Dual(double a, double b) : v(a), d(b) {}
};

__device__ __forceinline__ double value(double x) { return x; }
__device__ __forceinline__ double value(const Dual& x) { return x.v; }
__device__ __forceinline__ double tangent(double) { return 0.0; }
__device__ __forceinline__ double tangent(const Dual& x) { return x.d; }

__device__ __forceinline__ Dual operator+(Dual a, Dual b) { return {a.v + b.v, a.d + b.d}; }
__device__ __forceinline__ Dual operator+(Dual a, double b) { return {a.v + b, a.d}; }
__device__ __forceinline__ Dual operator+(double a, Dual b) { return {a + b.v, b.d}; }
__device__ __forceinline__ Dual operator-(Dual a, Dual b) { return {a.v - b.v, a.d - b.d}; }
__device__ __forceinline__ Dual operator-(Dual a, double b) { return {a.v - b, a.d}; }
__device__ __forceinline__ Dual operator-(double a, Dual b) { return {a - b.v, -b.d}; }
__device__ __forceinline__ Dual operator-(Dual a) { return {-a.v, -a.d}; }
__device__ __forceinline__ Dual operator*(Dual a, Dual b) { return {a.v * b.v, fma(a.d, b.v, a.v * b.d)}; }
__device__ __forceinline__ Dual operator*(Dual a, double b) { return {a.v * b, a.d * b}; }
__device__ __forceinline__ Dual operator*(double a, Dual b) { return {a * b.v, a * b.d}; }
__device__ __forceinline__ Dual operator/(Dual a, Dual b)
{
    const double q = a.v / b.v;
    return {q, (a.d - q * b.d) / b.v};
}
__device__ __forceinline__ Dual operator/(Dual a, double b) { return {a.v / b, a.d / b}; }
__device__ __forceinline__ Dual operator/(double a, Dual b)
{
    const double q = a / b.v;
    return {q, -q * b.d / b.v};
}
__device__ __forceinline__ Dual& operator+=(Dual& a, Dual b) { return a = a + b; }
__device__ __forceinline__ Dual& operator-=(Dual& a, Dual b) { return a = a - b; }
__device__ __forceinline__ Dual& operator*=(Dual& a, Dual b) { return a = a * b; }
__device__ __forceinline__ bool operator<(Dual a, double b) { return a.v < b; }
__device__ __forceinline__ bool operator>=(Dual a, double b) { return a.v >= b; }
__device__ __forceinline__ Dual fma(Dual a, Dual b, Dual c) { return {::fma(a.v, b.v, c.v), a.d * b.v + a.v * b.d + c.d}; }
__device__ __forceinline__ Dual fma(Dual a, double b, Dual c) { return {::fma(a.v, b, c.v), ::fma(a.d, b, c.d)}; }
__device__ __forceinline__ Dual fma(double a, Dual b, Dual c) { return {::fma(a, b.v, c.v), ::fma(a, b.d, c.d)}; }
__device__ __forceinline__ Dual fma(Dual a, Dual b, double c) { return {::fma(a.v, b.v, c), a.d * b.v + a.v * b.d}; }
__device__ __forceinline__ Dual fma(Dual a, double b, double c) { return {::fma(a.v, b, c), a.d * b}; }
__device__ __forceinline__ Dual fma(double a, Dual b, double c) { return {::fma(a, b.v, c), a * b.d}; }
__device__ __forceinline__ Dual fma(double a, double b, Dual c) { return {::fma(a, b, c.v), c.d}; }
__device__ __forceinline__ Dual exp_poly(Dual x)
{
    const double e = exp_poly(x.v);
    return {e, e * x.d};
}
__device__ __forceinline__ Dual exp(Dual x)
{
    const double e = ::exp(x.v);
    return {e, e * x.d};
}
__device__ __forceinline__ Dual recip(Dual x)
{
    const double r = recip(x.v);
    return {r, -(r * r) * x.d};
}
__device__ __forceinline__ Dual log(Dual x) { return {::log(x.v), x.d / x.v}; }
__device__ __forceinline__ Dual log10(Dual x) { return {::log10(x.v), x.d / (x.v * 2.302585092994045684)}; }

// Accumulate a parameter product: the value itself times sc (1, or 0 on the
// lanes of a lane group that only repeat its leader's first-order terms), or
// for a dual number its derivative along the evaluation's direction (the
// second-order term, whatever sc).
__device__ __forceinline__ void param_acc(double& a, double g, double sc) { a = ::fma(g, sc, a); }
__device__ __forceinline__ void param_acc(double& a, const Dual& g, double) { a += g.d; }

}  // namespace chem_math
