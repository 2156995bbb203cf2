// math.hip -- device math used by the generated source terms.
//
// exp(x) by Tang's table-driven method (P. T. P. Tang, "Table-driven
// implementation of the exponential function in IEEE floating-point
// arithmetic", ACM TOMS 15(2), 1989), with 64 table entries:
//     x = (64 m + j) ln2/64 + r,  |r| <= ln2/128,
//     exp(x) = 2^m * 2^(j/64) * exp(r),
// exp(r) - 1 from its degree-5 Taylor polynomial (truncation below 4e-17 on
// that interval), 2^(j/64) from a table held in LDS.  The reduction
// r = x - n ln2/64 uses a two-part ln2/64 through fused multiply-adds.  No
// special-case branches: NaN propagates, arguments beyond the double range
// give 0 or inf through ldexp, +-inf give NaN (a failed step for the caller).
// The table values (2^(j/64) rounded to double) come with the generated code
// as EXP2_J64.

namespace chem_math {

__shared__ double exp2_j64[64];

// Copy the table into LDS.  Every thread of the workgroup must call this
// (it contains a barrier) before the first exp_tang.
__device__ __forceinline__ void exp_table_init(const double* __restrict__ src)
{
    for (int i = threadIdx.x; i < 64; i += blockDim.x) exp2_j64[i] = src[i];
    __syncthreads();
}

__device__ __forceinline__ double exp_tang(double x)
{
    constexpr double kInvL = 92.33248261689366;            // 64 / ln 2
    constexpr double kL1 = 0.010830424696249145;           // ln2/64, leading part
    constexpr double kL2 = 3.623510646634843e-19;          // ln2/64 - kL1
    const double nd = __builtin_rint(x * kInvL);
    const int n = (int)nd;
    double r = fma(-nd, kL1, x);
    r = fma(-nd, kL2, r);
    // p = exp(r) - 1; scalar constants enter as multiplicands or through a
    // separate add (an FMA with a scalar addend costs two extra moves)
    double q = r * (1.0 / 120.0);
    q = q + (1.0 / 24.0);
    q = q * r;
    q = q + (1.0 / 6.0);
    q = fma(r, q, 0.5);
    const double p = fma(r * r, q, r);
    const double s = exp2_j64[n & 63];
    return ldexp(fma(s, p, s), n >> 6);
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
__device__ __forceinline__ Dual exp_tang(Dual x)
{
    const double e = exp_tang(x.v);
    return {e, e * x.d};
}
__device__ __forceinline__ Dual exp(Dual x)
{
    const double e = ::exp(x.v);
    return {e, e * x.d};
}
__device__ __forceinline__ Dual log(Dual x) { return {::log(x.v), x.d / x.v}; }
__device__ __forceinline__ Dual log10(Dual x) { return {::log10(x.v), x.d / (x.v * 2.302585092994045684)}; }

}  // namespace chem_math
