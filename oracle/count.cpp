/*
 * count.cpp -- counted mode of the oracle: the generic chemistry and Rosenbrock
 * step (chem_generic.inc) instantiated for a scalar that counts its own
 * arithmetic, so one RODAS4 step attempt reports how many additions,
 * multiplications, divisions and transcendentals the method performs
 * (source terms, analytic Jacobian, LU with partial pivoting, the six stages,
 * the solution and the error estimate).  Negation and comparisons are not
 * counted; an addition or multiplication with a constant is.
 *
 * TEST INFRASTRUCTURE ONLY (see oracle.h): used to check the per-substep
 * work that the roofline figures are based on.
 */
#include <cmath>
#include <cstring>

#include "oracle.h"
#include "oracle_internal.h"

namespace {

struct Counts {
    long add, mul, div, exp, log;
};
Counts g_counts;

struct Cnt {
    double v;
    Cnt() : v(0.0) {}
    Cnt(double x) : v(x) {}
};

inline Cnt operator+(Cnt a, Cnt b) { ++g_counts.add; return Cnt(a.v + b.v); }
inline Cnt operator-(Cnt a, Cnt b) { ++g_counts.add; return Cnt(a.v - b.v); }
inline Cnt operator*(Cnt a, Cnt b) { ++g_counts.mul; return Cnt(a.v * b.v); }
inline Cnt operator/(Cnt a, Cnt b) { ++g_counts.div; return Cnt(a.v / b.v); }
inline Cnt operator+(Cnt a, double b) { return a + Cnt(b); }
inline Cnt operator+(double a, Cnt b) { return Cnt(a) + b; }
inline Cnt operator-(Cnt a, double b) { return a - Cnt(b); }
inline Cnt operator-(double a, Cnt b) { return Cnt(a) - b; }
inline Cnt operator*(Cnt a, double b) { return a * Cnt(b); }
inline Cnt operator*(double a, Cnt b) { return Cnt(a) * b; }
inline Cnt operator/(Cnt a, double b) { return a / Cnt(b); }
inline Cnt operator/(double a, Cnt b) { return Cnt(a) / b; }
inline Cnt operator-(Cnt a) { return Cnt(-a.v); }
inline Cnt cnt_exp(Cnt a) { ++g_counts.exp; return Cnt(std::exp(a.v)); }
inline Cnt cnt_log(Cnt a) { ++g_counts.log; return Cnt(std::log(a.v)); }

#define S Cnt
#define F(name) name##_c
#define EXP cnt_exp
#define LOG cnt_log
#define RE(x) ((x).v)
#include "chem_generic.inc"
#undef S
#undef F
#undef EXP
#undef LOG
#undef RE

}  // namespace

/* One RODAS4 step attempt of size h from y (the mechanism's own parameters):
   out = {additions (incl. subtractions), multiplications, divisions, exp, log}.
   Returns 0, or -1 if the tableau is unavailable or the step matrix singular. */
extern "C" int om_count_step(const omech *m, double p, const double *y, double h, long *out)
{
    int s = 0;
    double gamma = 0.0, a[OM_SMAX * OM_SMAX], c[OM_SMAX * OM_SMAX], mw[OM_SMAX], e[OM_SMAX];
    if (om_tableau(OM_RODAS4, &s, &gamma, a, c, mw, e)) return -1;
    omtab t;
    std::memset(&t, 0, sizeof t);
    t.s = s;
    t.gamma = gamma;
    for (int i = 0; i < OM_SMAX; ++i) {
        for (int j = 0; j < OM_SMAX; ++j) {
            t.a[i][j] = a[i * OM_SMAX + j];
            t.c[i][j] = c[i * OM_SMAX + j];
        }
        t.m[i] = mw[i];
        t.e[i] = e[i];
    }
    const int n = m->ns + 1, np = 3 * m->nr;
    Cnt par[3 * OM_NRMAX], yc[OM_NMAX], yn[OM_NMAX], err[OM_NMAX];
    for (int j = 0; j < np; ++j) par[j] = Cnt(m->par[j]);
    for (int k = 0; k < n; ++k) yc[k] = Cnt(y[k]);
    g_counts = Counts{0, 0, 0, 0, 0};
    const int rc = ros_step_c(m, par, &t, p, yc, h, yn, err);
    out[0] = g_counts.add;
    out[1] = g_counts.mul;
    out[2] = g_counts.div;
    out[3] = g_counts.exp;
    out[4] = g_counts.log;
    return rc;
}
