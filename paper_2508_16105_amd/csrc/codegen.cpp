// codegen.cpp -- emits the mechanism-specific device code (namespace mech):
// NASA-7 thermo, modified-Arrhenius forward rates, equilibrium-constant
// reverse rates, third-body and Lindemann/Troe falloff, the constant-pressure
// source terms (species production rates and heat release, Appendix A
// eqs. (20)-(21)) and their analytic Jacobian, all as straight-line code with
// compile-time species indices so each lane keeps its cell in registers.
//
// The Arrhenius parameters (ln A, b, Ea/R) are read from a device buffer so
// they can change without recompiling; every other constant is a literal.
#include "codegen.hpp"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <map>
#include <sstream>

namespace chemmi {
namespace {

std::string lit(double v)
{
    char buf[40];
    std::snprintf(buf, sizeof buf, "%.17g", v);
    std::string s(buf);
    if (s.find_first_of(".eEn") == std::string::npos) s += ".0";
    return s;
}

// C[k] written as a product term for stoichiometric coefficient nu
std::string powc(int k, int nu)
{
    std::string s = "C[" + std::to_string(k) + "]";
    std::string r = s;
    for (int i = 1; i < nu; ++i) r += "*" + s;
    return r;
}

// product of C^nu over a side, optionally skipping one occurrence of species `skip`
// (the derivative of C_m^nu is nu C_m^(nu-1))
std::string side_product(const std::vector<Term>& side, int dsp = -1)
{
    std::string r;
    bool hit = false;
    for (const auto& t : side) {
        int nu = t.nu;
        std::string factor;
        if (t.sp == dsp) {
            hit = true;
            if (nu > 1) factor = lit((double)nu) + (nu - 1 > 0 ? "*" + powc(t.sp, nu - 1) : "");
            else factor = "1.0";
        } else {
            factor = powc(t.sp, nu);
        }
        r += (r.empty() ? "" : "*") + factor;
    }
    if (dsp >= 0 && !hit) return "";
    return r.empty() ? "1.0" : r;
}

// G_k(T) = S_k/R - H_k/RT of species k from its NASA-7 set (host side, for
// the range checks of the generator)
double gibbs_of(const SpeciesData& sp, double T)
{
    const double* a = T < sp.tmid ? sp.lo : sp.hi;
    const double lnT = std::log(T);
    const double s = a[0] * lnT + a[1] * T + a[2] * T * T / 2 + a[3] * T * T * T / 3 + a[4] * T * T * T * T / 4 + a[6];
    const double h = a[0] + a[1] * T / 2 + a[2] * T * T / 3 + a[3] * T * T * T / 4 + a[4] * T * T * T * T / 5 +
                     a[5] / T;
    return s - h;
}

// The reverse rate k_r = k_f / K_c with 1/K_c as a product of per-species
// factors, e^{G_k} for each reactant and e^{-G_k} for each product (times
// (RT/P_atm)^dnu), so a reversible reaction costs a few multiplies instead of
// an exponential of its own (ln K_c = sum_k nu_k G_k + dnu ln(P_atm/RT), the
// standard-state equilibrium constant of the mass-action law).  The factors
// are multiplied reactant, product, reactant, ... ; a reaction keeps the
// exponential of ln k_f - ln K_c when some partial product would leave
// [e^-650, e^650] anywhere on 200 .. 6000 K.
struct SpeciesKc {
    std::vector<bool> product_form;   // per reaction
    std::vector<bool> need_gp, need_gm;   // per species: e^{G_k}, e^{-G_k}
    bool any_dnu = false;
};

std::vector<std::pair<int, int>> kc_factor_order(const ReactionData& r)
{
    // (species, +1 for e^{G}, -1 for e^{-G}), one entry per unit of nu, alternating sides
    std::vector<int> a, b;
    for (const auto& t : r.reac)
        for (int i = 0; i < t.nu; ++i) a.push_back(t.sp);
    for (const auto& t : r.prod)
        for (int i = 0; i < t.nu; ++i) b.push_back(t.sp);
    std::vector<std::pair<int, int>> out;
    for (size_t i = 0; i < std::max(a.size(), b.size()); ++i) {
        if (i < a.size()) out.push_back({a[i], +1});
        if (i < b.size()) out.push_back({b[i], -1});
    }
    return out;
}

SpeciesKc plan_species_kc(const MechanismData& m)
{
    SpeciesKc p;
    const int ns = m.ns(), nr = m.nr();
    p.product_form.assign(nr, false);
    p.need_gp.assign(ns, false);
    p.need_gm.assign(ns, false);
    std::vector<double> temps;
    for (double T = 200.0; T <= 6000.0; T += 5.0) temps.push_back(T);
    for (const auto& sp : m.species) {
        temps.push_back(sp.tmid);
        temps.push_back(std::nextafter(sp.tmid, 0.0));
    }
    const double lim = 650.0;
    for (int j = 0; j < nr; ++j) {
        const auto& r = m.reactions[j];
        if (!r.reversible) continue;
        const auto order = kc_factor_order(r);
        bool ok = true;
        for (double T : temps) {
            double acc = 0.0;
            for (const auto& f : order) {
                const double g = gibbs_of(m.species[f.first], T);
                if (std::fabs(g) > lim) ok = false;
                acc += f.second * g;
                if (std::fabs(acc) > lim) ok = false;
            }
            acc += r.dnu * std::log(kRu * T / kPatm);
            if (std::fabs(acc) > lim) ok = false;
            if (!ok) break;
        }
        p.product_form[j] = ok;
        if (!ok) continue;
        for (const auto& f : order) (f.second > 0 ? p.need_gp : p.need_gm)[f.first] = true;
        if (r.dnu != 0) p.any_dnu = true;
    }
    return p;
}

// c_1 e_1 + c_2 e_2 + ... as source text, led by its first term rather than
// by "0.0 +" (x + 0.0 is not x for x = -0.0, so a compiler must keep such an
// addition); "0.0" when there are no terms
std::string lin_sum(const std::vector<std::pair<double, std::string>>& terms)
{
    if (terms.empty()) return "0.0";
    std::string out;
    for (size_t i = 0; i < terms.size(); ++i) {
        const double c = terms[i].first;
        const std::string& e = terms[i].second;
        if (i == 0) out = c == 1.0 ? e : (c == -1.0 ? "-(" + e + ")" : lit(c) + "*" + e);
        else if (c == 1.0) out += " + " + e;
        else if (c == -1.0) out += " - " + e;
        else if (c < 0.0) out += " - " + lit(-c) + "*" + e;
        else out += " + " + lit(c) + "*" + e;
    }
    return out;
}

// Species no reaction produces or consumes (net coefficient zero in every
// reaction): their rows of the source terms and of the Jacobian are zero.
std::vector<bool> inert_species(const MechanismData& m)
{
    std::vector<bool> inert(m.ns(), true);
    for (const auto& r : m.reactions) {
        std::vector<int> nu(m.ns(), 0);
        for (const auto& t : r.reac) nu[t.sp] -= t.nu;
        for (const auto& t : r.prod) nu[t.sp] += t.nu;
        for (int k = 0; k < m.ns(); ++k)
            if (nu[k]) inert[k] = false;
    }
    return inert;
}

// Structural non-zeros of d wdot_k / d C_m: species k changed by a reaction
// whose rate depends on C_m (a reactant, a product of a reversible reaction,
// or a collision partner with non-zero efficiency).
std::vector<std::vector<bool>> jc_pattern(const MechanismData& m)
{
    const int ns = m.ns();
    std::vector<std::vector<bool>> nz(ns, std::vector<bool>(ns, false));
    for (const auto& r : m.reactions) {
        std::vector<int> nu(ns, 0);
        for (const auto& t : r.reac) nu[t.sp] -= t.nu;
        for (const auto& t : r.prod) nu[t.sp] += t.nu;
        std::vector<bool> dep(ns, false);
        for (const auto& t : r.reac) dep[t.sp] = true;
        if (r.reversible)
            for (const auto& t : r.prod) dep[t.sp] = true;
        if (r.kind == RxnKind::ThirdBody || is_falloff(r.kind))
            for (int k = 0; k < ns; ++k)
                if (r.eff[k] != 0.0) dep[k] = true;
        for (int k = 0; k < ns; ++k)
            if (nu[k])
                for (int mm = 0; mm < ns; ++mm)
                    if (dep[mm]) nz[k][mm] = true;
    }
    return nz;
}

struct Emitter {
    const MechanismData& m;
    std::ostringstream o;
    int ns, nr;
    SpeciesKc kc;
    std::vector<bool> inert;
    std::vector<std::vector<bool>> jnz;

    explicit Emitter(const MechanismData& mm)
        : m(mm), ns(mm.ns()), nr(mm.nr()), kc(plan_species_kc(mm)), inert(inert_species(mm)),
          jnz(jc_pattern(mm)) {}

    // NASA-7 coefficient table, per species and range (0: T < T_mid, 1: T >= T_mid):
    //  [0..4]  cp/R  = c0 + T(c1 + T(c2 + T(c3 + T c4)))          (a1..a5)
    //  [5..8]  H/RT  = c0 + T(c5 + T(c6 + T(c7 + T c8))) + c9/T    (a2/2, a3/3, a4/4, a5/5)
    //  [9]     a6
    //  [10..13] G = S/R - H/RT = c0 lnT + T(c10 + T(c11 + T(c12 + T c13))) + c14 - c9/T
    //           (a2/2, a3/6, a4/12, a5/20), [14] = a7 - a1
    //  [15..18] d(cp/R)/dT = c15 + T(c16 + T(c17 + T c18))            (a2, 2a3, 3a4, 4a5)
    void thermo_table()
    {
        // constant-address-space view: loads through it are scalar (uniform)
        o << "typedef const __attribute__((address_space(4))) double cdbl;\n"
             "// a zero the compiler cannot see through, known to be wave-uniform\n"
             "__device__ __forceinline__ int opaque_zero()\n{\n"
             "  int z;\n  asm volatile(\"s_mov_b32 %0, 0\" : \"=s\"(z));\n"
             "  return __builtin_amdgcn_readfirstlane(z);\n}\n";
        o << "// molar masses: W_k, 1/W_k, R/W_k\n__constant__ double MWTAB[3 * NS] = {";
        for (int t = 0; t < 3; ++t)
            for (int k = 0; k < ns; ++k) {
                const double W = m.species[k].W;
                o << lit(t == 0 ? W : (t == 1 ? 1.0 / W : kRu / W)) << ((t == 2 && k == ns - 1) ? "};\n" : ", ");
            }
        // species enthalpy at 298.15 K (J/kg, the NASA-7 set the kernels choose
        // there): the chemical enthalpy whose release the coupled energy equation sees
        o << "__constant__ double HF298[NS] = {";
        for (int k = 0; k < ns; ++k) {
            const auto& sp = m.species[k];
            const double T = 298.15;
            const double* a = T < sp.tmid ? sp.lo : sp.hi;
            const double hrt = a[0] + a[1] * T / 2 + a[2] * T * T / 3 + a[3] * T * T * T / 4 +
                               a[4] * T * T * T * T / 5 + a[5] / T;
            o << lit(kRu * T * hrt / sp.W) << (k + 1 < ns ? ", " : "};\n");
        }
        o << "__constant__ double THERMO_TMID[NS] = {";
        for (int k = 0; k < ns; ++k) o << lit(m.species[k].tmid) << (k + 1 < ns ? ", " : "};\n");
        o << "__constant__ double THERMO[NS][2][20] = {\n";
        for (int k = 0; k < ns; ++k) {
            o << "  {";
            for (int half = 0; half < 2; ++half) {
                const double* a = half == 0 ? m.species[k].lo : m.species[k].hi;
                const double c[20] = {a[0], a[1], a[2], a[3], a[4], a[1] / 2, a[2] / 3, a[3] / 4, a[4] / 5,
                                      a[5], a[1] / 2, a[2] / 6, a[3] / 12, a[4] / 20, a[6] - a[0],
                                      a[1], 2 * a[2], 3 * a[3], 4 * a[4], 0.0};
                o << "{";
                for (int i = 0; i < 20; ++i) o << lit(c[i]) << (i < 19 ? ", " : "");
                o << "}" << (half == 0 ? ", " : "");
            }
            o << "}" << (k + 1 < ns ? ",\n" : "\n");
        }
        o << "};\n\n";
    }

    // The NASA-7 polynomials at T from the table row c, as power sums over
    // T, T^2, T^3, T^4 (computed once per evaluation) so every step is a
    // multiply-accumulate with the scalar coefficient as a multiplicand (one
    // instruction; a scalar addend would cost two extra moves).
    void poly_body(const std::string& sfx, bool with_dcp)
    {
        o << "        { S a = T4 * c[4]; a = fma(T3, c[3], a); a = fma(T2, c[2], a); a = fma(T, c[1], a);\n"
             "          cpR" << sfx << " = a + c[0]; }\n"
             "        { S a = T4 * c[8]; a = fma(T3, c[7], a); a = fma(T2, c[6], a); a = fma(T, c[5], a);\n"
             "          a = fma(iT, c[9], a); HRT" << sfx << " = a + c[0]; }\n"
             "        { S a = T4 * c[13]; a = fma(T3, c[12], a); a = fma(T2, c[11], a); a = fma(T, c[10], a);\n"
             "          a = fma(lnT, c[0], a); a = fma(-iT, c[9], a); G" << sfx << " = a + c[14]; }\n";
        if (with_dcp)
            o << "        { S a = T3 * c[18]; a = fma(T2, c[17], a); a = fma(T, c[16], a); dcpR" << sfx
              << " = a + c[15]; }\n";
    }

    void thermo_one(const std::string& base, const std::string& sfx, bool with_dcp)
    {
        o << "        { cdbl* c = " << base << ";\n";
        poly_body(sfx, with_dcp);
        o << "        }\n";
    }

    void thermo(bool with_dcp)
    {
        // Group species by T_mid.  When every lane of the wave is on the same
        // side of T_mid the range index is wave-uniform and the coefficients
        // come in by scalar loads; a wave straddling T_mid evaluates both
        // ranges and selects per lane.
        std::vector<double> tmids;
        for (auto& s : m.species) {
            bool seen = false;
            for (double t : tmids) seen = seen || t == s.tmid;
            if (!seen) tmids.push_back(s.tmid);
        }
        for (double tm : tmids) {
            o << "  {\n    const bool below = T < " << lit(tm) << ";\n"
                 "    const bool all_lo = __all(below), all_hi = __all(!below);\n"
                 "    if (all_lo || all_hi) {\n"
                 "      const int r = all_lo ? 0 : 20;\n";
            for (int k = 0; k < ns; ++k) {
                if (m.species[k].tmid != tm) continue;
                const std::string idx = "[" + std::to_string(k) + "]";
                o << "      { cdbl* c = TH + " << k * 40 << " + r;\n";
                poly_body(idx, with_dcp);
                o << "      }\n";
            }
            o << "    } else {\n";
            for (int k = 0; k < ns; ++k) {
                if (m.species[k].tmid != tm) continue;
                const std::string idx = "[" + std::to_string(k) + "]";
                o << "      { S cpR_l, HRT_l, G_l, dcpR_l, cpR_h, HRT_h, G_h, dcpR_h;\n";
                thermo_one("TH + " + std::to_string(k * 40), "_l", with_dcp);
                thermo_one("TH + " + std::to_string(k * 40 + 20), "_h", with_dcp);
                o << "        cpR" << idx << " = below ? cpR_l : cpR_h;\n"
                     "        HRT" << idx << " = below ? HRT_l : HRT_h;\n"
                     "        G" << idx << " = below ? G_l : G_h;\n";
                if (with_dcp) o << "        dcpR" << idx << " = below ? dcpR_l : dcpR_h;\n";
                o << "      }\n";
            }
            o << "    }\n  }\n";
        }
    }

    // state common to rhs and rhs_jac
    void prologue(bool jac)
    {
        // The table and parameter addresses are offset by an opaque zero so the
        // scalar loads of the constants stay inside this evaluation instead of
        // being hoisted out of the substep loop (where ~300 live constants
        // would spill).
        o << "  const int z = opaque_zero();\n"
             "  cdbl* TH = (cdbl*)&THERMO[0][0][0] + z;\n"
             "  cdbl* P = (cdbl*)par + z;\n"
             "  cdbl* MW = (cdbl*)&MWTAB[0] + z;\n"
             "  const S T = y[0];\n"
             "  const S lnT = log(T);\n"
             "  const S iT = chem_math::recip(T);\n"
             "  const S T2 = T * T, T3 = T2 * T, T4 = T2 * T2;\n"
             "  S cpR[NS], HRT[NS], G[NS];\n";
        if (jac) o << "  S dcpR[NS];\n";
        thermo(jac);
        // per-species equilibrium factors e^{G_k}, e^{-G_k} (see SpeciesKc)
        for (int k = 0; k < ns; ++k) {
            if (kc.need_gp[k] || kc.need_gm[k])
                o << "  const S gp" << k << " = chem_math::exp_poly(G[" << k << "]);\n";
            if (kc.need_gm[k]) o << "  const S gm" << k << " = chem_math::recip(gp" << k << ");\n";
        }
        if (kc.any_dnu)
            o << "  const S rtp = T * " << lit(kRu / kPatm) << ";\n"
                 "  const S prt = iT * " << lit(kPatm / kRu) << ";\n";
        o << "  S sig = 0.0;\n";
        for (int k = 0; k < ns; ++k)
            o << "  sig = fma(y[" << 1 + k << "], MW[" << ns + k << "], sig);\n";
        // rho = p / (R T sig); 1/rho = R T sig / p with 1/p given
        o << "  const S Wbar = chem_math::recip(sig);\n"
             "  const S rho = p * Wbar * iT * " << lit(1.0 / kRu) << ";\n"
             "  const S irho = " << lit(kRu) << " * T * sig * ip;\n"
             "  const S ctot = p * iT * " << lit(1.0 / kRu) << ";\n"
             "  S C[NS];\n";
        for (int k = 0; k < ns; ++k)
            o << "  C[" << k << "] = rho * (y[" << 1 + k << "] * MW[" << ns + k << "]);\n";
        o << "  const S lnPRT = " << lit(std::log(kPatm / kRu)) << " - lnT;\n"
             "  S wd[NS];\n"
             "#pragma unroll\n  for (int k = 0; k < NS; ++k) wd[k] = 0.0;\n";
        for (const auto& r : m.reactions)
            if (r.kind == RxnKind::Plog) {
                o << "  const double lnp = log(p);\n";
                break;
            }
    }

    // PLOG: the Arrhenius set at this pressure (pla, plb, ple), linear in ln p
    // between the tabulated pressures and the end sets outside them, written
    // without branches: with w_i = clamp((ln p - ln p_i) / (ln p_i+1 - ln p_i),
    // 0, 1) the set is x_0 + sum_i w_i (x_i+1 - x_i), which telescopes to x_i +
    // w_i (x_i+1 - x_i) inside interval i and to the end sets outside.
    void plog_set(const ReactionData& r)
    {
        const auto& e = r.plog;
        o << "    double pla = " << lit(e[0].lnA) << ", plb = " << lit(e[0].b) << ", ple = " << lit(e[0].EaR)
          << ";\n";
        for (size_t i = 0; i + 1 < e.size(); ++i) {
            o << "    { const double w = fmin(1.0, fmax(0.0, (lnp - " << lit(e[i].lnp) << ") * "
              << lit(1.0 / (e[i + 1].lnp - e[i].lnp)) << "));\n"
                 "      pla = fma(w, " << lit(e[i + 1].lnA - e[i].lnA) << ", pla);\n"
                 "      plb = fma(w, " << lit(e[i + 1].b - e[i].b) << ", plb);\n"
                 "      ple = fma(w, " << lit(e[i + 1].EaR - e[i].EaR) << ", ple); }\n";
        }
    }

    std::string third_body_sum(const ReactionData& r)
    {
        std::string s = "ctot";
        for (int k = 0; k < ns; ++k)
            if (r.eff[k] != 1.0) s += " + " + lit(r.eff[k] - 1.0) + "*C[" + std::to_string(k) + "]";
        return s;
    }

    // mode 0: source terms; 1: source terms and Jacobian; 3: production rates,
    // the Jacobian-transpose product J^T w and the parameter products
    void reaction(int j, int mode)
    {
        const bool jtv = mode == 3;
        const bool jac = mode == 1 || jtv;
        const auto& r = m.reactions[j];
        o << "  { // reaction " << j << "\n";
        // ln k = ln A + b ln T - (Ea/R) / T, one scalar operand per instruction
        o << "    S lnk = lnT * P[" << nr + j << "];\n"
             "    lnk = fma(-iT, P[" << 2 * nr + j << "], lnk);\n"
             "    lnk = lnk + P[" << j << "];\n";
        const bool plog = r.kind == RxnKind::Plog, rev_on = r.reversible;
        if (plog) {
            plog_set(r);
            o << "    lnk = lnk + (lnT * plb - iT * ple + pla);\n";
        }
        const bool pform = rev_on && kc.product_form[j];
        if (pform) {
            // 1/K_c = prod_reac e^{G} prod_prod e^{-G} (RT/P_atm)^dnu
            std::string f;
            for (const auto& t : kc_factor_order(r))
                f += (f.empty() ? "" : " * ") + std::string(t.second > 0 ? "gp" : "gm") + std::to_string(t.first);
            for (int i = 0; i < std::abs(r.dnu); ++i) f += (f.empty() ? "" : " * ") + std::string(r.dnu > 0 ? "rtp" : "prt");
            o << "    const S ikc = " << (f.empty() ? std::string("1.0") : f) << ";\n";
        } else if (rev_on) {
            // ln K_c = sum nu (S/R - H/RT) + dnu ln(P_atm / RT)
            std::vector<std::pair<double, std::string>> lnkc;
            for (auto& t : r.prod) lnkc.push_back({(double)t.nu, "G[" + std::to_string(t.sp) + "]"});
            for (auto& t : r.reac) lnkc.push_back({-(double)t.nu, "G[" + std::to_string(t.sp) + "]"});
            if (r.dnu != 0) lnkc.push_back({(double)r.dnu, "lnPRT"});
            o << "    const S lnKc = " << lin_sum(lnkc) << ";\n";
        }
        const bool falloff = is_falloff(r.kind);
        if (r.kind != RxnKind::Elementary && !plog) o << "    const S Mc = " << third_body_sum(r) << ";\n";
        if (!falloff) {
            o << "    const S kf = chem_math::exp_poly(lnk);\n";
            if (pform) {
                if (jac) o << "    const S kr = kf * ikc;\n";
            } else if (rev_on) {
                o << "    const S kr = chem_math::exp_poly(lnk - lnKc);\n";
            }
        } else {
            // P_r = k0 [M] / k_inf, one exponential for the ratio
            o << "    const S kinf = chem_math::exp_poly(lnk);\n"
                 "    const S lnr0 = " << lit(r.lnA0) << " + " << lit(r.b0) << "*lnT - "
              << lit(r.EaR0) << "*iT - lnk;\n"
                 "    const S r0 = chem_math::exp_poly(lnr0);\n"
                 "    const S Pr = r0 * Mc;\n"
                 "    const bool floored = !(Pr >= 1e-300);\n"
                 "    const S logPr = floored ? -300.0 : log10(Pr);\n";
            if (r.kind == RxnKind::Troe) {
                o << "    const S e3 = exp(-T * " << lit(1.0 / r.T3) << ");\n"
                     "    const S e1 = exp(-T * " << lit(1.0 / r.T1) << ");\n";
                o << "    S Fc = " << lit(1.0 - r.alpha) << "*e3 + " << lit(r.alpha) << "*e1;\n";
                if (jac)
                    o << "    S dFc = " << lit(-(1.0 - r.alpha) / r.T3) << "*e3 + "
                      << lit(-r.alpha / r.T1) << "*e1;\n";
                if (r.has_T2) {
                    o << "    const S e2 = exp(" << lit(-r.T2) << " * iT);\n"
                         "    Fc += e2;\n";
                    if (jac) o << "    dFc += " << lit(r.T2) << "*iT*iT*e2;\n";
                }
                o << "    const S logFc = log10(Fc);\n"
                     "    const S tc = -0.4 - 0.67*logFc;\n"
                     "    const S tn = 0.75 - 1.27*logFc;\n"
                     "    const S tu = logPr + tc;\n"
                     "    const S tden = tn - 0.14*tu;\n"
                     "    const S tx = tu * chem_math::recip(tden);\n"
                     "    const S opx2 = 1.0 + tx*tx;\n"
                     "    const S logF = logFc * chem_math::recip(opx2);\n"
                     "    const S Fb = exp(" << lit(std::log(10.0)) << " * logF);\n";
                if (jac) {
                    o << "    const S tg = -logFc * 2.0 * tx / (opx2*opx2);\n"
                         "    const S dF_dPr = floored ? 0.0 : tg * tn / (tden*tden);\n"
                         "    const S dF_dFc = 1.0/opx2 + tg * (-0.67*tn + 1.27*tu) / (tden*tden);\n"
                         "    const S dlogFc_dT = dFc / (Fc * " << lit(std::log(10.0)) << ");\n";
                }
            } else if (r.kind == RxnKind::Sri) {
                // F = d [a exp(-b/T) + exp(-T/c)]^X T^e with X = 1 / (1 + log10(P_r)^2)
                const double* c = r.sri;
                o << "    const S sea = " << (c[0] != 0.0 ? lit(c[0]) + " * chem_math::exp_poly(" + lit(-c[1]) + " * iT)"
                                                         : std::string("0.0")) << ";\n"
                     "    const S sec = chem_math::exp_poly(-T * " << lit(1.0 / c[2]) << ");\n"
                     "    const S sY = sea + sec;\n"
                     "    const S lnsY = log(sY);\n"
                     "    const S sX = chem_math::recip(1.0 + logPr * logPr);\n"
                     "    const S Fb = chem_math::exp_poly(sX * lnsY + " << lit(c[4]) << " * lnT + " << lit(std::log(c[3]))
                  << ");\n";
                if (jac)
                    o << "    const S dF_dPr = floored ? 0.0 : lnsY * " << lit(-2.0 / std::log(10.0))
                      << " * logPr * sX * sX;\n"
                         "    const S dF_dFc = 0.0, dlogFc_dT = 0.0;\n"
                         "    const S dlnF_T = sX * (sea * " << lit(c[1]) << " * iT * iT - sec * " << lit(1.0 / c[2])
                      << ") / sY + " << lit(c[4]) << " * iT;\n";
            } else {
                o << "    const S Fb = 1.0;\n";
                if (jac) o << "    const S dF_dPr = 0.0, dF_dFc = 0.0, dlogFc_dT = 0.0;\n";
            }
            o << "    const S ipr1 = chem_math::recip(1.0 + Pr);\n"
                 "    const S kf = kinf * Pr * ipr1 * Fb;\n";
            if (pform) {
                if (jac)
                    o << "    const S iKc = ikc;\n"
                         "    const S kr = kf * iKc;\n";
            } else if (rev_on)
                o << "    const S iKc = chem_math::exp_poly(-lnKc);\n"
                     "    const S kr = kf * iKc;\n";
        }
        if (pform && !jac) {
            // source terms alone: q = k_f (prod_reac C - prod_prod C / K_c),
            // one rounding for the difference
            o << "    const S pf = " << side_product(r.reac) << ";\n"
                 "    const S pr = " << side_product(r.prod) << ";\n"
                 "    const S q = " << (r.kind == RxnKind::ThirdBody ? "Mc * " : "") << "(kf * fma(-ikc, pr, pf));\n";
        } else if (rev_on)
            o << "    const S pf = " << side_product(r.reac) << ";\n"
                 "    const S pr = " << side_product(r.prod) << ";\n"
                 "    const S fwd = kf * pf;\n"
                 "    const S rev = kr * pr;\n";
        else
            o << "    const S pf = " << side_product(r.reac) << ";\n"
                 "    const S fwd = kf * pf;\n";
        const std::string net = rev_on ? "(fwd - rev)" : "fwd";
        if (!(pform && !jac)) {
            if (r.kind == RxnKind::ThirdBody) o << "    const S q = Mc * " << net << ";\n";
            else o << "    const S q = " << (rev_on ? "fwd - rev" : "fwd") << ";\n";
        }
        // production rates
        std::vector<int> nu(ns, 0);
        for (auto& t : r.reac) nu[t.sp] -= t.nu;
        for (auto& t : r.prod) nu[t.sp] += t.nu;
        for (int k = 0; k < ns; ++k)
            if (nu[k]) o << "    wd[" << k << "] = fma(" << lit(nu[k]) << ", q, wd[" << k << "]);\n";
        if (jac) {
            // d ln k_f / dT at fixed [M]; d ln K_c / dT = (sum nu H/RT - dnu) / T
            std::vector<std::pair<double, std::string>> sh;
            for (auto& t : r.prod) sh.push_back({(double)t.nu, "HRT[" + std::to_string(t.sp) + "]"});
            for (auto& t : r.reac) sh.push_back({-(double)t.nu, "HRT[" + std::to_string(t.sp) + "]"});
            if (rev_on)
                o << "    const S dlnKc = (" << lin_sum(sh)
                  << (r.dnu != 0 ? " - " + lit(r.dnu) : std::string()) << ") * iT;\n";
            if (plog)
                o << "    const S dlnkinf = (P[" << nr + j << "] + plb + (P[" << 2 * nr + j << "] + ple)*iT) * iT;\n";
            else
                o << "    const S dlnkinf = (P[" << nr + j << "] + P[" << 2 * nr + j << "]*iT) * iT;\n";
            if (!falloff) {
                o << "    const S dlnkf = dlnkinf;\n";
            } else {
                o << "    const S dlnk0 = (" << lit(r.b0) << " + " << lit(r.EaR0) << "*iT) * iT;\n"
                     "    const S dlnkf = dlnkinf + (ipr1 + dF_dPr) * (dlnk0 - dlnkinf) + ";
                if (r.kind == RxnKind::Sri) o << "dlnF_T;\n";
                else o << lit(std::log(10.0)) << " * dF_dFc * dlogFc_dT;\n";
                o << "    const S dkdM = kinf * r0 * Fb * (ipr1*ipr1 + dF_dPr*ipr1);\n";
            }
            std::string fac = r.kind == RxnKind::ThirdBody ? "Mc * " : "";
            if (rev_on) o << "    const S dqT = " << fac << "(dlnkf * fwd - (dlnkf - dlnKc) * rev);\n";
            else o << "    const S dqT = " << fac << "(dlnkf * fwd);\n";
            // d q / d C_m (dense over the species that enter)
            std::vector<std::string> dq(ns);
            for (int mm = 0; mm < ns; ++mm) {
                std::string t;
                std::string a = side_product(r.reac, mm);
                std::string b = rev_on ? side_product(r.prod, mm) : std::string();
                if (!a.empty()) t += "kf*(" + a + ")";
                if (!b.empty()) t += (t.empty() ? "-" : " - ") + std::string("kr*(") + b + ")";
                if (!t.empty() && r.kind == RxnKind::ThirdBody) t = "Mc*(" + t + ")";
                if (r.kind == RxnKind::ThirdBody && r.eff[mm] != 0.0)
                    t += (t.empty() ? "" : " + ") + lit(r.eff[mm]) + "*" + net;
                if (falloff && r.eff[mm] != 0.0)
                    t += (t.empty() ? "" : " + ") + lit(r.eff[mm]) + "*dMterm";
                dq[mm] = t;
            }
            // k_r = k_f / K_c, so both directions scale with d k_f / d[M]
            if (falloff) o << "    const S dMterm = dkdM*" << (rev_on ? "(pf - iKc*pr)" : "pf") << ";\n";
            for (int mm = 0; mm < ns; ++mm)
                if (!dq[mm].empty()) o << "    const S dq" << mm << " = " << dq[mm] << ";\n";
            if (jtv) {
                // weights of this reaction's rate in w . f (species rows) and in the
                // heat release: wY = sum_k nu_k W_k w_{1+k}, hs = sum_k nu_k H_k/RT;
                // the columns of J^T w collect wY dq_m and hs dq_m; s = sum_m dq_m C_m
                std::vector<std::pair<double, std::string>> ws, hsum, sj;
                for (int k = 0; k < ns; ++k)
                    if (nu[k]) ws.push_back({(double)nu[k], "(MW[" + std::to_string(k) + "]*w[" + std::to_string(1 + k) + "])"});
                for (int k = 0; k < ns; ++k)
                    if (nu[k]) hsum.push_back({(double)nu[k], "HRT[" + std::to_string(k) + "]"});
                for (int mm = 0; mm < ns; ++mm)
                    if (!dq[mm].empty()) sj.push_back({1.0, "dq" + std::to_string(mm) + "*C[" + std::to_string(mm) + "]"});
                o << "    const S wY = " << lin_sum(ws) << ";\n"
                     "    const S hs = " << lin_sum(hsum) << ";\n"
                     "    const S sj = " << lin_sum(sj) << ";\n";
                for (int mm = 0; mm < ns; ++mm)
                    if (!dq[mm].empty())
                        o << "    colA[" << mm << "] = fma(wY, dq" << mm << ", colA[" << mm << "]); colH[" << mm
                          << "] = fma(hs, dq" << mm << ", colH[" << mm << "]);\n";
                o << "    SwY = fma(wY, sj, SwY); HSa = fma(hs, sj, HSa);\n"
                     "    wYT = fma(wY, dqT, wYT); HwT = fma(hs, dqT, HwT);\n";
                // parameter products w . df/dq_j times d q_j / d(ln A, b, Ea)
                o << "    const S wsum = wY * irho - w[0] * (" << lit(kRu) << " * T) * hs * rcpinv;\n";
                if (falloff) o << "    const S qA = q * (Pr * ipr1 - dF_dPr);\n";
                else o << "    const S qA = q;\n";
                o << "    const S g = wsum * qA;\n"
                     "    chem_math::param_acc(gA[" << j << " * GS], g, gsc);\n"
                     "    chem_math::param_acc(gb[" << j << " * GS], g * lnT, gsc);\n"
                     "    chem_math::param_acc(gE[" << j << " * GS], g * (-iT * " << lit(1.0 / kRu) << "), gsc);\n  }\n";
                return;
            }
            for (int k = 0; k < ns; ++k) {
                if (!nu[k]) continue;
                for (int mm = 0; mm < ns; ++mm)
                    if (!dq[mm].empty())
                        o << "    J[" << 1 + k << "][" << 1 + mm << "] = fma(" << lit(nu[k]) << ", dq" << mm
                          << ", J[" << 1 + k << "][" << 1 + mm << "]);\n";
                o << "    J[" << 1 + k << "][0] = fma(" << lit(nu[k]) << ", dqT, J[" << 1 + k << "][0]);\n";
            }
        }
        o << "  }\n";
    }

    void rhs_tail()
    {
        // 1/(rho cp) = T sig / (p cpm)
        o << "  const S icpm = chem_math::recip(cpm);\n"
             "  const S rcpinv = T * sig * ip * icpm;\n";
        // (species no reaction changes have wdot = 0: no terms, zero rows)
        o << "  S hw = 0.0;\n";
        for (int k = 0; k < ns; ++k)
            if (!inert[k]) o << "  hw = fma(HRT[" << k << "], wd[" << k << "], hw);\n";
        for (int k = 0; k < ns; ++k) {
            if (inert[k]) o << "  f[" << 1 + k << "] = 0.0;\n";
            else o << "  f[" << 1 + k << "] = MW[" << k << "] * (irho * wd[" << k << "]);\n";
        }
        o << "  f[0] = -" << lit(kRu) << " * T * hw * rcpinv;\n";
    }

    void cp_sum(bool jac)
    {
        o << "  S cpm = 0.0;\n";
        for (int k = 0; k < ns; ++k)
            o << "  cpm = fma(cpR[" << k << "], y[" << 1 + k << "] * MW[" << ns + k << "], cpm);\n";
        o << "  const S cp = " << lit(kRu) << " * cpm;\n";
        if (jac) {
            o << "  S dcpm = 0.0;\n";
            for (int k = 0; k < ns; ++k)
                o << "  dcpm = fma(dcpR[" << k << "], y[" << 1 + k << "] * MW[" << ns + k << "], dcpm);\n";
            o << "  const S dcp = " << lit(kRu) << " * dcpm;\n";
        }
    }

    void chain_rule()
    {
        // J holds Jc_km = d wdot_k / d C_m (at fixed T) in its species block and
        // wT_k = d wdot_k / dT (at fixed C) in column 0 of the species rows.
        // With S_k = sum_l Jc_kl C_l:
        //   J_km = (W_k/W_m) Jc_km + (Wbar/W_m)(f_k - W_k S_k / rho)
        //   J_k0 = (W_k / rho)(wT_k - S_k / T) + f_k / T
        //   J_0m = -R T (rho HJ_m - Wbar HS) / (W_m rho cp) - f_T (cp_m / cp - Wbar / W_m)
        //   J_00 = -R (cpw + T HwT - HS) / (rho cp) - f_T (dcp / cp - 1/T)
        // where HJ_m = sum_k H_k/RT Jc_km, HS = sum_k H_k/RT S_k, HwT = sum_k H_k/RT wT_k,
        // cpw = sum_k cp_k/R wdot_k.
        // (sums run over the structural non-zeros of Jc only: a literal zero
        // times a value is not folded away by the compiler, as the value could
        // be infinite; rows of species no reaction changes are zero)
        o << "  S Sk[NS];\n";
        for (int k = 0; k < ns; ++k) {
            std::vector<std::pair<double, std::string>> t;
            for (int l = 0; l < ns; ++l)
                if (jnz[k][l])
                    t.push_back({1.0, "J[" + std::to_string(1 + k) + "][" + std::to_string(1 + l) + "]*C[" + std::to_string(l) + "]"});
            o << "  Sk[" << k << "] = " << lin_sum(t) << ";\n";
        }
        o << "  S HS = 0.0, HwT = 0.0, cpw = 0.0;\n";
        for (int k = 0; k < ns; ++k)
            if (!inert[k])
                o << "  HS = fma(HRT[" << k << "], Sk[" << k << "], HS); HwT = fma(HRT[" << k << "], J[" << 1 + k
                  << "][0], HwT); cpw = fma(cpR[" << k << "], wd[" << k << "], cpw);\n";
        o << "  const S fT = f[0];\n"
             "  const S RT = " << lit(kRu) << " * T;\n"
             "  const S icp = icpm * " << lit(1.0 / kRu) << ";\n";
        for (int mm = 0; mm < ns; ++mm) {
            std::vector<std::pair<double, std::string>> hj;
            for (int k = 0; k < ns; ++k)
                if (jnz[k][mm])
                    hj.push_back({1.0, "HRT[" + std::to_string(k) + "]*J[" + std::to_string(1 + k) + "][" + std::to_string(1 + mm) + "]"});
            o << "  { S HJ = " << lin_sum(hj) << ";\n"
                 "    S t = fma(rho, HJ, -Wbar*HS) * (-RT * rcpinv);\n"
                 "    S u = fma(cpR[" << mm << "], icp * " << lit(kRu) << ", -Wbar);\n"
                 "    J[0][" << 1 + mm << "] = fma(-fT, u, t) * MW[" << ns + mm << "]; }\n";
        }
        o << "  J[0][0] = -" << lit(kRu) << " * (cpw + T*HwT - HS) * rcpinv - fT * (dcp * icp - iT);\n";
        for (int k = 0; k < ns; ++k) {
            if (inert[k]) continue;   // a zero row
            // J_km = (1/W_m)(W_k Jc_km + Wbar g_k), g_k = f_k - W_k S_k / rho
            o << "  { const S g = fma(-MW[" << k << "], Sk[" << k << "] * irho, f[" << 1 + k << "]);\n"
                 "    const S wg = Wbar * g;\n";
            for (int mm = 0; mm < ns; ++mm)
                o << "    J[" << 1 + k << "][" << 1 + mm << "] = fma(J[" << 1 + k << "][" << 1 + mm << "], MW[" << k
                  << "], wg) * MW[" << ns + mm << "];\n";
            o << "    J[" << 1 + k << "][0] = fma(MW[" << k << "] * irho, J[" << 1 + k << "][0] - Sk[" << k
              << "] * iT, f[" << 1 + k << "] * iT); }\n";
        }
    }

    std::string run()
    {
        o << "// generated mechanism code: " << m.name << " (" << ns << " species, " << nr << " reactions)\n"
          << "namespace mech {\n"
          << "constexpr int NS = " << ns << ";\n"
          << "constexpr int NR = " << nr << ";\n"
          << "constexpr int N = NS + 1;\n"
          << "constexpr double RU = " << lit(kRu) << ";\n";
        // elimination order of the step matrix: T and the species some reaction
        // changes first, then the species no reaction changes, whose rows of
        // M = I/(gamma h) - J are the diagonal alone
        {
            std::vector<int> perm{0};
            for (int k = 0; k < ns; ++k)
                if (!inert[k]) perm.push_back(1 + k);
            const int nact = (int)perm.size();
            for (int k = 0; k < ns; ++k)
                if (inert[k]) perm.push_back(1 + k);
            o << "constexpr int NACT = " << nact << ";   // components with a non-trivial row\n"
              << "constexpr int PERM[N] = {";
            for (int i = 0; i <= ns; ++i) o << perm[i] << (i < ns ? ", " : "};\n\n");
        }
        // source terms only
        thermo_table();
        o << "template <class S>\n__device__ __forceinline__ void rhs(const double* __restrict__ par, double p, "
             "double ip, const S (&y)[N], S (&f)[N])\n{\n";
        prologue(false);
        for (int j = 0; j < nr; ++j) reaction(j, 0);
        cp_sum(false);
        rhs_tail();
        o << "}\n\n";
        // source terms and Jacobian
        o << "template <class S>\n__device__ __forceinline__ void rhs_jac(const double* __restrict__ par, double p, "
             "double ip, const S (&y)[N], S (&f)[N], S (&J)[N][N])\n{\n";
        o << "#pragma unroll\n  for (int i = 0; i < N; ++i)\n#pragma unroll\n    for (int j = 0; j < N; ++j) J[i][j] = 0.0;\n";
        prologue(true);
        for (int j = 0; j < nr; ++j) reaction(j, 1);
        cp_sum(true);
        rhs_tail();
        chain_rule();
        o << "}\n\n";
        // v = J(y)^T w and the parameter products in one pass, without forming J:
        // every entry of J is assembled from per-reaction partials, so J^T w
        // needs only per-reaction weights and two column sums (see chain_rule):
        //   v_{1+m} = (colA_m + Wbar (w.f_Y - SwY/rho)) / W_m + w_0 J_{0,1+m}
        //   v_0     = (wYT - SwY/T)/rho + (w.f_Y)/T + w_0 J_00
        // with colA_m = sum_j wY_j dq_j/dC_m, colH_m = sum_j hs_j dq_j/dC_m (= HJ_m),
        // SwY = sum_j wY_j s_j, HS = sum_j hs_j s_j, wYT = sum_j wY_j dq_j/dT,
        // HwT = sum_j hs_j dq_j/dT, s_j = sum_m dq_j/dC_m C_m.
        // (the parameter products go to double accumulators, scaled by gsc; for
        // a dual S only their tangent is added, see chem_math::param_acc; GS is
        // the accumulators' element stride)
        o << "template <class S, int GS = 1>\n__device__ __forceinline__ void jtv_param(const double* __restrict__ par, double p, "
             "double ip, const S (&y)[N], const double (&w)[N], S (&v)[N], double* __restrict__ gA, "
             "double* __restrict__ gb, double* __restrict__ gE, double gsc)\n{\n";
        prologue(true);
        cp_sum(true);
        o << "  const S icpm = chem_math::recip(cpm);\n"
             "  const S rcpinv = T * sig * ip * icpm;\n"
             "  S colA[NS], colH[NS];\n"
             "#pragma unroll\n  for (int k = 0; k < NS; ++k) { colA[k] = 0.0; colH[k] = 0.0; }\n"
             "  S SwY = 0.0, HSa = 0.0, wYT = 0.0, HwT = 0.0;\n";
        for (int j = 0; j < nr; ++j) reaction(j, 3);
        o << "  S hw = 0.0, Wf = 0.0, cpw = 0.0;\n";
        for (int k = 0; k < ns; ++k)
            if (!inert[k])
                o << "  hw = fma(HRT[" << k << "], wd[" << k << "], hw); cpw = fma(cpR[" << k << "], wd[" << k
                  << "], cpw); Wf = fma(w[" << 1 + k << "], MW[" << k << "] * (irho * wd[" << k << "]), Wf);\n";
        o << "  const S fT = -" << lit(kRu) << " * T * hw * rcpinv;\n"
             "  const S RT = " << lit(kRu) << " * T;\n"
             "  const S icp = icpm * " << lit(1.0 / kRu) << ";\n"
             "  const S SwYg = Wf - irho * SwY;\n"
             "  const S wg = Wbar * SwYg;\n";
        for (int mm = 0; mm < ns; ++mm)
            o << "  { S t = fma(rho, colH[" << mm << "], -Wbar*HSa) * (-RT * rcpinv);\n"
                 "    S u = fma(cpR[" << mm << "], icp * " << lit(kRu) << ", -Wbar);\n"
                 "    const S J0m = fma(-fT, u, t) * MW[" << ns + mm << "];\n"
                 "    v[" << 1 + mm << "] = fma(colA[" << mm << "] + wg, MW[" << ns + mm << "], w[0] * J0m); }\n";
        o << "  const S J00 = -" << lit(kRu) << " * (cpw + T*HwT - HSa) * rcpinv - fT * (dcp * icp - iT);\n"
             "  v[0] = fma(irho, wYT - SwY * iT, fma(iT, Wf, w[0] * J00));\n";
        o << "}\n\n}  // namespace mech\n";
        return o.str();
    }
};

}  // namespace

std::string generate_mechanism_source(const MechanismData& m) { return Emitter(m).run(); }

WideLayout wide_layout(const MechanismData& m)
{
    WideLayout w;
    const int ns = m.ns(), nr = m.nr(), n = ns + 1;
    if (n > 64) {
        w.G = 0;
        return w;
    }
    w.G = 16;
    while (w.G < n) w.G *= 2;
    w.maxt = 1;
    for (const auto& r : m.reactions) w.maxt = std::max<int>(w.maxt, (int)std::max(r.reac.size(), r.prod.size()));
    if (w.maxt > 3) {
        w.G = 0;
        return w;
    }
    for (const auto& r : m.reactions) {   // the packed reaction table's field widths
        for (const auto* side : {&r.reac, &r.prod})
            for (const auto& t : *side)
                if (t.nu > 3) w.G = 0;
        if (r.dnu < -4 || r.dnu > 3) w.G = 0;
    }
    int n_eff = 0, n_plog = 0;
    for (const auto& r : m.reactions) {
        if (r.kind == RxnKind::Plog) ++n_plog;
        else if (r.kind != RxnKind::Elementary) ++n_eff;
    }
    if (n_eff > 511 || n_plog > 511 || nr > 65535 || w.G == 0) {
        w.G = 0;
        return w;
    }
    w.nslot = 2 * w.maxt;
    w.pw = w.nslot + 2;
    w.jw = (ns + 1) % 2 ? ns + 1 : ns + 2;
    w.l_y = 0;
    w.l_c = w.l_y + n;
    w.l_g = w.l_c + ns;
    w.l_h = w.l_g + ns;
    w.l_q = w.l_h + ns;
    w.l_p = w.l_q + nr;
    w.l_j = w.l_p + nr * w.pw;
    w.l_t0 = w.l_j + ns * w.jw;
    w.l_w = w.l_t0 + ns;
    w.lds_cell = w.l_w + n;
    w.adj_lds_cell = 2 * w.lds_cell + 2 * n;
    return w;
}

std::string generate_wide_source(const MechanismData& m, const WideLayout& w)
{
    Emitter e(m);
    std::ostringstream& o = e.o;
    const int ns = m.ns(), nr = m.nr();
    o << "// generated mechanism tables (wave-cooperative form): " << m.name << " (" << ns << " species, " << nr
      << " reactions)\n"
      << "namespace mech {\n"
      << "constexpr int NS = " << ns << ";\n"
      << "constexpr int NR = " << nr << ";\n"
      << "constexpr int N = NS + 1;\n"
      << "constexpr int G = " << w.G << ";            // lanes per cell\n"
      << "constexpr int MAXT = " << w.maxt << ";         // most terms on a reaction side\n"
      << "constexpr int NSLOT = " << w.nslot << ", PW = " << w.pw << ", JW = " << w.jw << ";\n"
      << "constexpr int L_Y = " << w.l_y << ", L_C = " << w.l_c << ", L_G = " << w.l_g << ", L_H = " << w.l_h
      << ", L_Q = " << w.l_q << ", L_P = " << w.l_p << ", L_J = " << w.l_j << ", L_T0 = " << w.l_t0
      << ", L_W = " << w.l_w << ";\n"
      << "constexpr int LDS_CELL = " << w.lds_cell << ";  // doubles of LDS scratch per cell\n"
      << "constexpr int ADJ_LDS_CELL = " << w.adj_lds_cell << ";  // per cell in the adjoint\n"
      << "constexpr double RU = " << lit(kRu) << ";\n"
      << "constexpr double LN_PATM_R = " << lit(std::log(kPatm / kRu)) << ";\n"
      << "constexpr double LN10 = " << lit(std::log(10.0)) << ";\n";
    e.thermo_table();
    o << "__constant__ double TMID[NS] = {";
    for (int k = 0; k < ns; ++k) o << lit(m.species[k].tmid) << (k + 1 < ns ? ", " : "};\n");
    // reactions in evaluation order: grouped by kind so a round of lanes mostly
    // takes one branch
    std::vector<int> order;
    for (int kind = 0; kind < 6; ++kind)
        for (int j = 0; j < nr; ++j)
            if ((int)m.reactions[j].kind == kind) order.push_back(j);
    std::vector<int> slot_of(nr);
    for (int s = 0; s < nr; ++s) slot_of[order[s]] = s;
    // per slot: its EFF row (third body and falloff) or its PLOG table (PLOG)
    std::vector<int> effrow(nr, -1);
    int neff = 0, nplog = 0;
    for (int s = 0; s < nr; ++s) {
        const RxnKind k = m.reactions[order[s]].kind;
        if (k == RxnKind::Plog) effrow[s] = nplog++;
        else if (k != RxnKind::Elementary) effrow[s] = neff++;
    }
    auto ints = [&](const char* name, const std::vector<int>& v) {
        o << "__constant__ int " << name << "[" << std::max<size_t>(v.size(), 1) << "] = {";
        if (v.empty()) o << "0";
        for (size_t i = 0; i < v.size(); ++i) o << v[i] << (i + 1 < v.size() ? ", " : "");
        o << "};\n";
    };
    auto dbls = [&](const char* name, const std::vector<double>& v) {
        o << "__constant__ double " << name << "[" << std::max<size_t>(v.size(), 1) << "] = {";
        if (v.empty()) o << "0.0";
        for (size_t i = 0; i < v.size(); ++i) o << lit(v[i]) << (i + 1 < v.size() ? ", " : "");
        o << "};\n";
    };
    // per slot: original index; species of the MAXT reactant then MAXT product
    // slots (-1: unused)
    std::vector<int> orig, sp;
    std::vector<double> low, troe, eff, plog;
    std::vector<int> plog_off(1, 0);
    for (int s = 0; s < nr; ++s) {
        const auto& r = m.reactions[order[s]];
        orig.push_back(order[s]);
        for (int t = 0; t < w.maxt; ++t) sp.push_back(t < (int)r.reac.size() ? r.reac[t].sp : -1);
        for (int t = 0; t < w.maxt; ++t) sp.push_back(t < (int)r.prod.size() ? r.prod[t].sp : -1);
        low.insert(low.end(), {r.lnA0, r.b0, r.EaR0});
        const bool tr = r.kind == RxnKind::Troe;
        if (r.kind == RxnKind::Sri)
            troe.insert(troe.end(), {r.sri[0], -r.sri[1], 1.0 / r.sri[2], r.sri[1], std::log(r.sri[3]), r.sri[4],
                                     0.0, 0.0});
        else
            troe.insert(troe.end(), {tr ? 1.0 - r.alpha : 0.0, tr ? r.alpha : 0.0, tr ? 1.0 / r.T3 : 0.0,
                                     tr ? 1.0 / r.T1 : 0.0, tr && r.has_T2 ? r.T2 : 0.0,
                                     tr ? -(1.0 - r.alpha) / r.T3 : 0.0, tr ? -r.alpha / r.T1 : 0.0,
                                     tr && r.has_T2 ? 1.0 : 0.0});
        if (r.kind == RxnKind::Plog) {
            for (const auto& e : r.plog) plog.insert(plog.end(), {e.lnp, e.lnA, e.b, e.EaR});
            plog_off.push_back((int)(plog.size() / 4));
        } else if (effrow[s] >= 0) {
            for (int k = 0; k < ns; ++k) eff.push_back(r.eff[k]);
        }
    }
    // packed per slot, for one load per reaction round: species slots (8 bits
    // each: species index + 1 in the low 6 bits, coefficient in the top 2;
    // 0 = unused) in two words, then kind | irreversible << 3 | (dnu + 4) << 4 |
    // (EFF row or PLOG table + 1) << 7 | orig << 16
    {
        std::vector<int> pack;
        for (int s = 0; s < nr; ++s) {
            const auto& r = m.reactions[order[s]];
            unsigned long long slots = 0;
            for (int t = 0; t < 2 * w.maxt; ++t) {
                const bool isr = t < w.maxt;
                const auto& side = isr ? r.reac : r.prod;
                const int q = isr ? t : t - w.maxt;
                unsigned v = 0;
                if (q < (int)side.size()) v = (unsigned)(side[q].sp + 1) | ((unsigned)side[q].nu << 6);
                slots |= (unsigned long long)v << (8 * t);
            }
            pack.push_back((int)(unsigned)(slots & 0xffffffffull));
            pack.push_back((int)(unsigned)(slots >> 32));
            pack.push_back((int)((unsigned)r.kind | ((r.reversible ? 0u : 1u) << 3) | ((unsigned)(r.dnu + 4) << 4) |
                                 ((unsigned)(effrow[s] + 1) << 7) | ((unsigned)order[s] << 16)));
        }
        o << "// per slot: species slots (two words, 8 bits each: index + 1 | nu << 6), then\n"
             "// kind | irreversible << 3 | (dnu + 4) << 4 | (EFF row or PLOG table + 1) << 7 |\n"
             "// original index << 16\n";
        ints("RX_PACK", pack);
    }
    o << "// reactions in evaluation order (slot s): original index (kind, species\n"
         "// slots and coefficients are in RX_PACK)\n";
    ints("RX_ORIG", orig);
    o << "// low-pressure limit (ln A0 SI, b0, Ea0/R); Troe: 1-alpha, alpha, 1/T***,\n"
         "// 1/T*, T**, -(1-alpha)/T***, -alpha/T*, [T** given]; SRI: a, -b, 1/c, b, ln d, e\n";
    dbls("RX_LOW", low);
    dbls("RX_TROE", troe);
    {
        bool sri = false, irrev = false;
        for (const auto& r : m.reactions) {
            sri = sri || r.kind == RxnKind::Sri;
            irrev = irrev || !r.reversible;
        }
        o << "// reaction forms present (the kernels leave out the code of the absent ones)\n"
             "constexpr bool HAS_PLOG = " << (nplog > 0 ? "true" : "false") << ";\n"
             "constexpr bool HAS_SRI = " << (sri ? "true" : "false") << ";\n"
             "constexpr bool HAS_IRREV = " << (irrev ? "true" : "false") << ";\n";
    }
    o << "// PLOG tables: entries RX_PLOG_OFF[t] .. RX_PLOG_OFF[t+1] of (ln p, ln A SI, b, Ea/R)\n";
    ints("RX_PLOG_OFF", plog_off);
    dbls("RX_PLOG", plog);
    o << "// third-body efficiencies, one dense row per non-elementary reaction\n";
    dbls("EFF", eff);
    // species -> reactions that change it (slot, net coefficient)
    std::vector<int> off(1, 0), srx, snu;
    for (int k = 0; k < ns; ++k) {
        for (int s = 0; s < nr; ++s) {
            const auto& r = m.reactions[order[s]];
            int v = 0;
            for (auto& t : r.reac) if (t.sp == k) v -= t.nu;
            for (auto& t : r.prod) if (t.sp == k) v += t.nu;
            if (v) {
                srx.push_back(s);
                snu.push_back(v);
            }
        }
        while ((srx.size() - off.back()) % 4) {   // padded to a multiple of 4 (coefficient 0)
            srx.push_back(0);
            snu.push_back(0);
        }
        off.push_back((int)srx.size());
    }
    o << "// species k: the reactions that change it, SP_RX[SP_OFF[k] .. SP_OFF[k+1]),\n"
         "// with net coefficients SP_NU (padded to a multiple of 4 by coefficient 0)\n";
    ints("SP_OFF", off);
    ints("SP_RX", srx);
    ints("SP_NU", snu);
    // the same entries packed for the Jacobian rows, so one round of loads gives
    // everything an entry needs: slot | (net coefficient & 255) << 16, then the
    // species of the reaction's slots 0-3 and 4-5 as bytes (index + 1, 0 unused)
    {
        std::vector<int> jp;
        for (size_t e = 0; e < srx.size(); ++e) {
            const int slot = srx[e];
            jp.push_back((int)((unsigned)slot | (((unsigned)snu[e] & 255u) << 16)));
            unsigned b[2] = {0u, 0u};
            for (int t = 0; t < w.nslot; ++t) {
                const int spc = sp[slot * w.nslot + t];
                b[t / 4] |= (unsigned)(spc + 1) << (8 * (t % 4));
            }
            jp.push_back((int)b[0]);
            jp.push_back((int)b[1]);
        }
        o << "// per SP entry: slot | (net coefficient & 255) << 16, slot species 0-3, 4-5 (bytes, index + 1)\n";
        ints("SP_JPACK", jp);
    }
    // third-body and falloff reactions t (EFF row t): their slot, and the net
    // coefficient of every species in them (the dense third-body part of the
    // Jacobian rows)
    std::vector<int> tbslot;
    std::vector<double> nutb;
    for (int s = 0; s < nr; ++s)
        if (effrow[s] >= 0 && m.reactions[order[s]].kind != RxnKind::Plog) tbslot.push_back(s);
    for (int k = 0; k < ns; ++k)
        for (int s : tbslot) {
            const auto& r = m.reactions[order[s]];
            int v = 0;
            for (auto& t : r.reac) if (t.sp == k) v -= t.nu;
            for (auto& t : r.prod) if (t.sp == k) v += t.nu;
            nutb.push_back((double)v);
        }
    o << "constexpr int NTB = " << tbslot.size() << ";\n"
         "static_assert(NTB == 0 || sizeof(EFF) == sizeof(double) * NTB * NS, \"one EFF row per third-body "
         "reaction\");\n"
         "// third-body or falloff reaction t: its slot (EFF row t); the net coefficient of\n"
         "// species k in it as a 4-bit field (coefficient + 8), eight per word:\n"
         "// NU_TB4[k * NTBW + t / 8] >> (4 (t % 8))\n";
    ints("TB_SLOT", tbslot);
    {
        const int ntb = (int)tbslot.size(), ntbw = std::max(1, (ntb + 7) / 8);
        std::vector<int> packed((size_t)ns * ntbw, 0);
        for (int k = 0; k < ns; ++k)
            for (int t = 0; t < ntb; ++t) {
                const int v = (int)nutb[(size_t)k * ntb + t];
                packed[(size_t)k * ntbw + t / 8] |= (int)((unsigned)(v + 8) << (4 * (t % 8)));
            }
        o << "constexpr int NTBW = " << ntbw << ";\n";
        ints("NU_TB4", packed);
    }
    o << "}  // namespace mech\n";
    return o.str();
}

}  // namespace chemmi
