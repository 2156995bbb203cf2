// chemkin.cpp -- reader for mechanisms in the CHEMKIN text format: ELEMENTS,
// SPECIES, THERMO (NASA-7 four-line records) and REACTIONS sections, with
// reversible (=, <=>) and irreversible (=>) reactions, "+M" third bodies,
// "(+M)" and "(+species)" falloff with LOW / TROE / SRI, efficiencies,
// PLOG tables, DUPLICATE markers and the unit keywords of the REACTIONS line.
// It fills the same MechanismData as the `chemmi-mech 1` reader, so the device
// code is generated from the same representation either way.
#include <algorithm>
#include <cctype>
#include <cmath>
#include <fstream>
#include <map>
#include <set>
#include <sstream>

#include "../../include/chem.h"
#include "mechanism.hpp"

namespace chemmi {
namespace {

// Standard atomic weights, g/mol (IUPAC abridged values), for elements that
// the ELEMENTS section names without a weight of its own.
const std::map<std::string, double>& atomic_weights()
{
    static const std::map<std::string, double> w = {
        {"H", 1.008},   {"D", 2.014},    {"HE", 4.0026}, {"C", 12.011}, {"N", 14.007},
        {"O", 15.999},  {"F", 18.998},   {"NE", 20.180}, {"SI", 28.085}, {"S", 32.06},
        {"CL", 35.45},  {"AR", 39.95},   {"KR", 83.798}, {"XE", 131.29}};
    return w;
}

std::string upper(std::string s)
{
    for (auto& c : s) c = (char)std::toupper((unsigned char)c);
    return s;
}

std::string trim(const std::string& s)
{
    size_t a = 0, b = s.size();
    while (a < b && std::isspace((unsigned char)s[a])) ++a;
    while (b > a && std::isspace((unsigned char)s[b - 1])) --b;
    return s.substr(a, b - a);
}

// A Fortran-style real: D exponents allowed.
bool real(std::string s, double& v)
{
    s = trim(s);
    if (s.empty()) return false;
    for (auto& c : s)
        if (c == 'D' || c == 'd') c = 'E';
    char* end = nullptr;
    v = std::strtod(s.c_str(), &end);
    return end && *end == 0 && std::isfinite(v);
}

bool section_keyword(const std::string& tok, std::string& which)
{
    const std::string u = upper(tok);
    if (u == "ELEMENTS" || u == "ELEM") which = "ELEM";
    else if (u == "SPECIES" || u == "SPEC") which = "SPEC";
    else if (u == "THERMO" || u == "THER") which = "THERMO";
    else if (u == "REACTIONS" || u == "REAC") which = "REAC";
    else return false;
    return true;
}

struct Line {
    int no;
    std::string text;   // comment ('!') removed, right-trimmed
};

std::vector<Line> read_lines(std::istream& in)
{
    std::vector<Line> out;
    std::string s;
    int no = 0;
    while (std::getline(in, s)) {
        ++no;
        const auto bang = s.find('!');
        if (bang != std::string::npos) s.resize(bang);
        while (!s.empty() && (s.back() == '\r' || std::isspace((unsigned char)s.back()))) s.pop_back();
        out.push_back({no, s});
    }
    return out;
}

struct ThermoRecord {
    std::map<std::string, int> comp;   // element (upper case) -> count
    double tmid = 1000.0;
    double lo[7], hi[7];
};

struct CkReader {
    MechanismData& m;
    std::string& err;
    std::string file;
    std::map<std::string, int> sp_index;
    std::map<std::string, ThermoRecord> thermo;   // first record of each species wins
    double tdef[3] = {300.0, 1000.0, 5000.0};
    double e_mult = 4.184;           // activation energy unit -> J/mol (default cal/mol)
    bool e_kelvin = false;

    int fail(int code, int line, const std::string& msg)
    {
        err = file + (line > 0 ? ":" + std::to_string(line) : std::string()) + ": " + msg;
        return code;
    }

    // ---------------- ELEMENTS ----------------
    int elements(const std::string& body, int line)
    {
        // symbols, each optionally followed by /weight/
        size_t i = 0;
        while (i < body.size()) {
            if (std::isspace((unsigned char)body[i])) { ++i; continue; }
            size_t j = i;
            while (j < body.size() && !std::isspace((unsigned char)body[j]) && body[j] != '/') ++j;
            const std::string sym = upper(body.substr(i, j - i));
            i = j;
            while (i < body.size() && std::isspace((unsigned char)body[i])) ++i;
            double w = 0.0;
            if (i < body.size() && body[i] == '/') {
                const size_t k = body.find('/', i + 1);
                if (k == std::string::npos || !real(body.substr(i + 1, k - i - 1), w) || !(w > 0.0))
                    return fail(CHEM_E_PARSE, line, "bad weight for element " + sym);
                i = k + 1;
            } else {
                auto it = atomic_weights().find(sym);
                if (it == atomic_weights().end())
                    return fail(CHEM_E_PARSE, line, "element " + sym + " needs its weight (/w/)");
                w = it->second;
            }
            if (std::find(m.elements.begin(), m.elements.end(), sym) != m.elements.end())
                return fail(CHEM_E_PARSE, line, "element " + sym + " listed twice");
            m.elements.push_back(sym);
            m.element_w.push_back(w);
        }
        return 0;
    }

    // ---------------- SPECIES ----------------
    int species(const std::string& body, int line)
    {
        std::istringstream ss(body);
        for (std::string nm; ss >> nm;) {
            if (sp_index.count(nm)) return fail(CHEM_E_PARSE, line, "species " + nm + " listed twice");
            SpeciesData s;
            s.name = nm;
            sp_index[nm] = (int)m.species.size();
            m.species.push_back(std::move(s));
        }
        return 0;
    }

    // ---------------- THERMO ----------------
    // Records of four lines; fixed columns: name 1-18, composition 25-44 (and
    // 74-78), phase 45, T_low 46-55, T_high 56-65, T_common 66-73; then three
    // lines of 15-column reals: a1..a7 of the upper range, a1..a7 of the lower.
    int thermo_block(const std::vector<Line>& L, size_t& i, size_t end, bool allow_header)
    {
        // optional line of the three default temperatures
        if (allow_header && i < end) {
            std::istringstream ss(L[i].text);
            double t[3];
            std::string extra;
            if (ss >> t[0] >> t[1] >> t[2] && !(ss >> extra)) {
                std::copy(t, t + 3, tdef);
                ++i;
            }
        }
        while (i < end) {
            if (trim(L[i].text).empty()) { ++i; continue; }
            std::istringstream fs(L[i].text);
            std::string first, kw;
            fs >> first;
            if (upper(first) == "END" || section_keyword(first, kw)) break;
            if (i + 3 >= end) return fail(CHEM_E_PARSE, L[i].no, "truncated thermo record");
            std::string l1 = L[i].text, l2 = L[i + 1].text, l3 = L[i + 2].text, l4 = L[i + 3].text;
            l1.resize(std::max<size_t>(l1.size(), 80), ' ');
            for (auto* l : {&l2, &l3, &l4}) l->resize(std::max<size_t>(l->size(), 80), ' ');
            std::istringstream ns(l1.substr(0, 18));
            std::string name;
            ns >> name;
            ThermoRecord r;
            auto add_elem = [&](const std::string& f) -> int {
                const std::string sym = upper(trim(f.substr(0, 2)));
                const std::string cnt = trim(f.substr(2));
                if (sym.empty()) return 0;
                double c = 0.0;
                if (cnt.empty()) return 0;
                if (!real(cnt, c) || c < 0.0 || c != std::floor(c))
                    return fail(CHEM_E_PARSE, L[i].no, "bad composition of " + name);
                if (c > 0.0) r.comp[sym] += (int)c;
                return 0;
            };
            for (int e = 0; e < 4; ++e)
                if (int rc = add_elem(l1.substr(24 + 5 * e, 5))) return rc;
            if (int rc = add_elem(l1.substr(73, 5))) return rc;
            double tl, th, tm;
            if (!real(l1.substr(45, 10), tl) || !real(l1.substr(55, 10), th))
                return fail(CHEM_E_PARSE, L[i].no, "bad temperature range of " + name);
            r.tmid = real(l1.substr(65, 8), tm) ? tm : tdef[1];
            double a[14];
            const std::string* rows[3] = {&l2, &l3, &l4};
            for (int q = 0; q < 14; ++q) {
                const std::string& row = *rows[q / 5];
                if (!real(row.substr(15 * (q % 5), 15), a[q]))
                    return fail(CHEM_E_PARSE, L[i + 1 + q / 5].no, "bad thermo coefficient of " + name);
            }
            for (int q = 0; q < 7; ++q) {
                r.hi[q] = a[q];
                r.lo[q] = a[7 + q];
            }
            if (!name.empty() && !thermo.count(name)) thermo[name] = r;
            i += 4;
        }
        return 0;
    }

    // ---------------- REACTIONS ----------------
    int units(const std::vector<std::string>& toks, int line)
    {
        for (const auto& t : toks) {
            const std::string u = upper(t);
            if (u == "CAL/MOLE") e_mult = 4.184;
            else if (u == "KCAL/MOLE") e_mult = 4184.0;
            else if (u == "JOULES/MOLE") e_mult = 1.0;
            else if (u == "KJOULES/MOLE") e_mult = 1e3;
            else if (u == "KELVINS") e_kelvin = true;
            else if (u == "EVOLTS") e_mult = 96485.33212;   // the Faraday constant, J/(mol eV)
            else if (u == "MOLES") continue;
            else if (u == "MOLECULES") return fail(CHEM_E_UNSUPPORTED, line, "MOLECULES units are not supported");
            else return fail(CHEM_E_PARSE, line, "unknown unit keyword " + t);
        }
        return 0;
    }

    // E / R in K, converted as the other reader converts kJ/mol
    double to_K(double E) const { return e_kelvin ? E : E * e_mult / kRu; }

    struct Pending {
        ReactionData r;
        int line = 0;
        int order = 0;            // sum of reactant coefficients
        bool third = false;       // "+M"
        bool falloff = false;     // "(+M)" or "(+species)"
        int collider = -1;        // "(+species)"
        bool dup = false, has_low = false, has_troe = false, has_sri = false;
        double A = 0.0, b = 0.0, E = 0.0;
    };

    // one side of the equation: "2H2+O2+M", "H+O2(+M)"
    int side(std::string txt, std::vector<Term>& out, bool& m_here, std::string& fo, int line)
    {
        m_here = false;
        fo.clear();
        const size_t a = txt.find("(+");
        if (a != std::string::npos) {
            const size_t b = txt.find(')', a);
            if (b == std::string::npos) return fail(CHEM_E_PARSE, line, "unclosed '(+'");
            fo = txt.substr(a + 2, b - a - 2);
            txt = txt.substr(0, a) + txt.substr(b + 1);
        }
        std::vector<std::string> parts;
        std::string cur;
        for (size_t i = 0; i < txt.size(); ++i) {
            // a '+' right after another or at the start belongs to a name (ions)
            if (txt[i] == '+' && !cur.empty()) {
                parts.push_back(cur);
                cur.clear();
            } else {
                cur.push_back(txt[i]);
            }
        }
        if (!cur.empty()) parts.push_back(cur);
        for (const auto& t : parts) {
            if (upper(t) == "M") {
                if (m_here) return fail(CHEM_E_PARSE, line, "'+M' twice on one side");
                m_here = true;
                continue;
            }
            int nu = 1;
            std::string nm = t;
            if (!sp_index.count(t)) {
                size_t k = 0;
                while (k < t.size() && (std::isdigit((unsigned char)t[k]) || t[k] == '.')) ++k;
                double c = 0.0;
                if (k == 0 || !real(t.substr(0, k), c)) return fail(CHEM_E_PARSE, line, "unknown species " + t);
                if (c != std::floor(c) || c < 1.0)
                    return fail(CHEM_E_UNSUPPORTED, line, "non-integer coefficient in " + t);
                nu = (int)c;
                nm = t.substr(k);
                if (!sp_index.count(nm)) return fail(CHEM_E_PARSE, line, "unknown species " + nm);
            }
            const int sp = sp_index[nm];
            bool merged = false;
            for (auto& x : out)
                if (x.sp == sp) {
                    x.nu += nu;
                    merged = true;
                }
            if (!merged) out.push_back({sp, nu});
        }
        if (out.empty()) return fail(CHEM_E_PARSE, line, "empty reaction side");
        return 0;
    }

    int equation(const std::string& eq, Pending& p, int line)
    {
        std::string lhs, rhs;
        size_t k;
        if ((k = eq.find("<=>")) != std::string::npos) {
            lhs = eq.substr(0, k);
            rhs = eq.substr(k + 3);
        } else if ((k = eq.find("=>")) != std::string::npos) {
            lhs = eq.substr(0, k);
            rhs = eq.substr(k + 2);
            p.r.reversible = false;
        } else if ((k = eq.find('=')) != std::string::npos) {
            lhs = eq.substr(0, k);
            rhs = eq.substr(k + 1);
        } else {
            return fail(CHEM_E_PARSE, line, "no '=' in reaction");
        }
        bool ml, mr;
        std::string fl, fr;
        if (int rc = side(lhs, p.r.reac, ml, fl, line)) return rc;
        if (int rc = side(rhs, p.r.prod, mr, fr, line)) return rc;
        if (ml != mr) return fail(CHEM_E_PARSE, line, "'+M' on one side only");
        if (fl != fr) return fail(CHEM_E_PARSE, line, "falloff collider differs between the sides");
        if (ml && !fl.empty()) return fail(CHEM_E_PARSE, line, "both '+M' and '(+M)'");
        p.third = ml;
        p.falloff = !fl.empty();
        if (p.falloff && upper(fl) != "M") {
            if (!sp_index.count(fl)) return fail(CHEM_E_PARSE, line, "unknown collider " + fl);
            p.collider = sp_index[fl];
        }
        for (auto& x : p.r.reac) {
            p.order += x.nu;
            p.r.dnu -= x.nu;
        }
        for (auto& x : p.r.prod) p.r.dnu += x.nu;
        return 0;
    }

    // auxiliary line: KEYWORD /values/ pairs, or species /efficiency/ pairs
    int auxiliary(const std::string& text, Pending& p, int line)
    {
        size_t i = 0;
        while (i < text.size()) {
            if (std::isspace((unsigned char)text[i])) { ++i; continue; }
            size_t j = i;
            while (j < text.size() && !std::isspace((unsigned char)text[j]) && text[j] != '/') ++j;
            const std::string key = text.substr(i, j - i);
            const std::string ukey = upper(key);
            static const std::set<std::string> unsupported = {
                "REV", "HIGH", "FORD", "RORD", "CHEB", "TCHEB", "PCHEB", "LT", "RLT", "UNITS", "MOME",
                "XSMI", "TDEP", "EXCI", "JAN", "FIT1", "USRPROG"};
            if (unsupported.count(ukey))
                return fail(CHEM_E_UNSUPPORTED, line, "auxiliary keyword " + ukey + " is not supported");
            i = j;
            while (i < text.size() && std::isspace((unsigned char)text[i])) ++i;
            std::vector<double> vals;
            bool has_vals = false;
            if (i < text.size() && text[i] == '/') {
                const size_t k = text.find('/', i + 1);
                if (k == std::string::npos) return fail(CHEM_E_PARSE, line, "unclosed '/' after " + key);
                std::istringstream vs(text.substr(i + 1, k - i - 1));
                for (std::string w; vs >> w;) {
                    double v;
                    if (!real(w, v)) return fail(CHEM_E_PARSE, line, "bad number '" + w + "' after " + key);
                    vals.push_back(v);
                }
                has_vals = true;
                i = k + 1;
            }
            if (ukey == "DUP" || ukey == "DUPLICATE") {
                p.dup = true;
            } else if (ukey == "LOW") {
                if (!p.falloff || vals.size() != 3) return fail(CHEM_E_PARSE, line, "LOW needs a falloff reaction and 3 numbers");
                if (!(vals[0] > 0.0)) return fail(CHEM_E_MECH_INVALID, line, "LOW A must be positive");
                p.r.lnA0 = std::log(vals[0]) + p.order * std::log(1e-6);
                p.r.b0 = vals[1];
                p.r.EaR0 = to_K(vals[2]);
                p.has_low = true;
            } else if (ukey == "TROE") {
                if (!p.falloff || (vals.size() != 3 && vals.size() != 4))
                    return fail(CHEM_E_PARSE, line, "TROE needs a falloff reaction and 3 or 4 numbers");
                p.r.alpha = vals[0];
                p.r.T3 = vals[1];
                p.r.T1 = vals[2];
                p.r.has_T2 = vals.size() == 4;
                p.r.T2 = p.r.has_T2 ? vals[3] : 0.0;
                if (!(p.r.T3 > 0.0) || !(p.r.T1 > 0.0))
                    return fail(CHEM_E_MECH_INVALID, line, "Troe T*** and T* must be positive");
                p.has_troe = true;
            } else if (ukey == "SRI") {
                if (!p.falloff || (vals.size() != 3 && vals.size() != 5))
                    return fail(CHEM_E_PARSE, line, "SRI needs a falloff reaction and 3 or 5 numbers");
                for (size_t q = 0; q < vals.size(); ++q) p.r.sri[q] = vals[q];
                if (vals.size() == 3) {
                    p.r.sri[3] = 1.0;
                    p.r.sri[4] = 0.0;
                }
                if (!(p.r.sri[0] >= 0.0) || !(p.r.sri[2] > 0.0) || !(p.r.sri[3] > 0.0))
                    return fail(CHEM_E_MECH_INVALID, line, "SRI needs a >= 0, c > 0, d > 0");
                p.has_sri = true;
            } else if (ukey == "PLOG") {
                if (vals.size() != 4) return fail(CHEM_E_PARSE, line, "PLOG needs 4 numbers");
                if (!(vals[0] > 0.0) || !(vals[1] > 0.0))
                    return fail(CHEM_E_MECH_INVALID, line, "PLOG pressure and A must be positive");
                const double lnp = std::log(vals[0] * kPatm);
                if (!p.r.plog.empty() && !(lnp > p.r.plog.back().lnp))
                    return fail(CHEM_E_UNSUPPORTED, line,
                                "PLOG pressures must increase (repeated pressures are not supported)");
                p.r.plog.push_back({lnp, std::log(vals[1]) + (p.order - 1) * std::log(1e-6), vals[2], to_K(vals[3])});
            } else if (sp_index.count(key) && has_vals) {
                if (!(p.third || p.falloff) || p.collider >= 0)
                    return fail(CHEM_E_PARSE, line, "efficiency on a reaction without '+M' or '(+M)'");
                if (vals.size() != 1 || vals[0] < 0.0) return fail(CHEM_E_PARSE, line, "bad efficiency of " + key);
                p.r.eff[sp_index[key]] = vals[0];
            } else {
                return fail(CHEM_E_PARSE, line, "unknown keyword or species '" + key + "'");
            }
        }
        return 0;
    }

    int finish(Pending& p)
    {
        ReactionData& r = p.r;
        if (!(p.A > 0.0)) return fail(CHEM_E_MECH_INVALID, p.line, "A must be positive");
        if (!r.plog.empty()) {
            if (p.third || p.falloff) return fail(CHEM_E_UNSUPPORTED, p.line, "PLOG with a third body");
            if (r.plog.size() > kMaxPlog) return fail(CHEM_E_UNSUPPORTED, p.line, "more than 16 PLOG pressures");
            // the main-line rate is not used: the table is the rate
            r.kind = RxnKind::Plog;
            r.lnA = 0.0;
            r.b = 0.0;
            r.EaR = 0.0;
        } else if (p.falloff) {
            if (!p.has_low) return fail(CHEM_E_PARSE, p.line, "falloff reaction without LOW");
            if (p.has_troe && p.has_sri) return fail(CHEM_E_PARSE, p.line, "both TROE and SRI");
            r.kind = p.has_troe ? RxnKind::Troe : p.has_sri ? RxnKind::Sri : RxnKind::Lindemann;
            if (p.collider >= 0)
                for (int k = 0; k < (int)r.eff.size(); ++k) r.eff[k] = k == p.collider ? 1.0 : 0.0;
        } else {
            if (p.has_low || p.has_troe || p.has_sri)
                return fail(CHEM_E_PARSE, p.line, "LOW/TROE/SRI on a reaction without '(+M)'");
            r.kind = p.third ? RxnKind::ThirdBody : RxnKind::Elementary;
        }
        if (r.kind != RxnKind::Plog) {
            // cm-mol-s to SI: one cm^3/mol per concentration factor beyond the first
            const int orderA = p.order + (p.third ? 1 : 0);
            r.lnA = std::log(p.A) + (orderA - 1) * std::log(1e-6);
            r.b = p.b;
            r.EaR = to_K(p.E);
        }
        for (size_t e = 0; e < m.elements.size(); ++e) {
            long bal = 0;
            for (auto& x : r.reac) bal -= (long)x.nu * m.species[x.sp].atoms[e];
            for (auto& x : r.prod) bal += (long)x.nu * m.species[x.sp].atoms[e];
            if (bal != 0) return fail(CHEM_E_MECH_INVALID, p.line, "element " + m.elements[e] + " is not balanced");
        }
        return 0;
    }

    int reactions(const std::vector<Line>& L, size_t i, size_t end)
    {
        std::vector<Pending> rx;
        for (; i < end; ++i) {
            const std::string t = trim(L[i].text);
            if (t.empty()) continue;
            if (upper(t) == "END") break;
            if (t.find('=') != std::string::npos) {
                std::istringstream ss(t);
                std::vector<std::string> tok;
                for (std::string w; ss >> w;) tok.push_back(w);
                if (tok.size() < 4) return fail(CHEM_E_PARSE, L[i].no, "reaction line needs A, b, E");
                Pending p;
                p.line = L[i].no;
                p.r.eff.assign(m.species.size(), 1.0);
                const size_t n = tok.size();
                if (!real(tok[n - 3], p.A) || !real(tok[n - 2], p.b) || !real(tok[n - 1], p.E))
                    return fail(CHEM_E_PARSE, L[i].no, "bad Arrhenius numbers");
                std::string eq;
                for (size_t q = 0; q + 3 < n; ++q) eq += tok[q];
                if (int rc = equation(eq, p, L[i].no)) return rc;
                rx.push_back(std::move(p));
            } else {
                if (rx.empty()) return fail(CHEM_E_PARSE, L[i].no, "auxiliary data before any reaction");
                if (int rc = auxiliary(t, rx.back(), L[i].no)) return rc;
            }
        }
        for (auto& p : rx)
            if (int rc = finish(p)) return rc;
        // reactions with the same species on each side (either way round) and the
        // same third-body form must all be marked DUPLICATE, and a DUPLICATE needs
        // a partner
        auto key = [&](const Pending& p, bool flip) {
            auto side = [](std::vector<Term> s) {
                std::sort(s.begin(), s.end(), [](const Term& a, const Term& b) { return a.sp < b.sp; });
                std::string k;
                for (auto& t : s) k += std::to_string(t.sp) + "*" + std::to_string(t.nu) + ",";
                return k;
            };
            const std::string a = side(p.r.reac), b = side(p.r.prod);
            return (flip ? b + "=" + a : a + "=" + b) + "|" + std::to_string((int)p.third) +
                   std::to_string((int)p.falloff) + std::to_string(p.collider);
        };
        std::map<std::string, std::vector<size_t>> groups;
        for (size_t q = 0; q < rx.size(); ++q) {
            const std::string k1 = key(rx[q], false), k2 = key(rx[q], true);
            groups[std::min(k1, k2)].push_back(q);
        }
        for (auto& g : groups) {
            for (size_t q : g.second) {
                if (g.second.size() > 1 && !rx[q].dup)
                    return fail(CHEM_E_MECH_INVALID, rx[q].line, "duplicate reaction not marked DUPLICATE");
                if (g.second.size() == 1 && rx[q].dup)
                    return fail(CHEM_E_MECH_INVALID, rx[q].line, "DUPLICATE reaction without a duplicate");
            }
        }
        for (auto& p : rx) m.reactions.push_back(std::move(p.r));
        return 0;
    }

    int species_data()
    {
        for (auto& s : m.species) {
            auto it = thermo.find(s.name);
            if (it == thermo.end()) return fail(CHEM_E_MECH_INVALID, 0, "species " + s.name + " has no thermo data");
            const ThermoRecord& r = it->second;
            s.atoms.assign(m.elements.size(), 0);
            double w = 0.0;
            for (auto& [sym, n] : r.comp) {
                auto e = std::find(m.elements.begin(), m.elements.end(), sym);
                if (e == m.elements.end())
                    return fail(CHEM_E_MECH_INVALID, 0, "species " + s.name + " has element " + sym +
                                                            " that ELEMENTS does not list");
                const size_t idx = (size_t)(e - m.elements.begin());
                s.atoms[idx] += n;
            }
            // in the order of ELEMENTS, as the other reader sums them
            for (size_t e = 0; e < m.elements.size(); ++e)
                if (s.atoms[e]) w += s.atoms[e] * m.element_w[e];
            if (!(w > 0.0)) return fail(CHEM_E_MECH_INVALID, 0, "species " + s.name + " has no atoms");
            s.W = w * 1e-3;
            s.tmid = r.tmid;
            std::copy(r.lo, r.lo + 7, s.lo);
            std::copy(r.hi, r.hi + 7, s.hi);
            s.has_thermo = true;
        }
        return 0;
    }
};

bool open_lines(const std::string& path, std::vector<Line>& out)
{
    std::ifstream in(path);
    if (!in) return false;
    out = read_lines(in);
    return true;
}

}  // namespace

int parse_chemkin(const std::string& path, const std::string& thermo_path, MechanismData& m, std::string& err)
{
    std::vector<Line> L;
    if (!open_lines(path, L)) {
        err = "cannot open " + path;
        return CHEM_E_INVAL;
    }
    m = MechanismData{};
    {
        auto slash = path.find_last_of('/');
        std::string base = slash == std::string::npos ? path : path.substr(slash + 1);
        m.name = base.substr(0, base.find('.'));
    }
    CkReader rd{m, err, path};
    // sections in file order; a section runs to END or to the next section keyword
    bool seen_reac = false, seen_elem = false, seen_spec = false;
    size_t i = 0;
    while (i < L.size()) {
        const std::string t = trim(L[i].text);
        if (t.empty()) { ++i; continue; }
        std::istringstream ss(t);
        std::string first;
        ss >> first;
        std::string which;
        if (!section_keyword(first, which)) return rd.fail(CHEM_E_PARSE, L[i].no, "expected a section keyword");
        std::string rest;
        std::getline(ss, rest);
        const int line0 = L[i].no;
        ++i;
        if (which == "THERMO") {
            // "THERMO" or "THERMO ALL": either way every species needs a record
            // here or in the separate thermo file (there is no built-in database)
            if (int rc = rd.thermo_block(L, i, L.size(), true)) return rc;
            if (i < L.size() && upper(trim(L[i].text)) == "END") ++i;
            continue;
        }
        if (which == "REAC") {
            std::istringstream us(rest);
            std::vector<std::string> toks;
            for (std::string w; us >> w;) toks.push_back(w);
            if (int rc = rd.units(toks, line0)) return rc;
            if (!seen_elem || !seen_spec) return rd.fail(CHEM_E_PARSE, line0, "REACTIONS before ELEMENTS and SPECIES");
            if (!thermo_path.empty()) {
                std::vector<Line> TL;
                if (!open_lines(thermo_path, TL)) {
                    err = "cannot open " + thermo_path;
                    return CHEM_E_INVAL;
                }
                size_t k = 0;
                while (k < TL.size() && trim(TL[k].text).empty()) ++k;
                std::string tw;
                bool header = false;
                if (k < TL.size()) {
                    std::istringstream hs(trim(TL[k].text));
                    hs >> tw;
                    std::string which2;
                    if (section_keyword(tw, which2) && which2 == "THERMO") {
                        ++k;
                        header = true;
                    }
                }
                const std::string keep = rd.file;
                rd.file = thermo_path;
                // records already read from the mechanism file take precedence
                if (int rc = rd.thermo_block(TL, k, TL.size(), header)) return rc;
                rd.file = keep;
            }
            if (int rc = rd.species_data()) return rc;
            size_t end = i;
            while (end < L.size() && upper(trim(L[end].text)) != "END") ++end;
            if (int rc = rd.reactions(L, i, end)) return rc;
            i = end + 1;
            seen_reac = true;
            continue;
        }
        // ELEMENTS / SPECIES: everything up to END or the next section keyword,
        // the rest of the keyword's own line included
        std::string body = rest;
        while (i < L.size()) {
            std::istringstream ls(trim(L[i].text));
            std::string w, kw;
            ls >> w;
            if (upper(w) == "END") { ++i; break; }
            if (section_keyword(w, kw)) break;
            body += " " + L[i].text;
            ++i;
        }
        if (which == "ELEM") {
            if (int rc = rd.elements(body, line0)) return rc;
            seen_elem = true;
        } else {
            if (!seen_elem) return rd.fail(CHEM_E_PARSE, line0, "SPECIES before ELEMENTS");
            if (int rc = rd.species(body, line0)) return rc;
            seen_spec = true;
        }
    }
    if (!seen_reac) {
        // a mechanism with no REACTIONS section: species and thermo only
        if (!seen_elem || !seen_spec) {
            err = path + ": no ELEMENTS or SPECIES section";
            return CHEM_E_PARSE;
        }
        if (!thermo_path.empty()) {
            err = path + ": a separate thermo file needs a REACTIONS section";
            return CHEM_E_PARSE;
        }
        if (int rc = rd.species_data()) return rc;
    }
    return validate_mechanism(m, err);
}

}  // namespace chemmi
