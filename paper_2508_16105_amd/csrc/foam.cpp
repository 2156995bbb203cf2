// foam.cpp -- reader for mechanisms in OpenFOAM's chemistry dictionary format:
// a `reactions` file (species list and a `reactions` dictionary of typed
// reaction entries) and a `thermo` file (per-species molWeight, NASA-7
// `janaf` coefficients and element composition).  It fills the same
// MechanismData as the other readers.  OpenFOAM's rates are per kmol: A in
// (m^3/kmol)^(n-1)/s for a reaction of order n, and Ta = Ea/R in K.
#include <cctype>
#include <cmath>
#include <fstream>
#include <map>
#include <memory>
#include <sstream>

#include "../../include/chem.h"
#include "mechanism.hpp"

namespace chemmi {
namespace {

// ---------------- dictionary syntax ----------------
// A dictionary maps keywords to sub-dictionaries or to primitive entries (the
// tokens up to ';', lists in parentheses kept as tokens).

struct Dict;
struct Entry {
    std::unique_ptr<Dict> dict;
    std::vector<std::string> toks;
};
struct Dict {
    std::vector<std::pair<std::string, Entry>> items;
    const Entry* find(const std::string& k) const
    {
        for (auto& [key, e] : items)
            if (key == k) return &e;
        return nullptr;
    }
};

struct Lexer {
    std::string s;
    size_t i = 0;
    std::string err;

    bool next(std::string& t)
    {
        for (;;) {
            while (i < s.size() && std::isspace((unsigned char)s[i])) ++i;
            if (i + 1 < s.size() && s[i] == '/' && s[i + 1] == '/') {
                while (i < s.size() && s[i] != '\n') ++i;
                continue;
            }
            if (i + 1 < s.size() && s[i] == '/' && s[i + 1] == '*') {
                const size_t k = s.find("*/", i + 2);
                i = k == std::string::npos ? s.size() : k + 2;
                continue;
            }
            break;
        }
        if (i >= s.size()) return false;
        const char c = s[i];
        if (c == '{' || c == '}' || c == '(' || c == ')' || c == ';') {
            t = std::string(1, c);
            ++i;
            return true;
        }
        if (c == '"') {
            const size_t k = s.find('"', i + 1);
            if (k == std::string::npos) {
                err = "unterminated string";
                return false;
            }
            t = s.substr(i, k - i + 1);
            i = k + 1;
            return true;
        }
        const size_t a = i;
        while (i < s.size() && !std::isspace((unsigned char)s[i]) && s[i] != '{' && s[i] != '}' && s[i] != '(' &&
               s[i] != ')' && s[i] != ';' && s[i] != '"')
            ++i;
        t = s.substr(a, i - a);
        return true;
    }
};

bool parse_dict(Lexer& L, Dict& d, bool top)
{
    std::string t;
    while (L.next(t)) {
        if (t == "}") return !top;
        if (t == ";") continue;
        const std::string key = t;
        if (!L.next(t)) {
            L.err = "entry '" + key + "' has no value";
            return false;
        }
        Entry e;
        if (t == "{") {
            e.dict = std::make_unique<Dict>();
            if (!parse_dict(L, *e.dict, false)) {
                if (L.err.empty()) L.err = "unbalanced braces after '" + key + "'";
                return false;
            }
        } else {
            int depth = 0;
            for (;;) {
                if (t == "(") ++depth;
                if (t == ")") --depth;
                if (t == ";" && depth == 0) break;
                if (t == "{" || t == "}") {
                    L.err = "unexpected brace in entry '" + key + "'";
                    return false;
                }
                e.toks.push_back(t);
                if (!L.next(t)) {
                    L.err = "entry '" + key + "' is not terminated by ';'";
                    return false;
                }
            }
        }
        d.items.emplace_back(key, std::move(e));
    }
    if (!L.err.empty()) return false;
    if (!top) L.err = "unbalanced braces";
    return top;
}

int read_dict(const std::string& path, Dict& d, std::string& err)
{
    std::ifstream in(path);
    if (!in) {
        err = "cannot open " + path;
        return CHEM_E_INVAL;
    }
    Lexer L;
    L.s.assign(std::istreambuf_iterator<char>(in), std::istreambuf_iterator<char>());
    if (!parse_dict(L, d, true)) {
        err = path + ": " + L.err;
        return CHEM_E_PARSE;
    }
    return 0;
}

bool num(const std::string& s, double& v)
{
    char* end = nullptr;
    v = std::strtod(s.c_str(), &end);
    return !s.empty() && end && *end == 0 && std::isfinite(v);
}

// words of a list entry "N ( a b c )" or "( a b c )", parentheses dropped
std::vector<std::string> list_words(const std::vector<std::string>& toks)
{
    std::vector<std::string> out;
    size_t k = 0;
    double n;
    if (!toks.empty() && num(toks[0], n) && toks.size() > 1 && toks[1] == "(") k = 1;
    for (; k < toks.size(); ++k)
        if (toks[k] != "(" && toks[k] != ")") out.push_back(toks[k]);
    return out;
}

struct FoamReader {
    MechanismData& m;
    std::string& err;
    std::string file;
    std::map<std::string, int> sp_index;

    int fail(int code, const std::string& where, const std::string& msg)
    {
        err = file + ": " + where + ": " + msg;
        return code;
    }

    int scalar(const Dict& d, const std::string& k, double& v, const std::string& where)
    {
        const Entry* e = d.find(k);
        if (!e || e->dict || e->toks.size() != 1 || !num(e->toks[0], v))
            return fail(CHEM_E_PARSE, where, "needs a number '" + k + "'");
        return 0;
    }

    // Arrhenius triple (A, beta, Ta) of dictionary d; A converted from kmol
    // units for a rate of the given order to mol units
    int arrhenius(const Dict& d, int order, double& lnA, double& b, double& TaK, const std::string& where)
    {
        double A;
        if (int rc = scalar(d, "A", A, where)) return rc;
        if (int rc = scalar(d, "beta", b, where)) return rc;
        if (int rc = scalar(d, "Ta", TaK, where)) return rc;
        if (!(A > 0.0)) return fail(CHEM_E_MECH_INVALID, where, "A must be positive");
        lnA = std::log(A) + (order - 1) * std::log(1e-3);
        return 0;
    }

    int side(std::string txt, std::vector<Term>& out, const std::string& where)
    {
        // terms separated by '+', with or without spaces around it
        std::string spaced;
        for (char c : txt) spaced += c == '+' ? std::string(" + ") : std::string(1, c);
        std::istringstream ss(spaced);
        std::string w;
        bool want_term = true;
        while (ss >> w) {
            if (w == "+") {
                want_term = true;
                continue;
            }
            if (!want_term) return fail(CHEM_E_PARSE, where, "missing '+' before " + w);
            want_term = false;
            if (w.find('^') != std::string::npos)
                return fail(CHEM_E_UNSUPPORTED, where, "reaction orders (^) are not supported");
            size_t k = 0;
            while (k < w.size() && (std::isdigit((unsigned char)w[k]) || w[k] == '.')) ++k;
            int nu = 1;
            std::string nm = w;
            if (k > 0 && !sp_index.count(w)) {
                double c;
                if (!num(w.substr(0, k), c) || c != std::floor(c) || c < 1.0)
                    return fail(CHEM_E_UNSUPPORTED, where, "non-integer coefficient in " + w);
                nu = (int)c;
                nm = w.substr(k);
            }
            if (!sp_index.count(nm)) return fail(CHEM_E_PARSE, where, "unknown species " + nm);
            const int sp = sp_index[nm];
            bool merged = false;
            for (auto& x : out)
                if (x.sp == sp) {
                    x.nu += nu;
                    merged = true;
                }
            if (!merged) out.push_back({sp, nu});
        }
        if (out.empty()) return fail(CHEM_E_PARSE, where, "empty reaction side");
        return 0;
    }

    int efficiencies(const Dict& r, ReactionData& x, const std::string& where)
    {
        const Entry* tb = r.find("thirdBodyEfficiencies");
        if (!tb || !tb->dict) return fail(CHEM_E_PARSE, where, "needs thirdBodyEfficiencies");
        const Entry* c = tb->dict->find("coeffs");
        if (!c || c->dict) return fail(CHEM_E_PARSE, where, "thirdBodyEfficiencies needs coeffs");
        auto w = list_words(c->toks);
        if (w.size() % 2) return fail(CHEM_E_PARSE, where, "coeffs must be (species value) pairs");
        for (size_t k = 0; k < w.size(); k += 2) {
            double e;
            if (!sp_index.count(w[k]) || !num(w[k + 1], e) || e < 0.0)
                return fail(CHEM_E_PARSE, where, "bad efficiency (" + w[k] + " " + w[k + 1] + ")");
            x.eff[sp_index[w[k]]] = e;
        }
        return 0;
    }

    int reaction(const std::string& name, const Dict& r)
    {
        const std::string where = "reaction " + name;
        const Entry* te = r.find("type");
        const Entry* re = r.find("reaction");
        if (!te || te->toks.size() != 1 || !re || re->toks.size() != 1 || re->toks[0].size() < 2)
            return fail(CHEM_E_PARSE, where, "needs 'type' and 'reaction'");
        std::string type = te->toks[0];
        if (type.size() > 8 && type.compare(type.size() - 8, 8, "Reaction") == 0) type.resize(type.size() - 8);
        ReactionData x;
        x.eff.assign(m.species.size(), 1.0);
        std::string kind;
        if (type.rfind("reversible", 0) == 0) kind = type.substr(10);
        else if (type.rfind("irreversible", 0) == 0) {
            kind = type.substr(12);
            x.reversible = false;
        } else {
            return fail(CHEM_E_UNSUPPORTED, where, "reaction type " + type + " is not supported");
        }
        const std::string eq = re->toks[0].substr(1, re->toks[0].size() - 2);
        const size_t k = eq.find('=');
        if (k == std::string::npos || eq.find('=', k + 1) != std::string::npos)
            return fail(CHEM_E_PARSE, where, "reaction needs one '='");
        if (int rc = side(eq.substr(0, k), x.reac, where)) return rc;
        if (int rc = side(eq.substr(k + 1), x.prod, where)) return rc;
        int order = 0;
        for (auto& t : x.reac) {
            order += t.nu;
            x.dnu -= t.nu;
        }
        for (auto& t : x.prod) x.dnu += t.nu;
        if (kind == "Arrhenius") {
            x.kind = RxnKind::Elementary;
            if (int rc = arrhenius(r, order, x.lnA, x.b, x.EaR, where)) return rc;
        } else if (kind == "ThirdBodyArrhenius") {
            x.kind = RxnKind::ThirdBody;
            if (int rc = arrhenius(r, order + 1, x.lnA, x.b, x.EaR, where)) return rc;
            if (int rc = efficiencies(r, x, where)) return rc;
        } else if (kind == "ArrheniusLindemannFallOff" || kind == "ArrheniusTroeFallOff" ||
                   kind == "ArrheniusSRIFallOff") {
            const Entry* k0 = r.find("k0");
            const Entry* ki = r.find("kInf");
            const Entry* F = r.find("F");
            if (!k0 || !k0->dict || !ki || !ki->dict || !F || !F->dict)
                return fail(CHEM_E_PARSE, where, "falloff needs k0, kInf and F dictionaries");
            if (int rc = arrhenius(*ki->dict, order, x.lnA, x.b, x.EaR, where + " kInf")) return rc;
            if (int rc = arrhenius(*k0->dict, order + 1, x.lnA0, x.b0, x.EaR0, where + " k0")) return rc;
            if (int rc = efficiencies(r, x, where)) return rc;
            if (kind == "ArrheniusLindemannFallOff") {
                x.kind = RxnKind::Lindemann;
            } else if (kind == "ArrheniusTroeFallOff") {
                x.kind = RxnKind::Troe;
                if (int rc = scalar(*F->dict, "alpha", x.alpha, where)) return rc;
                if (int rc = scalar(*F->dict, "Tsss", x.T3, where)) return rc;
                if (int rc = scalar(*F->dict, "Ts", x.T1, where)) return rc;
                if (int rc = scalar(*F->dict, "Tss", x.T2, where)) return rc;
                x.has_T2 = true;
                if (!(x.T3 > 0.0) || !(x.T1 > 0.0))
                    return fail(CHEM_E_MECH_INVALID, where, "Troe Tsss and Ts must be positive");
            } else {
                x.kind = RxnKind::Sri;
                const char* names[5] = {"a", "b", "c", "d", "e"};
                for (int q = 0; q < 5; ++q)
                    if (int rc = scalar(*F->dict, names[q], x.sri[q], where)) return rc;
                if (!(x.sri[0] >= 0.0) || !(x.sri[2] > 0.0) || !(x.sri[3] > 0.0))
                    return fail(CHEM_E_MECH_INVALID, where, "SRI needs a >= 0, c > 0, d > 0");
            }
        } else {
            return fail(CHEM_E_UNSUPPORTED, where, "reaction type " + type + " is not supported");
        }
        for (size_t e = 0; e < m.elements.size(); ++e) {
            long bal = 0;
            for (auto& t : x.reac) bal -= (long)t.nu * m.species[t.sp].atoms[e];
            for (auto& t : x.prod) bal += (long)t.nu * m.species[t.sp].atoms[e];
            if (bal != 0) return fail(CHEM_E_MECH_INVALID, where, "element " + m.elements[e] + " is not balanced");
        }
        m.reactions.push_back(std::move(x));
        return 0;
    }
};

}  // namespace

int parse_openfoam(const std::string& reactions_path, const std::string& thermo_path, MechanismData& m,
                   std::string& err)
{
    Dict R, Th;
    if (int rc = read_dict(reactions_path, R, err)) return rc;
    if (int rc = read_dict(thermo_path, Th, err)) return rc;
    m = MechanismData{};
    {
        auto slash = reactions_path.find_last_of('/');
        std::string base = slash == std::string::npos ? reactions_path : reactions_path.substr(slash + 1);
        m.name = base.substr(0, base.find('.'));
    }
    FoamReader rd{m, err, reactions_path};
    const Entry* sp = R.find("species");
    if (!sp || sp->dict) return rd.fail(CHEM_E_PARSE, "species", "needs a species list");
    const auto names = list_words(sp->toks);
    if (names.empty()) return rd.fail(CHEM_E_MECH_INVALID, "species", "no species");
    // elements: the `elements` list if given, else in order of first use
    if (const Entry* el = R.find("elements"); el && !el->dict)
        for (auto& e : list_words(el->toks)) m.elements.push_back(e);
    rd.file = thermo_path;
    std::vector<std::map<std::string, int>> comps;
    for (const auto& nm : names) {
        if (rd.sp_index.count(nm)) return rd.fail(CHEM_E_PARSE, "species", nm + " listed twice");
        const Entry* se = Th.find(nm);
        if (!se || !se->dict) return rd.fail(CHEM_E_MECH_INVALID, nm, "no thermo entry");
        const Dict& d = *se->dict;
        SpeciesData s;
        s.name = nm;
        const Entry* spc = d.find("specie");
        const Entry* th = d.find("thermodynamics");
        const Entry* els = d.find("elements");
        double W = 0.0;
        if (!spc || !spc->dict) return rd.fail(CHEM_E_PARSE, nm, "needs specie { molWeight ...; }");
        if (int rc = rd.scalar(*spc->dict, "molWeight", W, nm)) return rc;
        if (!(W > 0.0)) return rd.fail(CHEM_E_MECH_INVALID, nm, "molWeight must be positive");
        s.W = W * 1e-3;   // kg/kmol -> kg/mol
        if (!th || !th->dict) return rd.fail(CHEM_E_PARSE, nm, "needs thermodynamics");
        double tl, th_, tc;
        if (int rc = rd.scalar(*th->dict, "Tlow", tl, nm)) return rc;
        if (int rc = rd.scalar(*th->dict, "Thigh", th_, nm)) return rc;
        if (int rc = rd.scalar(*th->dict, "Tcommon", tc, nm)) return rc;
        s.tmid = tc;
        for (auto [key, dst] : {std::pair<const char*, double*>{"lowCpCoeffs", s.lo}, {"highCpCoeffs", s.hi}}) {
            const Entry* c = th->dict->find(key);
            if (!c || c->dict) return rd.fail(CHEM_E_PARSE, nm, std::string("needs ") + key);
            auto w = list_words(c->toks);
            if (w.size() != 7) return rd.fail(CHEM_E_PARSE, nm, std::string(key) + " needs 7 values");
            for (int q = 0; q < 7; ++q)
                if (!num(w[q], dst[q])) return rd.fail(CHEM_E_PARSE, nm, std::string("bad value in ") + key);
        }
        if (!els || !els->dict) return rd.fail(CHEM_E_PARSE, nm, "needs elements");
        std::map<std::string, int> comp;
        for (auto& [e, ent] : els->dict->items) {
            double c;
            if (ent.dict || ent.toks.size() != 1 || !num(ent.toks[0], c) || c < 0.0 || c != std::floor(c))
                return rd.fail(CHEM_E_PARSE, nm, "bad element count of " + e);
            if (c == 0.0) continue;
            comp[e] = (int)c;
            bool known = false;
            for (auto& x : m.elements) known = known || x == e;
            if (!known) m.elements.push_back(e);
        }
        s.has_thermo = true;
        rd.sp_index[nm] = (int)m.species.size();
        m.species.push_back(std::move(s));
        comps.push_back(std::move(comp));
    }
    // compositions per element, once the element list is complete
    for (size_t q = 0; q < m.species.size(); ++q) {
        m.species[q].atoms.assign(m.elements.size(), 0);
        for (auto& [e, c] : comps[q])
            for (size_t k = 0; k < m.elements.size(); ++k)
                if (m.elements[k] == e) m.species[q].atoms[k] = c;
    }
    m.element_w.assign(m.elements.size(), 0.0);   // weights come from molWeight
    rd.file = reactions_path;
    const Entry* rx = R.find("reactions");
    if (!rx || !rx->dict) return rd.fail(CHEM_E_PARSE, "reactions", "needs a reactions dictionary");
    for (auto& [name, e] : rx->dict->items) {
        if (!e.dict) return rd.fail(CHEM_E_PARSE, name, "reaction entries are dictionaries");
        if (int rc = rd.reaction(name, *e.dict)) return rc;
    }
    return validate_mechanism(m, err);
}

}  // namespace chemmi
