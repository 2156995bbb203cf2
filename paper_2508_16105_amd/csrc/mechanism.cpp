// mechanism.cpp -- reader and validator for `chemmi-mech 1` files.
#include "mechanism.hpp"

#include <cmath>
#include <fstream>
#include <map>
#include <sstream>

#include "../../include/chem.h"

namespace chemmi {
namespace {

std::vector<std::string> split(const std::string& s, char sep)
{
    std::vector<std::string> out;
    std::string cur;
    for (char c : s) {
        if (c == sep) {
            out.push_back(cur);
            cur.clear();
        } else {
            cur.push_back(c);
        }
    }
    out.push_back(cur);
    return out;
}

bool to_double(const std::string& s, double& v)
{
    if (s.empty()) return false;
    char* end = nullptr;
    v = std::strtod(s.c_str(), &end);
    return end && *end == 0 && std::isfinite(v);
}

bool to_int(const std::string& s, int& v)
{
    if (s.empty()) return false;
    char* end = nullptr;
    long x = std::strtol(s.c_str(), &end, 10);
    if (!end || *end != 0 || x < -1000000 || x > 1000000) return false;
    v = (int)x;
    return true;
}

struct Reader {
    MechanismData& m;
    std::string& err;
    int line = 0;
    std::map<std::string, int> sp_index, el_index;

    int fail(int code, const std::string& msg)
    {
        err = "line " + std::to_string(line) + ": " + msg;
        return code;
    }

    int side(const std::string& txt, std::vector<Term>& out)
    {
        for (const auto& item : split(txt, ',')) {
            auto kv = split(item, '=');
            int nu = 0;
            if (kv.size() != 2 || !sp_index.count(kv[0]) || !to_int(kv[1], nu) || nu <= 0)
                return fail(CHEM_E_PARSE, "bad reaction side '" + txt + "'");
            out.push_back({sp_index[kv[0]], nu});
        }
        return out.empty() ? fail(CHEM_E_PARSE, "empty reaction side") : 0;
    }

    int reaction(const std::vector<std::string>& t)
    {
        ReactionData r;
        size_t need;
        if (t[1] == "elementary") { r.kind = RxnKind::Elementary; need = 7; }
        else if (t[1] == "thirdbody") { r.kind = RxnKind::ThirdBody; need = 7; }
        else if (t[1] == "lindemann") { r.kind = RxnKind::Lindemann; need = 10; }
        else if (t[1] == "troe") { r.kind = RxnKind::Troe; need = 14; }
        else if (t[1] == "sri") { r.kind = RxnKind::Sri; need = 15; }
        else if (t[1] == "plog") { r.kind = RxnKind::Plog; need = 7; }
        else return fail(CHEM_E_PARSE, "unknown reaction kind " + t[1]);
        if (t.size() < need) return fail(CHEM_E_PARSE, "wrong field count");
        // trailing flags, each at most once: eff=..., plog=..., irrev
        std::string eff_txt, plog_txt;
        bool irrev = false;
        for (size_t i = need; i < t.size(); ++i) {
            if (t[i].rfind("eff=", 0) == 0 && eff_txt.empty()) eff_txt = t[i].substr(4);
            else if (t[i].rfind("plog=", 0) == 0 && plog_txt.empty()) plog_txt = t[i].substr(5);
            else if (t[i] == "irrev" && !irrev) irrev = true;
            else return fail(CHEM_E_PARSE, "wrong field count or unknown flag '" + t[i] + "'");
        }
        if (!eff_txt.empty() && (r.kind == RxnKind::Elementary || r.kind == RxnKind::Plog))
            return fail(CHEM_E_PARSE, "efficiencies on a reaction without a third body");
        if ((r.kind == RxnKind::Plog) != !plog_txt.empty())
            return fail(CHEM_E_PARSE, "a plog= table belongs to (and only to) a plog reaction");
        r.reversible = !irrev;
        if (int rc = side(t[2], r.reac)) return rc;
        if (int rc = side(t[3], r.prod)) return rc;
        int order = 0;
        for (auto& x : r.reac) { order += x.nu; r.dnu -= x.nu; }
        for (auto& x : r.prod) r.dnu += x.nu;
        double A, b, Ea;
        if (!to_double(t[4], A) || !to_double(t[5], b) || !to_double(t[6], Ea))
            return fail(CHEM_E_PARSE, "bad Arrhenius numbers");
        if (!(A > 0.0)) return fail(CHEM_E_MECH_INVALID, "A must be positive");
        // cm-mol-s to SI: each concentration factor beyond the first carries
        // cm^3/mol; a plog reaction's main rate is a plain factor on its table
        const int orderA = r.kind == RxnKind::Plog ? 1 : order + (r.kind == RxnKind::ThirdBody ? 1 : 0);
        r.lnA = std::log(A) + (orderA - 1) * std::log(1e-6);
        r.b = b;
        r.EaR = Ea * 1e3 / kRu;
        r.eff.assign(m.species.size(), 1.0);
        if (is_falloff(r.kind)) {
            double A0, b0, Ea0;
            if (!to_double(t[7], A0) || !to_double(t[8], b0) || !to_double(t[9], Ea0))
                return fail(CHEM_E_PARSE, "bad low-pressure numbers");
            if (!(A0 > 0.0)) return fail(CHEM_E_MECH_INVALID, "A0 must be positive");
            r.lnA0 = std::log(A0) + order * std::log(1e-6);
            r.b0 = b0;
            r.EaR0 = Ea0 * 1e3 / kRu;
        }
        if (r.kind == RxnKind::Troe) {
            if (!to_double(t[10], r.alpha) || !to_double(t[11], r.T3) || !to_double(t[12], r.T1))
                return fail(CHEM_E_PARSE, "bad Troe numbers");
            r.has_T2 = t[13] != "-";
            if (r.has_T2 && !to_double(t[13], r.T2)) return fail(CHEM_E_PARSE, "bad Troe T2");
            if (!(r.T3 > 0.0) || !(r.T1 > 0.0))
                return fail(CHEM_E_MECH_INVALID, "Troe T3 and T1 must be positive");
        }
        if (r.kind == RxnKind::Sri) {
            for (int i = 0; i < 5; ++i)
                if (!to_double(t[10 + i], r.sri[i])) return fail(CHEM_E_PARSE, "bad SRI numbers");
            if (!(r.sri[0] >= 0.0) || !(r.sri[2] > 0.0) || !(r.sri[3] > 0.0))
                return fail(CHEM_E_MECH_INVALID, "SRI needs a >= 0, c > 0, d > 0");
        }
        if (r.kind == RxnKind::Plog) {
            for (const auto& item : split(plog_txt, ',')) {
                auto f = split(item, ':');
                double pp, pa, pb, pe;
                if (f.size() != 4 || !to_double(f[0], pp) || !to_double(f[1], pa) || !to_double(f[2], pb) ||
                    !to_double(f[3], pe))
                    return fail(CHEM_E_PARSE, "bad plog entry '" + item + "'");
                if (!(pp > 0.0) || !(pa > 0.0)) return fail(CHEM_E_MECH_INVALID, "plog p and A must be positive");
                const double lnp = std::log(pp);
                if (!r.plog.empty() && !(lnp > r.plog.back().lnp))
                    return fail(CHEM_E_MECH_INVALID, "plog pressures must increase");
                r.plog.push_back({lnp, std::log(pa) + (order - 1) * std::log(1e-6), pb, pe * 1e3 / kRu});
            }
            if (r.plog.size() > kMaxPlog) return fail(CHEM_E_UNSUPPORTED, "more than 16 plog pressures");
        }
        if (!eff_txt.empty()) {
            for (const auto& item : split(eff_txt, ',')) {
                auto kv = split(item, ':');
                double e;
                if (kv.size() != 2 || !sp_index.count(kv[0]) || !to_double(kv[1], e) || e < 0.0)
                    return fail(CHEM_E_PARSE, "bad efficiency '" + item + "'");
                r.eff[sp_index[kv[0]]] = e;
            }
        }
        if (int rc = balance(r)) return rc;
        m.reactions.push_back(std::move(r));
        return 0;
    }

    // element balance, exact in integers
    int balance(const ReactionData& r)
    {
        for (size_t e = 0; e < m.elements.size(); ++e) {
            long bal = 0;
            for (auto& x : r.reac) bal -= (long)x.nu * m.species[x.sp].atoms[e];
            for (auto& x : r.prod) bal += (long)x.nu * m.species[x.sp].atoms[e];
            if (bal != 0)
                return fail(CHEM_E_MECH_INVALID, "element " + m.elements[e] + " is not balanced");
        }
        return 0;
    }

    int record(const std::vector<std::string>& t)
    {
        const std::string& k = t[0];
        if (k == "name") {
            if (t.size() > 1) m.name = t[1];
            return 0;
        }
        if (k == "element") {
            double w;
            if (t.size() != 3 || !to_double(t[2], w) || !(w > 0.0) || el_index.count(t[1]))
                return fail(CHEM_E_PARSE, "bad element record");
            if (!m.species.empty()) return fail(CHEM_E_PARSE, "elements must precede species");
            el_index[t[1]] = (int)m.elements.size();
            m.elements.push_back(t[1]);
            m.element_w.push_back(w);
            return 0;
        }
        if (k == "species") {
            // species <name> <composition> [W=<molar mass g/mol>]
            if ((t.size() != 3 && t.size() != 4) || sp_index.count(t[1])) return fail(CHEM_E_PARSE, "bad species record");
            if (!m.reactions.empty()) return fail(CHEM_E_PARSE, "species must precede reactions");
            SpeciesData s;
            s.name = t[1];
            s.atoms.assign(m.elements.size(), 0);
            double w = 0.0;
            for (const auto& item : split(t[2], ',')) {
                auto kv = split(item, '=');
                int n = 0;
                if (kv.size() != 2 || !el_index.count(kv[0]) || !to_int(kv[1], n) || n <= 0)
                    return fail(CHEM_E_PARSE, "bad composition '" + item + "'");
                s.atoms[el_index[kv[0]]] += n;
                w += n * m.element_w[el_index[kv[0]]];
            }
            s.W = w * 1e-3;
            if (t.size() == 4) {
                double wg;
                if (t[3].rfind("W=", 0) != 0 || !to_double(t[3].substr(2), wg) || !(wg > 0.0))
                    return fail(CHEM_E_PARSE, "bad species weight '" + t[3] + "'");
                s.W = wg * 1e-3;
            }
            sp_index[s.name] = (int)m.species.size();
            m.species.push_back(std::move(s));
            return 0;
        }
        if (k == "thermo") {
            if (t.size() != 19 || !sp_index.count(t[1])) return fail(CHEM_E_PARSE, "bad thermo record");
            SpeciesData& s = m.species[sp_index[t[1]]];
            double tl, th;
            bool ok = to_double(t[2], tl) && to_double(t[3], s.tmid) && to_double(t[4], th);
            for (int i = 0; i < 7 && ok; ++i) ok = to_double(t[5 + i], s.lo[i]) && to_double(t[12 + i], s.hi[i]);
            if (!ok) return fail(CHEM_E_PARSE, "bad thermo numbers");
            s.has_thermo = true;
            return 0;
        }
        if (k == "reaction") {
            if (t.size() < 7) return fail(CHEM_E_PARSE, "short reaction record");
            return reaction(t);
        }
        return fail(CHEM_E_PARSE, "unknown record '" + k + "'");
    }
};

}  // namespace

int parse_mechanism(const std::string& path, MechanismData& m, std::string& err)
{
    std::ifstream in(path);
    if (!in) {
        err = "cannot open " + path;
        return CHEM_E_INVAL;
    }
    m = MechanismData{};
    Reader rd{m, err};
    std::string text;
    bool tag = false, ended = false;
    while (std::getline(in, text)) {
        ++rd.line;
        auto hash = text.find('#');
        if (hash != std::string::npos) text.resize(hash);
        std::istringstream ss(text);
        std::vector<std::string> tok;
        for (std::string w; ss >> w;) tok.push_back(w);
        if (tok.empty()) continue;
        if (!tag) {
            if (tok.size() != 2 || tok[0] != "chemmi-mech" || tok[1] != "1")
                return rd.fail(CHEM_E_PARSE, "missing 'chemmi-mech 1' header");
            tag = true;
            continue;
        }
        if (ended) return rd.fail(CHEM_E_PARSE, "text after 'end'");
        if (tok[0] == "end") {
            ended = true;
            continue;
        }
        if (int rc = rd.record(tok)) return rc;
    }
    if (!tag || !ended) {
        err = "truncated mechanism file (no 'end')";
        return CHEM_E_PARSE;
    }
    return validate_mechanism(m, err);
}

int validate_mechanism(MechanismData& m, std::string& err)
{
    if (m.species.empty()) {
        err = "no species";
        return CHEM_E_MECH_INVALID;
    }
    for (auto& s : m.species)
        if (!s.has_thermo) {
            err = "species " + s.name + " has no thermo data";
            return CHEM_E_MECH_INVALID;
        }
    if (m.species.size() > CHEM_MAX_SPECIES) {
        err = "more than " + std::to_string(CHEM_MAX_SPECIES) + " species";
        return CHEM_E_UNSUPPORTED;
    }
    return 0;
}

std::vector<double> pack_params(const MechanismData& m)
{
    const int nr = m.nr();
    std::vector<double> p(3 * (size_t)nr);
    for (int j = 0; j < nr; ++j) {
        p[j] = m.reactions[j].lnA;
        p[nr + j] = m.reactions[j].b;
        p[2 * nr + j] = m.reactions[j].EaR;
    }
    return p;
}

}  // namespace chemmi
