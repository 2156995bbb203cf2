// capi.cpp -- the C ABI (include/chem.h): argument checks, per-device state,
// and the launches of the plain, source-term and fixed-step kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <memory>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/chem.h"
#include "codegen.hpp"
#include "mechanism.hpp"
#include "module.hpp"
#include "runtime.hpp"

using namespace chemmi;

namespace {
// a cell's state, Jacobian and LU factors live in one lane's registers
// Mechanisms with up to kLaneSpecies species run one cell per lane (the
// cell's Jacobian and LU factors in one lane's registers); larger ones run
// wave-cooperatively.  At 13 species the lane form spills registers but keeps
// 64 cells in flight per SIMD against 8, and wins on large fields (28 M cells:
// 7.2 s against 9.4 s); the wave-cooperative form has the shorter latency per
// cell.  From 14 species on, the lane form's spills grow steeply and the
// wave-cooperative form is 3-4x faster even on a 65 k-cell field (14, 15, 16
// and 18 species measured), so 13 is the default limit.
// CHEM_LANE_MAX_SPECIES overrides the choice at load time (the lane form is
// built for at most kMaxLaneSpecies species).
constexpr int kLaneSpecies = 13;
constexpr int kMaxLaneSpecies = 20;

int lane_max_species()
{
    const char* e = std::getenv("CHEM_LANE_MAX_SPECIES");
    if (e && *e) {
        const int v = std::atoi(e);
        if (v >= 0) return std::min(v, kMaxLaneSpecies);
    }
    return kLaneSpecies;
}

}  // namespace

namespace chemmi {

thread_local std::string g_last_error;

int set_error(int code, const std::string& msg)
{
    g_last_error = msg;
    if (std::getenv("CHEM_LOG")) std::fprintf(stderr, "[chem] error %d: %s\n", code, msg.c_str());
    return code;
}

int hip_error(hipError_t e, const char* what)
{
    return set_error(e == hipErrorOutOfMemory ? CHEM_E_NOMEM : CHEM_E_HIP,
                     std::string(what) + ": " + hipGetErrorString(e));
}

bool is_device_ptr(const void* p)
{
    if (!p) return false;
    hipPointerAttribute_t a;
    if (hipPointerGetAttributes(&a, p) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged || a.isManaged;
}

int check_device_ptrs(std::initializer_list<std::pair<const void*, const char*>> ptrs)
{
    for (auto& pr : ptrs)
        if (!is_device_ptr(pr.first))
            return set_error(CHEM_E_INVAL, std::string(pr.second) + " is not a device pointer");
    return 0;
}

int check_tolerances(double dt, double rtol, double atol)
{
    if (!(dt > 0.0) || !std::isfinite(dt)) return set_error(CHEM_E_INVAL, "dt must be positive and finite");
    if (!(rtol > 0.0) || !std::isfinite(rtol)) return set_error(CHEM_E_INVAL, "rtol must be positive");
    if (!(atol >= 0.0) || !std::isfinite(atol)) return set_error(CHEM_E_INVAL, "atol must be >= 0");
    return 0;
}

Options resolve_options(const chem_options* o)
{
    Options r;
    if (o) {
        r.form = o->form;
        if (o->max_substeps > 0) r.max_substeps = o->max_substeps;
        if (o->hmin_rel > 0.0) r.hmin_rel = o->hmin_rel;
        r.h0 = o->h0;
        if (o->checkpoint_every > 0) r.checkpoint_every = o->checkpoint_every;
        r.block = o->block;
        r.waves_per_simd = o->waves_per_simd;
        r.refill = o->refill;
        r.order = o->order;
        r.cost = o->cost;
        r.adjoint_nacc = o->adjoint_nacc;
    }
    return r;
}

}  // namespace chemmi

namespace {

int finish_load(std::unique_ptr<chem_mechanism> m, chem_mechanism** out)
{
    std::string err;
    if (m->data.ns() > CHEM_MAX_SPECIES)
        return set_error(CHEM_E_UNSUPPORTED, "more than " + std::to_string(CHEM_MAX_SPECIES) + " species");
    m->params = pack_params(m->data);
    if (m->data.ns() <= lane_max_species()) {
        // the exponent conversion that saves two instructions per exp also
        // changes register allocation: in the one-cell-per-lane kernels of
        // mechanisms above 9 species, which spill, it raised the spill
        // (13 species: 1,392 -> 1,604 B per lane) and the run time (+18 %),
        // so those keep the clamped conversion
        m->source = device_source(generate_mechanism_source(m->data), false, m->data.ns() + 1 <= 10);
    } else {
        m->layout = wide_layout(m->data);
        if (m->layout.G == 0)
            return set_error(CHEM_E_UNSUPPORTED, "mechanism outside the wave-cooperative tables (over 3 terms or a "
                                                     "coefficient over 3 on a reaction side, |dnu| over 4, or over "
                                                     "511 third-body or falloff reactions, or over 511 PLOG reactions)");
        m->wide = true;
        m->source = device_source(generate_wide_source(m->data, m->layout), true, true);
    }
    if (int rc = build_code_object(m->source, m->code, err, &m->cache_file)) return set_error(rc, err);
    // with a gfx950 device current, load the code there now, so that the
    // allocation-free entry point finds it set up
    prepare_current_device(m.get());
    *out = m.release();
    return CHEM_OK;
}

// First word of the file that is not blank or a comment ('#' or '!').
std::string first_word(const char* path)
{
    std::ifstream in(path);
    std::string line;
    while (std::getline(in, line)) {
        for (char c : {'#', '!'}) {
            auto k = line.find(c);
            if (k != std::string::npos) line.resize(k);
        }
        std::istringstream ss(line);
        std::string w;
        if (ss >> w) return w;
    }
    return "";
}

}  // namespace

extern "C" {

const char* chem_last_error(void) { return g_last_error.c_str(); }

const char* chem_version(void) { return "chemmi 0.1 (gfx950, RODAS4, FP64)"; }

int chem_load_mechanism(const char* path, chem_mechanism** out)
{
    g_last_error.clear();
    if (!path || !out) return set_error(CHEM_E_INVAL, "null argument");
    *out = nullptr;
    auto m = std::make_unique<chem_mechanism>();
    std::string err;
    std::string w = first_word(path);
    for (auto& c : w) c = (char)std::toupper((unsigned char)c);
    const bool chemkin = w == "ELEMENTS" || w == "ELEM" || w == "SPECIES" || w == "SPEC" || w == "THERMO";
    if (int rc = chemkin ? parse_chemkin(path, "", m->data, err) : parse_mechanism(path, m->data, err))
        return set_error(rc, err);
    return finish_load(std::move(m), out);
}

int chem_load_openfoam(const char* reactions_path, const char* thermo_path, chem_mechanism** out)
{
    g_last_error.clear();
    if (!reactions_path || !thermo_path || !out) return set_error(CHEM_E_INVAL, "null argument");
    *out = nullptr;
    auto m = std::make_unique<chem_mechanism>();
    std::string err;
    if (int rc = parse_openfoam(reactions_path, thermo_path, m->data, err)) return set_error(rc, err);
    return finish_load(std::move(m), out);
}

int chem_load_chemkin(const char* mech_path, const char* thermo_path, chem_mechanism** out)
{
    g_last_error.clear();
    if (!mech_path || !out) return set_error(CHEM_E_INVAL, "null argument");
    *out = nullptr;
    auto m = std::make_unique<chem_mechanism>();
    std::string err;
    if (int rc = parse_chemkin(mech_path, thermo_path ? thermo_path : "", m->data, err)) return set_error(rc, err);
    return finish_load(std::move(m), out);
}

void chem_free_mechanism(chem_mechanism* m)
{
    if (!m) return;
    release_device_state(m);
    delete m;
}

int chem_mechanism_info(const chem_mechanism* m, int* ns, int* nr)
{
    if (!m) return set_error(CHEM_E_INVAL, "null mechanism");
    if (ns) *ns = m->data.ns();
    if (nr) *nr = m->data.nr();
    return CHEM_OK;
}

int chem_get_params(const chem_mechanism* m, double* lnA, double* b, double* Ea)
{
    if (!m || !lnA || !b || !Ea) return set_error(CHEM_E_INVAL, "null argument");
    const int nr = m->data.nr();
    for (int j = 0; j < nr; ++j) {
        lnA[j] = m->params[j];
        b[j] = m->params[nr + j];
        Ea[j] = m->params[2 * nr + j] * kRu;
    }
    return CHEM_OK;
}

namespace {
// Records the end of a call's work on its stream when the call returns (under
// the handle's lock), so the next call is ordered after it.
struct DoneMark {
    chem_mechanism* m;
    hipStream_t stream;
    ~DoneMark() { chemmi::mark_done(m, stream); }
};
}  // namespace

int chem_set_params(chem_mechanism* m, const double* lnA, const double* b, const double* Ea)
{
    if (!m || !lnA || !b || !Ea) return set_error(CHEM_E_INVAL, "null argument");
    const int nr = m->data.nr();
    for (int j = 0; j < nr; ++j)
        if (!std::isfinite(lnA[j]) || !std::isfinite(b[j]) || !std::isfinite(Ea[j]))
            return set_error(CHEM_E_INVAL, "non-finite parameter");
    std::lock_guard<std::mutex> lk(m->mu);
    for (int j = 0; j < nr; ++j) {
        m->params[j] = lnA[j];
        m->params[nr + j] = b[j];
        m->params[2 * nr + j] = Ea[j] / kRu;
    }
    ++m->params_version;
    return CHEM_OK;
}

int chem_eval_source(const chem_mechanism* mc, int64_t ncell, const double* T, const double* p,
                     const double* Y, double* f, double* J, void* stream)
{
    g_last_error.clear();
    auto* m = const_cast<chem_mechanism*>(mc);
    if (!m || ncell < 0) return set_error(CHEM_E_INVAL, "bad mechanism or ncell");
    if (ncell == 0) return CHEM_OK;
    if (int rc = check_device_ptrs({{T, "T"}, {p, "p"}, {Y, "Y"}, {f, "f"}})) return rc;
    if (J && !is_device_ptr(J)) return set_error(CHEM_E_INVAL, "J is not a device pointer");
    std::lock_guard<std::mutex> lk(m->mu);
    DoneMark mark{m, (hipStream_t)stream};
    DeviceState* d;
    if (int rc = device_state(m, (hipStream_t)stream, &d)) return rc;
    EvalArgs a{d->par, T, p, Y, (long)ncell, f, J};
    if (m->wide)
        return launch_1d(d->f_eval, ncell * m->layout.G, 64, &a, sizeof a, (hipStream_t)stream, "chem_eval",
                         m->layout.lds_bytes());
    return launch_1d(d->f_eval, ncell, 64, &a, sizeof a, (hipStream_t)stream, "chem_eval");
}

int chem_step_fixed(const chem_mechanism* mc, int64_t ncell, const double* T, const double* p,
                    const double* Y, double h, double rtol, double atol, double* ynew,
                    double* errnorm, int32_t* ok, void* stream)
{
    g_last_error.clear();
    auto* m = const_cast<chem_mechanism*>(mc);
    if (!m || ncell < 0) return set_error(CHEM_E_INVAL, "bad mechanism or ncell");
    if (int rc = check_tolerances(h, rtol, atol)) return rc;
    if (ncell == 0) return CHEM_OK;
    if (int rc = check_device_ptrs({{T, "T"}, {p, "p"}, {Y, "Y"}, {ynew, "ynew"},
                                    {errnorm, "errnorm"}, {ok, "ok"}}))
        return rc;
    std::lock_guard<std::mutex> lk(m->mu);
    DoneMark mark{m, (hipStream_t)stream};
    DeviceState* d;
    if (int rc = device_state(m, (hipStream_t)stream, &d)) return rc;
    FixedStepArgs a{d->par, T, p, Y, (long)ncell, h, ynew, errnorm, rtol, atol, ok};
    if (m->wide)
        return launch_1d(d->f_fixed, ncell * m->layout.G, 64, &a, sizeof a, (hipStream_t)stream, "chem_fixed_step",
                         m->layout.lds_bytes());
    return launch_1d(d->f_fixed, ncell, 64, &a, sizeof a, (hipStream_t)stream, "chem_fixed_step",
                     d->stage_lds(64));
}

int chem_integrate(const chem_mechanism* mc, int64_t ncell, double* T, const double* p, double* Y,
                   double dt, double rtol, double atol, const chem_options* opt, chem_stats* stats,
                   int32_t* cell_status, int32_t* nacc, int32_t* nrej, void* stream)
{
    g_last_error.clear();
    auto* m = const_cast<chem_mechanism*>(mc);
    if (!m || ncell < 0) return set_error(CHEM_E_INVAL, "bad mechanism or ncell");
    if (int rc = check_tolerances(dt, rtol, atol)) return rc;
    if (stats) std::memset(stats, 0, sizeof *stats);
    if (ncell == 0) return CHEM_OK;
    if (int rc = check_device_ptrs({{T, "T"}, {p, "p"}, {Y, "Y"}})) return rc;
    for (auto pr : {std::make_pair((const void*)cell_status, "cell_status"),
                    std::make_pair((const void*)nacc, "nacc"), std::make_pair((const void*)nrej, "nrej")})
        if (pr.first && !is_device_ptr(pr.first))
            return set_error(CHEM_E_INVAL, std::string(pr.second) + " is not a device pointer");
    Options o = resolve_options(opt);
    if (o.h0 && !is_device_ptr(o.h0)) return set_error(CHEM_E_INVAL, "h0 is not a device pointer");
    std::lock_guard<std::mutex> lk(m->mu);
    DoneMark mark{m, (hipStream_t)stream};
    if (o.form == CHEM_FORM_PERSISTENT) {
        const int32_t* cost = o.cost ? o.cost[0] : nullptr;
        if (cost && !is_device_ptr(cost)) return set_error(CHEM_E_INVAL, "cost[0] is not a device pointer");
        FieldView fv{T, p, Y, ncell, cell_status, nacc, nrej, o.h0, cost};
        return run_persistent(m, &fv, 1, dt, rtol, atol, o, stats, (hipStream_t)stream);
    }
    return run_plain(m, ncell, T, p, Y, dt, rtol, atol, o, stats, cell_status, nacc, nrej,
                     (hipStream_t)stream);
}

int chem_integrate_noalloc(const chem_mechanism* mc, int64_t ncell, double* T, const double* p, double* Y,
                           double dt, double rtol, double atol, const chem_options* opt, int32_t* cell_status,
                           int32_t* nacc, int32_t* nrej, void* stream)
{
    g_last_error.clear();
    auto* m = const_cast<chem_mechanism*>(mc);
    if (!m || ncell < 0) return set_error(CHEM_E_INVAL, "bad mechanism or ncell");
    if (int rc = check_tolerances(dt, rtol, atol)) return rc;
    if ((uint64_t)ncell > (uint64_t)CHEM_NOALLOC_MAX_CELLS)
        return set_error(CHEM_E_INVAL, "ncell exceeds CHEM_NOALLOC_MAX_CELLS");
    if (ncell == 0) return CHEM_OK;
    if (int rc = check_device_ptrs({{T, "T"}, {p, "p"}, {Y, "Y"}})) return rc;
    for (auto pr : {std::make_pair((const void*)cell_status, "cell_status"),
                    std::make_pair((const void*)nacc, "nacc"), std::make_pair((const void*)nrej, "nrej")})
        if (pr.first && !is_device_ptr(pr.first))
            return set_error(CHEM_E_INVAL, std::string(pr.second) + " is not a device pointer");
    Options o = resolve_options(opt);
    if (o.h0) return set_error(CHEM_E_INVAL, "h0 is not supported by the allocation-free (persistent) form");
    if (o.cost && o.cost[0] && !is_device_ptr(o.cost[0])) return set_error(CHEM_E_INVAL, "cost[0] is not a device pointer");
    std::lock_guard<std::mutex> lk(m->mu);
    DoneMark mark{m, (hipStream_t)stream};
    return run_noalloc(m, ncell, T, p, Y, dt, rtol, atol, o, cell_status, nacc, nrej, (hipStream_t)stream);
}

int chem_integrate_source(const chem_mechanism* mc, int64_t ncell, double* T, const double* p, double* Y,
                          double dt, double rtol, double atol, double* wdot, double* qdot,
                          const chem_options* opt, chem_stats* stats, int32_t* cell_status, void* stream)
{
    g_last_error.clear();
    auto* m = const_cast<chem_mechanism*>(mc);
    if (!m || ncell < 0) return set_error(CHEM_E_INVAL, "bad mechanism or ncell");
    if (int rc = check_tolerances(dt, rtol, atol)) return rc;
    if (stats) std::memset(stats, 0, sizeof *stats);
    if (ncell == 0) return CHEM_OK;
    if (int rc = check_device_ptrs({{T, "T"}, {p, "p"}, {Y, "Y"}, {wdot, "wdot"}, {qdot, "qdot"}})) return rc;
    if (cell_status && !is_device_ptr(cell_status)) return set_error(CHEM_E_INVAL, "cell_status is not a device pointer");
    Options o = resolve_options(opt);
    if (o.h0 && !is_device_ptr(o.h0)) return set_error(CHEM_E_INVAL, "h0 is not a device pointer");
    if (o.form == CHEM_FORM_PERSISTENT && o.cost && o.cost[0] && !is_device_ptr(o.cost[0]))
        return set_error(CHEM_E_INVAL, "cost[0] is not a device pointer");
    std::lock_guard<std::mutex> lk(m->mu);
    DoneMark mark{m, (hipStream_t)stream};
    return run_source(m, ncell, T, p, Y, dt, rtol, atol, o, stats, cell_status, wdot, qdot, (hipStream_t)stream);
}

int chem_euler1d_init(const chem_mechanism* mc, int64_t ncell, const double* T, const double* p,
                      const double* Y, const double* u, double* U, void* stream)
{
    g_last_error.clear();
    auto* m = const_cast<chem_mechanism*>(mc);
    if (!m || ncell < 0) return set_error(CHEM_E_INVAL, "bad mechanism or ncell");
    if (ncell == 0) return CHEM_OK;
    if (int rc = check_device_ptrs({{T, "T"}, {p, "p"}, {Y, "Y"}, {U, "U"}})) return rc;
    if (u && !is_device_ptr(u)) return set_error(CHEM_E_INVAL, "u is not a device pointer");
    std::lock_guard<std::mutex> lk(m->mu);
    DoneMark mark{m, (hipStream_t)stream};
    return run_euler1d_init(m, ncell, T, p, Y, u, U, (hipStream_t)stream);
}

int chem_euler1d_step(const chem_mechanism* mc, int64_t ncell, double dx, double dt, const double* U,
                      double* U_out, double* T, double rtol, double atol, const chem_options* opt,
                      chem_stats* stats, double* max_cfl, void* stream)
{
    g_last_error.clear();
    auto* m = const_cast<chem_mechanism*>(mc);
    if (!m || ncell < 1) return set_error(CHEM_E_INVAL, "bad mechanism or ncell");
    if (!(dx > 0.0) || !std::isfinite(dx)) return set_error(CHEM_E_INVAL, "dx must be positive");
    if (int rc = check_tolerances(dt, rtol, atol)) return rc;
    if (stats) std::memset(stats, 0, sizeof *stats);
    if (int rc = check_device_ptrs({{U, "U"}, {U_out, "U_out"}, {T, "T"}})) return rc;
    if (U == U_out) return set_error(CHEM_E_INVAL, "U_out must not be U");
    Options o = resolve_options(opt);
    if (o.h0) return set_error(CHEM_E_INVAL, "h0 is not used by the 1D driver");
    std::lock_guard<std::mutex> lk(m->mu);
    DoneMark mark{m, (hipStream_t)stream};
    return run_euler1d(m, ncell, dx, dt, U, U_out, T, rtol, atol, o, stats, max_cfl, (hipStream_t)stream);
}

int chem_integrate_batched(const chem_mechanism* mc, int nfield, double* const* T,
                           const double* const* p, double* const* Y, const int64_t* ncell, double dt,
                           double rtol, double atol, const chem_options* opt, chem_stats* stats,
                           void* stream)
{
    g_last_error.clear();
    auto* m = const_cast<chem_mechanism*>(mc);
    if (!m || nfield < 0 || (nfield > 0 && (!T || !p || !Y || !ncell)))
        return set_error(CHEM_E_INVAL, "bad arguments");
    if (int rc = check_tolerances(dt, rtol, atol)) return rc;
    if (stats) std::memset(stats, 0, sizeof *stats);
    std::vector<FieldView> fields;
    for (int f = 0; f < nfield; ++f) {
        if (ncell[f] < 0) return set_error(CHEM_E_INVAL, "negative field size");
        if (ncell[f] == 0) continue;
        if (int rc = check_device_ptrs({{T[f], "T[f]"}, {p[f], "p[f]"}, {Y[f], "Y[f]"}})) return rc;
        fields.push_back(FieldView{T[f], p[f], Y[f], ncell[f], nullptr, nullptr, nullptr, nullptr, nullptr});
    }
    if (fields.empty()) return CHEM_OK;
    Options o = resolve_options(opt);
    if (o.cost) {
        int i = 0;
        for (int f = 0; f < nfield; ++f) {
            if (ncell[f] == 0) continue;
            if (o.cost[f] && !is_device_ptr(o.cost[f]))
                return set_error(CHEM_E_INVAL, "cost[f] is not a device pointer");
            fields[i++].cost = o.cost[f];
        }
    }
    if (o.h0) return set_error(CHEM_E_INVAL, "h0 is per field; not supported by the batched call");
    std::lock_guard<std::mutex> lk(m->mu);
    DoneMark mark{m, (hipStream_t)stream};
    if (o.form == CHEM_FORM_PLAIN) {
        chem_stats total{};
        for (auto& fv : fields) {
            chem_stats s{};
            int rc = run_plain(m, fv.ncell, fv.T, fv.p, fv.Y, dt, rtol, atol, o, stats ? &s : nullptr,
                               nullptr, nullptr, nullptr, (hipStream_t)stream);
            if (rc && rc != CHEM_E_CELL_FAILED) return rc;
            total.cells += s.cells;
            total.accepted += s.accepted;
            total.rejected += s.rejected;
            total.failed += s.failed;
            total.max_substeps = std::max(total.max_substeps, s.max_substeps);
            total.kernel_ms += s.kernel_ms;
        }
        if (stats) {
            *stats = total;
            if (total.failed) return set_error(CHEM_E_CELL_FAILED, "some cells failed");
        }
        return CHEM_OK;
    }
    return run_persistent(m, fields.data(), (int)fields.size(), dt, rtol, atol, o, stats,
                          (hipStream_t)stream);
}

int chem_integrate_adjoint(const chem_mechanism* mc, int64_t ncell, const double* T0, const double* p,
                           const double* Y0, double dt, double rtol, double atol, const double* gT,
                           const double* gY, double* gT0, double* gY0, double* g_lnA, double* g_b,
                           double* g_Ea, double* T_end, double* Y_end, const chem_options* opt,
                           chem_stats* stats, void* stream)
{
    g_last_error.clear();
    auto* m = const_cast<chem_mechanism*>(mc);
    if (!m || ncell < 0) return set_error(CHEM_E_INVAL, "bad mechanism or ncell");
    if (int rc = check_tolerances(dt, rtol, atol)) return rc;
    if (stats) std::memset(stats, 0, sizeof *stats);
    if (int rc = check_device_ptrs({{g_lnA, "g_lnA"}, {g_b, "g_b"}, {g_Ea, "g_Ea"}})) return rc;
    if (ncell > 0)
        if (int rc = check_device_ptrs({{T0, "T0"}, {p, "p"}, {Y0, "Y0"}, {gT, "gT"}, {gY, "gY"},
                                        {gT0, "gT0"}, {gY0, "gY0"}}))
            return rc;
    if ((T_end && !is_device_ptr(T_end)) || (Y_end && !is_device_ptr(Y_end)))
        return set_error(CHEM_E_INVAL, "T_end/Y_end is not a device pointer");
    if (!T_end != !Y_end) return set_error(CHEM_E_INVAL, "give both T_end and Y_end or neither");
    Options o = resolve_options(opt);
    if (o.adjoint_nacc && ncell > 0 && !is_device_ptr(o.adjoint_nacc))
        return set_error(CHEM_E_INVAL, "adjoint_nacc is not a device pointer");
    if (o.h0 && !is_device_ptr(o.h0)) return set_error(CHEM_E_INVAL, "h0 is not a device pointer");
    std::lock_guard<std::mutex> lk(m->mu);
    DoneMark mark{m, (hipStream_t)stream};
    const int ns = m->data.ns();
    double *Te = T_end, *Ye = Y_end;
    void* own = nullptr;
    if (!Te && ncell > 0) {
        hipError_t e = hipMalloc(&own, sizeof(double) * (size_t)ncell * (ns + 1));
        if (e != hipSuccess) return hip_error(e, "hipMalloc T_end/Y_end");
        Te = (double*)own;
        Ye = Te + ncell;
    }
    int rc = run_adjoint(m, ncell, T0, p, Y0, dt, rtol, atol, gT, gY, gT0, gY0, g_lnA, g_b, g_Ea, Te, Ye, o,
                         stats, (hipStream_t)stream);
    if (own) {
        (void)hipStreamSynchronize((hipStream_t)stream);
        (void)hipFree(own);
    }
    return rc;
}

}  // extern "C"
