/*
 * abi.c -- the chemistry-step C ABI (oracle_abi.h) on top of the oracle's own
 * functions (oracle.h): argument checks, status and statistics as the GPU
 * library's entry points define them, the computation itself unchanged.
 *
 * TEST INFRASTRUCTURE ONLY (see oracle.h).
 */
#include "oracle_abi.h"

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>

#include "oracle.h"
#include "oracle_internal.h"

struct oracle_mechanism {
    omech *m;
};

static _Thread_local char g_err[512];

static int fail(int code, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return code;
}

static double now_ms(void)
{
    struct timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return 1e3 * (double)ts.tv_sec + 1e-6 * (double)ts.tv_nsec;
}

static int check_tolerances(double dt, double rtol, double atol)
{
    if (!(dt > 0.0) || !isfinite(dt)) return fail(ORACLE_E_INVAL, "dt must be positive and finite");
    if (!(rtol > 0.0) || !isfinite(rtol)) return fail(ORACLE_E_INVAL, "rtol must be positive");
    if (!(atol >= 0.0) || !isfinite(atol)) return fail(ORACLE_E_INVAL, "atol must be >= 0");
    return ORACLE_OK;
}

static om_opts resolve(const oracle_options *o)
{
    om_opts r = {OM_RODAS4, 0, 0.0};
    if (o) {
        r.max_substeps = o->max_substeps > 0 ? o->max_substeps : 0;
        r.hmin_rel = o->hmin_rel > 0.0 ? o->hmin_rel : 0.0;
    }
    return r;
}

static void tally(oracle_stats *s, int64_t ncell, const int32_t *st, const int32_t *na, const int32_t *nj,
                  double ms)
{
    memset(s, 0, sizeof *s);
    s->cells = ncell;
    for (int64_t c = 0; c < ncell; ++c) {
        s->accepted += na[c];
        s->rejected += nj[c];
        if (na[c] + nj[c] > s->max_substeps) s->max_substeps = na[c] + nj[c];
        s->failed += st[c] != OM_CELL_OK;
    }
    s->kernel_ms = ms;
}

int oracle_load_mechanism(const char *path, oracle_mechanism **out)
{
    g_err[0] = 0;
    if (!path || !out) return fail(ORACLE_E_INVAL, "null argument");
    *out = NULL;
    char msg[400] = "";
    omech *m = NULL;
    const int rc = om_load(path, &m, msg, (int)sizeof msg);
    switch (rc) {
    case OM_OK: break;
    case OM_E_IO: return fail(ORACLE_E_INVAL, "%s", msg);
    case OM_E_PARSE: return fail(ORACLE_E_PARSE, "%s", msg);
    case OM_E_INVALID: return fail(ORACLE_E_MECH_INVALID, "%s", msg);
    case OM_E_SIZE: return fail(ORACLE_E_UNSUPPORTED, "%s", msg);
    default: return fail(ORACLE_E_PARSE, "%s", msg);
    }
    oracle_mechanism *h = malloc(sizeof *h);
    if (!h) {
        om_free(m);
        return fail(ORACLE_E_INVAL, "out of host memory");
    }
    h->m = m;
    *out = h;
    return ORACLE_OK;
}

void oracle_free_mechanism(oracle_mechanism *h)
{
    if (!h) return;
    om_free(h->m);
    free(h);
}

int oracle_mechanism_info(const oracle_mechanism *h, int *n_species, int *n_reactions)
{
    g_err[0] = 0;
    if (!h) return fail(ORACLE_E_INVAL, "null mechanism");
    if (n_species) *n_species = om_nspecies(h->m);
    if (n_reactions) *n_reactions = om_nreactions(h->m);
    return ORACLE_OK;
}

int oracle_get_params(const oracle_mechanism *h, double *lnA, double *b, double *Ea)
{
    g_err[0] = 0;
    if (!h || !lnA || !b || !Ea) return fail(ORACLE_E_INVAL, "null argument");
    om_params(h->m, lnA, b, Ea);
    return ORACLE_OK;
}

int oracle_set_params(oracle_mechanism *h, const double *lnA, const double *b, const double *Ea)
{
    g_err[0] = 0;
    if (!h || !lnA || !b || !Ea) return fail(ORACLE_E_INVAL, "null argument");
    const int nr = h->m->nr;
    for (int j = 0; j < nr; ++j)
        if (!isfinite(lnA[j]) || !isfinite(b[j]) || !isfinite(Ea[j]))
            return fail(ORACLE_E_INVAL, "non-finite parameter");
    for (int j = 0; j < nr; ++j) {
        h->m->par[j] = lnA[j];
        h->m->par[nr + j] = b[j];
        h->m->par[2 * nr + j] = Ea[j];
    }
    return ORACLE_OK;
}

int oracle_eval_source(const oracle_mechanism *h, int64_t ncell, const double *T, const double *p,
                       const double *Y, double *f, double *J)
{
    g_err[0] = 0;
    if (!h || ncell < 0) return fail(ORACLE_E_INVAL, "bad mechanism or ncell");
    if (ncell == 0) return ORACLE_OK;
    if (!T || !p || !Y || !f) return fail(ORACLE_E_INVAL, "null argument");
    const int ns = h->m->ns, n = ns + 1;
    for (int64_t c = 0; c < ncell; ++c) {
        double y[OM_NMAX];
        y[0] = T[c];
        memcpy(y + 1, Y + c * ns, sizeof(double) * ns);
        om_rhs(h->m, NULL, p[c], y, f + c * n);
        if (J) om_jac(h->m, NULL, p[c], y, J + c * n * n);
    }
    return ORACLE_OK;
}

int oracle_step_fixed(const oracle_mechanism *h, int64_t ncell, const double *T, const double *p,
                      const double *Y, double step, double rtol, double atol, double *ynew,
                      double *errnorm, int32_t *ok)
{
    g_err[0] = 0;
    if (!h || ncell < 0) return fail(ORACLE_E_INVAL, "bad mechanism or ncell");
    int rc = check_tolerances(step, rtol, atol);
    if (rc) return rc;
    if (ncell == 0) return ORACLE_OK;
    if (!T || !p || !Y || !ynew || !errnorm || !ok) return fail(ORACLE_E_INVAL, "null argument");
    const int ns = h->m->ns, n = ns + 1;
    for (int64_t c = 0; c < ncell; ++c) {
        double y[OM_NMAX], err[OM_NMAX];
        y[0] = T[c];
        memcpy(y + 1, Y + c * ns, sizeof(double) * ns);
        double *yn = ynew + c * n;
        const int bad = om_step(h->m, NULL, OM_RODAS4, p[c], y, step, yn, err);
        double acc = 0.0;
        int good = !bad;
        for (int k = 0; k < n; ++k) {
            const double sc = atol + rtol * fmax(fabs(y[k]), fabs(yn[k]));
            acc += (err[k] / sc) * (err[k] / sc);
            good = good && isfinite(yn[k]);
        }
        errnorm[c] = sqrt(acc / n);
        ok[c] = good && isfinite(errnorm[c]);
    }
    return ORACLE_OK;
}

int oracle_integrate(const oracle_mechanism *h, int64_t ncell, double *T, const double *p, double *Y,
                     double dt, double rtol, double atol, const oracle_options *opt,
                     oracle_stats *stats, int32_t *cell_status, int32_t *nacc, int32_t *nrej)
{
    g_err[0] = 0;
    if (!h || ncell < 0) return fail(ORACLE_E_INVAL, "bad mechanism or ncell");
    int rc = check_tolerances(dt, rtol, atol);
    if (rc) return rc;
    if (stats) memset(stats, 0, sizeof *stats);
    if (ncell == 0) return ORACLE_OK;
    if (!T || !p || !Y) return fail(ORACLE_E_INVAL, "null argument");
    if (opt && opt->h0) return fail(ORACLE_E_UNSUPPORTED, "h0 is not supported by the oracle");
    const om_opts o = resolve(opt);
    int32_t *st = malloc(sizeof(int32_t) * 3 * (size_t)ncell);
    if (!st) return fail(ORACLE_E_INVAL, "out of host memory");
    int32_t *na = st + ncell, *nj = st + 2 * ncell;
    const double t0 = now_ms();
    om_integrate(h->m, NULL, (long)ncell, T, p, Y, dt, rtol, atol, &o, na, nj, st, 0);
    const double ms = now_ms() - t0;
    oracle_stats s;
    tally(&s, ncell, st, na, nj, ms);
    if (cell_status) memcpy(cell_status, st, sizeof(int32_t) * ncell);
    if (nacc) memcpy(nacc, na, sizeof(int32_t) * ncell);
    if (nrej) memcpy(nrej, nj, sizeof(int32_t) * ncell);
    free(st);
    if (stats) {
        *stats = s;
        if (s.failed) return fail(ORACLE_E_CELL_FAILED, "%lld cells failed", (long long)s.failed);
    }
    return ORACLE_OK;
}

int oracle_integrate_adjoint(const oracle_mechanism *h, int64_t ncell, const double *T0, const double *p,
                             const double *Y0, double dt, double rtol, double atol, const double *gT,
                             const double *gY, double *gT0, double *gY0, double *g_lnA, double *g_b,
                             double *g_Ea, double *T_end, double *Y_end, const oracle_options *opt,
                             oracle_stats *stats)
{
    g_err[0] = 0;
    if (!h || ncell < 0) return fail(ORACLE_E_INVAL, "bad mechanism or ncell");
    int rc = check_tolerances(dt, rtol, atol);
    if (rc) return rc;
    if (stats) memset(stats, 0, sizeof *stats);
    if (!g_lnA || !g_b || !g_Ea) return fail(ORACLE_E_INVAL, "null parameter gradient");
    if (ncell > 0 && (!T0 || !p || !Y0 || !gT || !gY || !gT0 || !gY0)) return fail(ORACLE_E_INVAL, "null argument");
    if (!T_end != !Y_end) return fail(ORACLE_E_INVAL, "give both T_end and Y_end or neither");
    if (opt && (opt->checkpoint_every > 16)) return fail(ORACLE_E_INVAL, "checkpoint_every must be 1..16");
    if (opt && opt->h0) return fail(ORACLE_E_UNSUPPORTED, "h0 is not supported by the oracle");
    const int ns = h->m->ns, nr = h->m->nr;
    if (ncell == 0) {
        for (int j = 0; j < nr; ++j) g_lnA[j] = g_b[j] = g_Ea[j] = 0.0;
        return ORACLE_OK;
    }
    const om_opts o = resolve(opt);
    /* the forward result and the per-cell statistics, from the same solve */
    double *Tw = malloc(sizeof(double) * (size_t)ncell * (ns + 1));
    int32_t *st = malloc(sizeof(int32_t) * 3 * (size_t)ncell);
    if (!Tw || !st) {
        free(Tw);
        free(st);
        return fail(ORACLE_E_INVAL, "out of host memory");
    }
    double *Yw = Tw + ncell;
    int32_t *na = st + ncell, *nj = st + 2 * ncell;
    memcpy(Tw, T0, sizeof(double) * ncell);
    memcpy(Yw, Y0, sizeof(double) * ncell * ns);
    const double t0 = now_ms();
    om_integrate(h->m, NULL, (long)ncell, Tw, p, Yw, dt, rtol, atol, &o, na, nj, st, 0);
    om_adjoint(h->m, OM_RODAS4, (long)ncell, T0, p, Y0, dt, rtol, atol, &o, gT, gY, gT0, gY0, g_lnA, g_b,
               g_Ea, 0);
    const double ms = now_ms() - t0;
    if (T_end) {                           /* bad-input cells were left untouched */
        memcpy(T_end, Tw, sizeof(double) * ncell);
        memcpy(Y_end, Yw, sizeof(double) * ncell * ns);
    }
    oracle_stats s;
    tally(&s, ncell, st, na, nj, ms);
    free(Tw);
    free(st);
    if (stats) *stats = s;
    if (s.failed) return fail(ORACLE_E_CELL_FAILED, "%lld cells failed", (long long)s.failed);
    return ORACLE_OK;
}

const char *oracle_last_error(void) { return g_err; }
