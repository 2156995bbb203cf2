/*
 * oracle.c -- plain CPU FP64 reference for the per-cell, constant-pressure,
 * adiabatic chemistry step: the species production rates (Appendix A eq. (21))
 * and heat release (eq. (20)) of the detailed-chemistry model (Sec. 2.1),
 * integrated over one flow step with an adaptive Rosenbrock method.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the test suite, the smoke check and the
 * benchmark's CPU-baseline leg, never by the product path.  Written plainly
 * (dense loops, textbook LU, no blocking or fusion) so it can be read against
 * the definitions; it shares no code with the GPU library.
 *
 * Readings of points the paper leaves open (it names only "detailed chemistry"
 * and "thermo data"):
 *   - ideal gas, constant pressure, adiabatic cell; state y = (T, Y_1..Y_ns);
 *   - NASA-7 two-range thermo, T >= T_mid uses the high set, no clamping;
 *   - modified Arrhenius k = A T^b exp(-Ea/RT), A given in cm-mol-s and
 *     converted to SI by (1e-6)^(order-1); every reaction reversible with
 *     k_r = k_f / K_c, K_c from NASA-7 Gibbs energies at 1 atm;
 *   - third-body [M] = sum eff_k C_k; Lindemann / Troe falloff, [M] entering
 *     falloff reactions only through P_r;
 *   - RODAS4 (Hairer & Wanner), RMS error norm over all n components with
 *     scale atol + rtol max(|y|, |y_new|); controller factor
 *     0.9 err^(-1/4) clipped to [0.2, 6], no growth right after a rejection.
 */
#include <complex.h>
#include <ctype.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include "oracle.h"

#include "oracle_internal.h"

/* ---------------- generic chemistry: real and complex instantiations ------------- */
#define S double
#define F(name) name##_d
#define EXP exp
#define LOG log
#define RE(x) (x)
#include "chem_generic.inc"
#undef S
#undef F
#undef EXP
#undef LOG
#undef RE

#define S double complex
#define F(name) name##_z
#define EXP cexp
#define LOG clog
#define RE(x) creal(x)
#include "chem_generic.inc"
#undef S
#undef F
#undef EXP
#undef LOG
#undef RE

/* ---------------- RODAS4 ----------------
 * Hairer & Wanner, Solving ODEs II (2nd ed., 1996), Sec. VI.4, method RODAS:
 * 6 stages, order 4 with an embedded order-3 estimate, stiffly accurate,
 * gamma = 1/4, in the transformed (u_i) form. */
static void tableau_rodas4(omtab *t)
{
    memset(t, 0, sizeof *t);
    t->s = 6;
    t->gamma = 0.25;
    t->a[1][0] = 1.544;
    t->a[2][0] = 0.9466785280815826;  t->a[2][1] = 0.2557011698983284;
    t->a[3][0] = 3.314825187068521;   t->a[3][1] = 2.896124015972201;
    t->a[3][2] = 0.9986419139977817;
    t->a[4][0] = 1.221224509226641;   t->a[4][1] = 6.019134481288629;
    t->a[4][2] = 12.53708332932087;   t->a[4][3] = -0.687886036105895;
    for (int j = 0; j < 4; ++j) t->a[5][j] = t->a[4][j];
    t->a[5][4] = 1.0;
    t->c[1][0] = -5.6688;
    t->c[2][0] = -2.430093356833875;  t->c[2][1] = -0.2063599157091915;
    t->c[3][0] = -0.1073529058151375; t->c[3][1] = -9.594562251023355;
    t->c[3][2] = -20.47028614809616;
    t->c[4][0] = 7.496443313967647;   t->c[4][1] = -10.24680431464352;
    t->c[4][2] = -33.99990352819905;  t->c[4][3] = 11.7089089320616;
    t->c[5][0] = 8.083246795921522;   t->c[5][1] = -7.981132988064893;
    t->c[5][2] = -31.52159432874371;  t->c[5][3] = 16.31930543123136;
    t->c[5][4] = -6.058818238834054;
    for (int j = 0; j < 4; ++j) t->m[j] = t->a[4][j];
    t->m[4] = 1.0;
    t->m[5] = 1.0;
    t->e[5] = 1.0;
}

/* ---------------- ROS4 ----------------
 * Hairer & Wanner, Solving ODEs II, Sec. IV.7 (Table 7.2, the L-stable
 * parameter set with gamma = 0.57282 of Shampine's 4-stage order-4(3)
 * family), transformed u-form.  Stage 4 has the same argument as stage 3,
 * so a method written for it needs three source evaluations per step; the
 * oracle simply evaluates it again. */
static void tableau_ros4(omtab *t)
{
    memset(t, 0, sizeof *t);
    t->s = 4;
    t->gamma = 0.57282;
    t->a[1][0] = 2.0;
    t->a[2][0] = 1.867943637803922;   t->a[2][1] = 0.2344449711399156;
    t->a[3][0] = 1.867943637803922;   t->a[3][1] = 0.2344449711399156;
    t->c[1][0] = -7.13761503641231;
    t->c[2][0] = 2.580708087951457;   t->c[2][1] = 0.6515950076447975;
    t->c[3][0] = -2.137148994382534;  t->c[3][1] = -0.3214669691237626;
    t->c[3][2] = -0.6949742501781779;
    t->m[0] = 2.255570073418735;      t->m[1] = 0.2870493262186792;
    t->m[2] = 0.435317943184018;      t->m[3] = 1.093502252409163;
    t->e[0] = -0.2815431932141155;    t->e[1] = -0.0727619912493892;
    t->e[2] = -0.1082196201495311;    t->e[3] = -1.093502252409163;
}

static int get_tableau(int method, omtab *t)
{
    if (method == OM_RODAS4) tableau_rodas4(t);
    else if (method == OM_ROS4) tableau_ros4(t);
    else return -1;
    return 0;
}

/* ---------------- mechanism file reader ---------------- */
static int find_species(const omech *m, const char *name)
{
    for (int k = 0; k < m->ns; ++k)
        if (strcmp(m->sname[k], name) == 0) return k;
    return -1;
}

static int find_element(const omech *m, const char *name)
{
    for (int e = 0; e < m->ne; ++e)
        if (strcmp(m->ename[e], name) == 0) return e;
    return -1;
}

/* "A=2,B=1" -> species indices and coefficients */
static int parse_side(const omech *m, char *txt, int *sp, int *nu, int *cnt)
{
    *cnt = 0;
    for (char *tok = strtok(txt, ","); tok; tok = strtok(NULL, ",")) {
        char *eq = strchr(tok, '=');
        if (!eq || *cnt >= OM_MAXSIDE) return -1;
        *eq = 0;
        int k = find_species(m, tok);
        int v = atoi(eq + 1);
        if (k < 0 || v <= 0) return -1;
        sp[*cnt] = k;
        nu[*cnt] = v;
        ++*cnt;
    }
    return *cnt > 0 ? 0 : -1;
}

#define FAIL(code, ...) do { snprintf(err, errlen, __VA_ARGS__); rc = code; goto done; } while (0)

int om_load(const char *path, omech **out, char *err, int errlen)
{
    int rc = OM_OK, lineno = 0;
    char line[8192];
    *out = NULL;
    FILE *fp = fopen(path, "r");
    if (!fp) { snprintf(err, errlen, "cannot open %s", path); return OM_E_IO; }
    omech *m = calloc(1, sizeof *m);
    int seen_tag = 0, ended = 0;
    while (fgets(line, sizeof line, fp)) {
        ++lineno;
        char *hash = strchr(line, '#');
        if (hash) *hash = 0;
        char *tok[64];
        int nt = 0;
        for (char *t = strtok(line, " \t\r\n"); t && nt < 64; t = strtok(NULL, " \t\r\n"))
            tok[nt++] = t;
        if (nt == 0) continue;
        if (!seen_tag) {
            if (nt != 2 || strcmp(tok[0], "chemmi-mech") || strcmp(tok[1], "1"))
                FAIL(OM_E_PARSE, "line %d: missing 'chemmi-mech 1' header", lineno);
            seen_tag = 1;
            continue;
        }
        if (ended) FAIL(OM_E_PARSE, "line %d: text after 'end'", lineno);
        if (!strcmp(tok[0], "name")) continue;
        if (!strcmp(tok[0], "end")) { ended = 1; continue; }
        if (!strcmp(tok[0], "element")) {
            if (nt != 3 || m->ne >= OM_NEMAX) FAIL(OM_E_PARSE, "line %d: bad element", lineno);
            snprintf(m->ename[m->ne], 8, "%s", tok[1]);
            m->ew[m->ne++] = atof(tok[2]);
        } else if (!strcmp(tok[0], "species")) {
            if ((nt != 3 && nt != 4) || m->ns >= OM_NSMAX) FAIL(OM_E_SIZE, "line %d: bad species", lineno);
            int k = m->ns++;
            snprintf(m->sname[k], 24, "%s", tok[1]);
            double w = 0.0;
            for (char *t = strtok(tok[2], ","); t; t = strtok(NULL, ",")) {
                char *eq = strchr(t, '=');
                if (!eq) FAIL(OM_E_PARSE, "line %d: bad composition", lineno);
                *eq = 0;
                int e = find_element(m, t);
                if (e < 0) FAIL(OM_E_PARSE, "line %d: unknown element %s", lineno, t);
                m->comp[k][e] += atoi(eq + 1);
                w += m->ew[e] * atoi(eq + 1);
            }
            m->W[k] = w * 1e-3;
            if (nt == 4) {                      /* W=<molar mass, g/mol> given explicitly */
                if (strncmp(tok[3], "W=", 2) || !(atof(tok[3] + 2) > 0.0))
                    FAIL(OM_E_PARSE, "line %d: bad species weight", lineno);
                m->W[k] = atof(tok[3] + 2) * 1e-3;
            }
        } else if (!strcmp(tok[0], "thermo")) {
            if (nt != 19) FAIL(OM_E_PARSE, "line %d: thermo needs 17 numbers", lineno);
            int k = find_species(m, tok[1]);
            if (k < 0) FAIL(OM_E_PARSE, "line %d: unknown species %s", lineno, tok[1]);
            m->tmid[k] = atof(tok[3]);
            for (int i = 0; i < 7; ++i) {
                m->lo[k][i] = atof(tok[5 + i]);
                m->hi[k][i] = atof(tok[12 + i]);
            }
            m->has_thermo[k] = 1;
        } else if (!strcmp(tok[0], "reaction")) {
            if (m->nr >= OM_NRMAX) FAIL(OM_E_SIZE, "line %d: too many reactions", lineno);
            omrxn *r = &m->rx[m->nr];
            memset(r, 0, sizeof *r);
            const char *kind = tok[1];
            int need;
            if (!strcmp(kind, "elementary")) { r->type = OMR_ELEMENTARY; need = 7; }
            else if (!strcmp(kind, "thirdbody")) { r->type = OMR_THIRDBODY; need = 7; }
            else if (!strcmp(kind, "lindemann")) { r->type = OMR_LINDEMANN; need = 10; }
            else if (!strcmp(kind, "troe")) { r->type = OMR_TROE; need = 14; }
            else if (!strcmp(kind, "sri")) { r->type = OMR_SRI; need = 15; }
            else if (!strcmp(kind, "plog")) { r->type = OMR_PLOG; need = 7; }
            else FAIL(OM_E_PARSE, "line %d: unknown reaction kind %s", lineno, kind);
            if (nt < need) FAIL(OM_E_PARSE, "line %d: wrong field count", lineno);
            /* optional trailing flags: eff=..., plog=..., irrev */
            char *efft = NULL, *plogt = NULL;
            for (int i = need; i < nt; ++i) {
                if (!strncmp(tok[i], "eff=", 4) && !efft) efft = tok[i] + 4;
                else if (!strncmp(tok[i], "plog=", 5) && !plogt) plogt = tok[i] + 5;
                else if (!strcmp(tok[i], "irrev") && !r->irrev) r->irrev = 1;
                else FAIL(OM_E_PARSE, "line %d: unknown field %s", lineno, tok[i]);
            }
            if (efft && (r->type == OMR_ELEMENTARY || r->type == OMR_PLOG))
                FAIL(OM_E_PARSE, "line %d: efficiencies without a third body", lineno);
            if ((r->type == OMR_PLOG) != (plogt != NULL))
                FAIL(OM_E_PARSE, "line %d: plog table and plog kind go together", lineno);
            if (parse_side(m, tok[2], r->rsp, r->rnu, &r->nre) ||
                parse_side(m, tok[3], r->psp, r->pnu, &r->np))
                FAIL(OM_E_PARSE, "line %d: bad reaction side", lineno);
            int order = 0;
            r->dnu = 0;
            for (int i = 0; i < r->nre; ++i) { order += r->rnu[i]; r->dnu -= r->rnu[i]; }
            for (int i = 0; i < r->np; ++i) r->dnu += r->pnu[i];
            double A = atof(tok[4]);
            if (!(A > 0.0)) FAIL(OM_E_INVALID, "line %d: A must be positive", lineno);
            /* cm^3/mol -> m^3/mol per concentration factor beyond the first; the
               main rate of a plog reaction is a plain factor on its table */
            int ordA = r->type == OMR_PLOG ? 1 : order + (r->type == OMR_THIRDBODY ? 1 : 0);
            r->lnA = log(A) + (ordA - 1) * log(1e-6);
            r->b = atof(tok[5]);
            r->Ea = atof(tok[6]) * 1e3;                           /* kJ/mol -> J/mol */
            for (int k = 0; k < OM_NSMAX; ++k) r->eff[k] = 1.0;
            if (r->type == OMR_LINDEMANN || r->type == OMR_TROE || r->type == OMR_SRI) {
                double A0 = atof(tok[7]);
                if (!(A0 > 0.0)) FAIL(OM_E_INVALID, "line %d: A0 must be positive", lineno);
                r->lnA0 = log(A0) + order * log(1e-6);           /* order + 1 - 1 */
                r->b0 = atof(tok[8]);
                r->Ea0 = atof(tok[9]) * 1e3;
            }
            if (r->type == OMR_TROE) {
                r->alpha = atof(tok[10]);
                r->T3 = atof(tok[11]);
                r->T1 = atof(tok[12]);
                r->has_T2 = strcmp(tok[13], "-") != 0;
                r->T2 = r->has_T2 ? atof(tok[13]) : 0.0;
                if (!(r->T3 > 0.0 && r->T1 > 0.0))
                    FAIL(OM_E_INVALID, "line %d: Troe T3, T1 must be positive", lineno);
            }
            if (r->type == OMR_SRI) {
                for (int i = 0; i < 5; ++i) r->sri[i] = atof(tok[10 + i]);
                if (!(r->sri[0] >= 0.0 && r->sri[2] > 0.0 && r->sri[3] > 0.0))
                    FAIL(OM_E_INVALID, "line %d: SRI needs a >= 0, c > 0, d > 0", lineno);
            }
            if (plogt) {
                for (char *t = strtok(plogt, ","); t; t = strtok(NULL, ",")) {
                    double v[4];
                    if (r->nplog >= OM_PLOGMAX) FAIL(OM_E_SIZE, "line %d: too many plog pressures", lineno);
                    if (sscanf(t, "%lf:%lf:%lf:%lf", &v[0], &v[1], &v[2], &v[3]) != 4)
                        FAIL(OM_E_PARSE, "line %d: bad plog entry", lineno);
                    if (!(v[0] > 0.0 && v[1] > 0.0)) FAIL(OM_E_INVALID, "line %d: plog p, A must be positive", lineno);
                    if (r->nplog && !(v[0] > r->plog_p[r->nplog - 1]))
                        FAIL(OM_E_INVALID, "line %d: plog pressures must increase", lineno);
                    r->plog_p[r->nplog] = v[0];
                    r->plog_lnA[r->nplog] = log(v[1]) + (order - 1) * log(1e-6);
                    r->plog_b[r->nplog] = v[2];
                    r->plog_Ea[r->nplog] = v[3] * 1e3;
                    r->nplog++;
                }
            }
            if (efft) {
                for (char *t = strtok(efft, ","); t; t = strtok(NULL, ",")) {
                    char *c = strchr(t, ':');
                    if (!c) FAIL(OM_E_PARSE, "line %d: bad efficiency", lineno);
                    *c = 0;
                    int k = find_species(m, t);
                    if (k < 0) FAIL(OM_E_PARSE, "line %d: unknown species %s", lineno, t);
                    r->eff[k] = atof(c + 1);
                }
            }
            /* element balance, exact in integers */
            for (int e = 0; e < m->ne; ++e) {
                int bal = 0;
                for (int i = 0; i < r->nre; ++i) bal -= r->rnu[i] * m->comp[r->rsp[i]][e];
                for (int i = 0; i < r->np; ++i) bal += r->pnu[i] * m->comp[r->psp[i]][e];
                if (bal) FAIL(OM_E_INVALID, "line %d: element %s not balanced", lineno, m->ename[e]);
            }
            m->nr++;
        } else {
            FAIL(OM_E_PARSE, "line %d: unknown record %s", lineno, tok[0]);
        }
    }
    if (!seen_tag || !ended) FAIL(OM_E_PARSE, "truncated mechanism file");
    if (m->ns == 0) FAIL(OM_E_INVALID, "no species");
    for (int k = 0; k < m->ns; ++k)
        if (!m->has_thermo[k]) FAIL(OM_E_INVALID, "species %s has no thermo", m->sname[k]);
    for (int j = 0; j < m->nr; ++j) {
        m->par[j] = m->rx[j].lnA;
        m->par[m->nr + j] = m->rx[j].b;
        m->par[2 * m->nr + j] = m->rx[j].Ea;
    }
done:
    fclose(fp);
    if (rc) { free(m); return rc; }
    *out = m;
    return OM_OK;
}

void om_free(omech *m) { free(m); }
int om_nspecies(const omech *m) { return m->ns; }
int om_nreactions(const omech *m) { return m->nr; }
void om_weights(const omech *m, double *W) { memcpy(W, m->W, sizeof(double) * m->ns); }
void om_params(const omech *m, double *lnA, double *b, double *Ea)
{
    memcpy(lnA, m->par, sizeof(double) * m->nr);
    memcpy(b, m->par + m->nr, sizeof(double) * m->nr);
    memcpy(Ea, m->par + 2 * m->nr, sizeof(double) * m->nr);
}

static const double *P(const omech *m, const double *par) { return par ? par : m->par; }

/* ---------------- point functions ---------------- */
void om_thermo(const omech *m, double T, double *cpR, double *HRT, double *SR)
{
    for (int k = 0; k < m->ns; ++k) thermo_k_d(m, k, T, &cpR[k], &HRT[k], &SR[k], NULL);
}

void om_rates(const omech *m, const double *par, double p, const double *y,
              double *kf, double *kr, double *q)
{
    state_d st;
    eval_d(m, P(m, par), p, y, &st);
    for (int j = 0; j < m->nr; ++j) {
        if (kf) kf[j] = st.kf[j];
        if (kr) kr[j] = st.kr[j];
        if (q) q[j] = st.q[j];
    }
}

void om_rhs(const omech *m, const double *par, double p, const double *y, double *f)
{
    rhs_d(m, P(m, par), p, y, f);
}

void om_jac(const omech *m, const double *par, double p, const double *y, double *J)
{
    double f[OM_NMAX];
    jac_d(m, P(m, par), p, y, J, f);
}

/* Complex-step derivative of f (Squire & Trapp 1998): df/dy_j = Im f(y + i h e_j) / h. */
void om_jac_cs(const omech *m, const double *par, double p, const double *y, double *J)
{
    const int n = m->ns + 1;
    const double h = 1e-30;
    double complex yz[OM_NMAX], fz[OM_NMAX], pz[3 * OM_NRMAX];
    const double *pp = P(m, par);
    for (int i = 0; i < 3 * m->nr; ++i) pz[i] = pp[i];
    for (int j = 0; j < n; ++j) {
        for (int k = 0; k < n; ++k) yz[k] = y[k];
        yz[j] += I * h;
        rhs_z(m, pz, p, yz, fz);
        for (int k = 0; k < n; ++k) J[k * n + j] = cimag(fz[k]) / h;
    }
}

int om_lu(int n, double *A, int *piv) { return lu_d(n, A, piv); }
void om_lu_solve(int n, const double *LU, const int *piv, double *b) { lu_solve_d(n, LU, piv, b); }

int om_tableau(int method, int *stages, double *gamma, double *a, double *c, double *mw, double *e)
{
    omtab t;
    if (get_tableau(method, &t)) return -1;
    *stages = t.s;
    *gamma = t.gamma;
    for (int i = 0; i < OM_SMAX; ++i) {
        for (int j = 0; j < OM_SMAX; ++j) {
            a[i * OM_SMAX + j] = t.a[i][j];
            c[i * OM_SMAX + j] = t.c[i][j];
        }
        mw[i] = t.m[i];
        e[i] = t.e[i];
    }
    return 0;
}

int om_step(const omech *m, const double *par, int method, double p, const double *y,
            double h, double *ynew, double *err)
{
    omtab t;
    if (get_tableau(method, &t)) return -1;
    return ros_step_d(m, P(m, par), &t, p, y, h, ynew, err);
}

/* ---------------- adaptive integration of one cell ---------------- */
static int all_finite(int n, const double *v)
{
    for (int i = 0; i < n; ++i)
        if (!isfinite(v[i])) return 0;
    return 1;
}

/* Integrate y over [0, dt]; on return y holds the last accepted state.
   If hs != NULL the accepted step sizes are stored (up to cap). */
static int integrate_cell(const omech *m, const double *par, const omtab *tb, double p,
                          double *y, double dt, double rtol, double atol, const om_opts *o,
                          int *nacc_out, int *nrej_out, double *hs, int cap, int *nh)
{
    const int n = m->ns + 1;
    double ynew[OM_NMAX], err[OM_NMAX];
    int nacc = 0, nrej = 0, status = OM_CELL_OK, rejected_last = 0;
    double t = 0.0, h = dt;
    const int maxs = o && o->max_substeps > 0 ? o->max_substeps : 100000;
    const double hmin = (o && o->hmin_rel > 0 ? o->hmin_rel : 1e-20) * dt;
    if (!(y[0] > 0.0) || !(p > 0.0) || !isfinite(p) || !all_finite(n, y)) {
        status = OM_CELL_BADINPUT;
        goto out;
    }
    while (t < dt) {
        if (nacc + nrej >= maxs) { status = OM_CELL_MAXSTEPS; break; }
        if (h < hmin) { status = OM_CELL_HMIN; break; }
        int last = 0;
        if (h >= dt - t) { h = dt - t; last = 1; }
        int bad = ros_step_d(m, par, tb, p, y, h, ynew, err);
        double en = 0.0;
        if (!bad && all_finite(n, ynew) && all_finite(n, err)) {
            for (int k = 0; k < n; ++k) {
                double sc = atol + rtol * fmax(fabs(y[k]), fabs(ynew[k]));
                en += (err[k] / sc) * (err[k] / sc);
            }
            en = sqrt(en / n);
            if (!isfinite(en)) bad = 1;
        } else {
            bad = 1;
        }
        if (!bad && en <= 1.0) {
            if (hs && nacc < cap) hs[nacc] = h;
            ++nacc;
            memcpy(y, ynew, sizeof(double) * n);
            t = last ? dt : t + h;
            double fac = 0.9 * pow(fmax(en, 1e-16), -0.25);   /* err = 0 -> growth capped anyway */
            fac = fmin(6.0, fmax(0.2, fac));
            if (rejected_last) fac = fmin(1.0, fac);
            h *= fac;
            rejected_last = 0;
        } else {
            ++nrej;
            h *= bad ? 0.2 : fmax(0.2, 0.9 * pow(en, -0.25));
            rejected_last = 1;
        }
    }
out:
    if (nacc_out) *nacc_out = nacc;
    if (nrej_out) *nrej_out = nrej;
    if (nh) *nh = nacc;
    return status;
}

int om_integrate(const omech *m, const double *par, long ncell, double *T, const double *p,
                 double *Y, double dt, double rtol, double atol, const om_opts *opt,
                 int *nacc, int *nrej, int *status, int nthreads)
{
    omtab tb;
    if (get_tableau(opt ? opt->method : OM_RODAS4, &tb)) return OM_E_INVALID;
    const int ns = m->ns;
    const double *pp = P(m, par);
    int anyfail = 0;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
#pragma omp parallel for schedule(dynamic, 16) reduction(|: anyfail)
    for (long c = 0; c < ncell; ++c) {
        double y[OM_NMAX];
        y[0] = T[c];
        memcpy(y + 1, Y + c * ns, sizeof(double) * ns);
        int na, nj;
        int st = integrate_cell(m, pp, &tb, p[c], y, dt, rtol, atol, opt, &na, &nj, NULL, 0, NULL);
        if (st != OM_CELL_BADINPUT) {
            T[c] = y[0];
            memcpy(Y + c * ns, y + 1, sizeof(double) * ns);
        }
        if (nacc) nacc[c] = na;
        if (nrej) nrej[c] = nj;
        if (status) status[c] = st;
        anyfail |= (st != OM_CELL_OK);
    }
    return anyfail ? 1 : 0;
}

int om_step_sizes(const omech *m, const double *par, double T, double p, const double *Y,
                  double dt, double rtol, double atol, const om_opts *opt,
                  int cap, double *hs, int *nh)
{
    omtab tb;
    if (get_tableau(opt ? opt->method : OM_RODAS4, &tb)) return OM_E_INVALID;
    double y[OM_NMAX];
    y[0] = T;
    memcpy(y + 1, Y, sizeof(double) * m->ns);
    int st = integrate_cell(m, P(m, par), &tb, p, y, dt, rtol, atol, opt, NULL, NULL, hs, cap, nh);
    if (*nh > cap) return OM_E_SIZE;
    return st;
}

int om_replay(const omech *m, const double *par, int method, double p, const double *y0,
              int nh, const double *hs, double *yend)
{
    omtab tb;
    if (get_tableau(method, &tb)) return OM_E_INVALID;
    return replay_d(m, P(m, par), &tb, p, y0, nh, hs, yend);
}

/* ---------------- derivatives of the frozen-step map ---------------- */
int om_replay_dir(const omech *m, int method, double p, const double *y0, int nh,
                  const double *hs, const double *dy0, const double *dpar, double *dyend)
{
    omtab tb;
    if (get_tableau(method, &tb)) return OM_E_INVALID;
    const int n = m->ns + 1;
    const double h = 1e-30;
    double complex yz[OM_NMAX], ez[OM_NMAX], pz[3 * OM_NRMAX];
    for (int k = 0; k < n; ++k) yz[k] = y0[k] + I * h * (dy0 ? dy0[k] : 0.0);
    for (int i = 0; i < 3 * m->nr; ++i) pz[i] = m->par[i] + I * h * (dpar ? dpar[i] : 0.0);
    int rc = replay_z(m, pz, &tb, p, yz, nh, hs, ez);
    for (int k = 0; k < n; ++k) dyend[k] = cimag(ez[k]) / h;
    return rc;
}

/* Reverse accumulation over the accepted steps of one cell: with
   Phi_i the i-th frozen step, lambda <- (dPhi_i/dy)^T lambda and
   gpar += (dPhi_i/dpar)^T lambda, both Jacobians by complex step of the step
   function (one complex step per column). */
static int adjoint_cell(const omech *m, const omtab *tb, double p, const double *y0,
                        int nh, const double *hs, const double *lam_end,
                        double *lam0, double *gpar)
{
    const int n = m->ns + 1, np3 = 3 * m->nr;
    const double hc = 1e-30;
    double *ys = malloc(sizeof(double) * (size_t)(nh + 1) * n);
    double complex yz[OM_NMAX], ez[OM_NMAX];
    double complex *pz = malloc(sizeof(double complex) * np3);
    double lam[OM_NMAX], lnew[OM_NMAX];
    int rc = 0;
    memcpy(ys, y0, sizeof(double) * n);
    for (int i = 0; i < nh && !rc; ++i)
        rc = ros_step_d(m, m->par, tb, p, ys + (size_t)i * n, hs[i], ys + (size_t)(i + 1) * n, NULL);
    memcpy(lam, lam_end, sizeof(double) * n);
    for (int i = nh - 1; i >= 0 && !rc; --i) {
        const double *yi = ys + (size_t)i * n;
        for (int q = 0; q < np3; ++q) pz[q] = m->par[q];
        for (int j = 0; j < n; ++j) {              /* column j of dPhi/dy */
            for (int k = 0; k < n; ++k) yz[k] = yi[k];
            yz[j] += I * hc;
            rc |= ros_step_z(m, pz, tb, p, yz, hs[i], ez, NULL);
            double s = 0.0;
            for (int k = 0; k < n; ++k) s += lam[k] * cimag(ez[k]) / hc;
            lnew[j] = s;
        }
        for (int k = 0; k < n; ++k) yz[k] = yi[k];
        for (int q = 0; q < np3; ++q) {            /* column q of dPhi/dpar */
            pz[q] = m->par[q] + I * hc;
            rc |= ros_step_z(m, pz, tb, p, yz, hs[i], ez, NULL);
            pz[q] = m->par[q];
            double s = 0.0;
            for (int k = 0; k < n; ++k) s += lam[k] * cimag(ez[k]) / hc;
            gpar[q] += s;
        }
        memcpy(lam, lnew, sizeof(double) * n);
    }
    memcpy(lam0, lam, sizeof(double) * n);
    free(pz);
    free(ys);
    return rc;
}

int om_adjoint(const omech *m, int method, long ncell, const double *T0, const double *p,
               const double *Y0, double dt, double rtol, double atol, const om_opts *opt,
               const double *gT, const double *gY, double *gT0, double *gY0,
               double *g_lnA, double *g_b, double *g_Ea, int nthreads)
{
    omtab tb;
    if (get_tableau(method, &tb)) return OM_E_INVALID;
    const int ns = m->ns, n = ns + 1, nr = m->nr;
    double *gcell = calloc((size_t)ncell * 3 * nr, sizeof(double));
    int rc = 0;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
#pragma omp parallel for schedule(dynamic, 1) reduction(|: rc)
    for (long c = 0; c < ncell; ++c) {
        double y[OM_NMAX], lam[OM_NMAX], lam0[OM_NMAX];
        int cap = 1 << 16, nh = 0;
        double *hs = malloc(sizeof(double) * cap);
        y[0] = T0[c];
        memcpy(y + 1, Y0 + c * ns, sizeof(double) * ns);
        int st = integrate_cell(m, m->par, &tb, p[c], y, dt, rtol, atol, opt, NULL, NULL, hs, cap, &nh);
        y[0] = T0[c];
        memcpy(y + 1, Y0 + c * ns, sizeof(double) * ns);
        lam[0] = gT[c];
        memcpy(lam + 1, gY + c * ns, sizeof(double) * ns);
        if (st == OM_CELL_OK && nh <= cap) {
            rc |= adjoint_cell(m, &tb, p[c], y, nh, hs, lam, lam0, gcell + (size_t)c * 3 * nr);
        } else {
            rc |= 1;
            for (int k = 0; k < n; ++k) lam0[k] = NAN;
        }
        gT0[c] = lam0[0];
        memcpy(gY0 + c * ns, lam0 + 1, sizeof(double) * ns);
        free(hs);
    }
    /* parameter gradients: fixed ascending cell order */
    for (int j = 0; j < nr; ++j) { g_lnA[j] = 0.0; g_b[j] = 0.0; g_Ea[j] = 0.0; }
    for (long c = 0; c < ncell; ++c)
        for (int j = 0; j < nr; ++j) {
            g_lnA[j] += gcell[(size_t)c * 3 * nr + j];
            g_b[j] += gcell[(size_t)c * 3 * nr + nr + j];
            g_Ea[j] += gcell[(size_t)c * 3 * nr + 2 * nr + j];
        }
    free(gcell);
    return rc;
}
