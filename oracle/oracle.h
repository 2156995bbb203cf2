/*
 * oracle.h -- plain, slow CPU FP64 reference for the per-cell, constant-pressure,
 * adiabatic stiff-chemistry step (the species and energy source terms of the
 * governing equations, Appendix A eqs. (20)-(21); detailed chemistry per Sec. 2.1).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or constant with the GPU library.
 *
 * Conventions: SI units inside (m, kg, mol, s, K, J).  A cell state is
 * y = (T, Y_1 .. Y_ns), n = ns + 1; p is fixed during a step.  All functions
 * work on host memory.  Functions returning int return 0 on success.
 */
#ifndef CHEM_ORACLE_H
#define CHEM_ORACLE_H
#ifdef __cplusplus
extern "C" {
#endif

typedef struct omech omech;

enum { OM_OK = 0, OM_E_IO = -1, OM_E_PARSE = -2, OM_E_INVALID = -3, OM_E_SIZE = -4 };
enum { OM_CELL_OK = 0, OM_CELL_MAXSTEPS = 1, OM_CELL_HMIN = 2, OM_CELL_NONFINITE = 3,
       OM_CELL_BADINPUT = 4 };
enum { OM_RODAS4 = 0, OM_ROS4 = 1 };

typedef struct {
    int method;          /* OM_RODAS4 or OM_ROS4 */
    int max_substeps;    /* attempts (accepted + rejected) per cell; default 100000 */
    double hmin_rel;     /* fail when h < hmin_rel * dt; default 1e-20 */
} om_opts;

/* ---- mechanism ---- */
int  om_load(const char *path, omech **out, char *err, int errlen);
void om_free(omech *m);
int  om_nspecies(const omech *m);
int  om_nreactions(const omech *m);
void om_weights(const omech *m, double *W);                      /* kg/mol [ns] */
/* Arrhenius parameters of each reaction's main rate (k_inf for falloff):
   ln A in SI units, b, Ea in J/mol. */
void om_params(const omech *m, double *lnA, double *b, double *Ea);

/* ---- point functions (one state); par = NULL uses the mechanism's own
   parameters, otherwise 3*nr values laid out lnA[nr], b[nr], Ea[nr] ---- */
void om_thermo(const omech *m, double T, double *cpR, double *HRT, double *SR);
void om_rates(const omech *m, const double *par, double p, const double *y,
              double *kf, double *kr, double *q);
void om_rhs(const omech *m, const double *par, double p, const double *y, double *f);
void om_jac(const omech *m, const double *par, double p, const double *y, double *J);
void om_jac_cs(const omech *m, const double *par, double p, const double *y, double *J);

/* ---- dense LU with partial pivoting (row-major n x n) ---- */
int  om_lu(int n, double *A, int *piv);
void om_lu_solve(int n, const double *LU, const int *piv, double *b);

/* ---- Rosenbrock ---- */
int om_tableau(int method, int *stages, double *gamma, double *a, double *c,
               double *mw, double *e);                          /* a, c: 6x6 row-major */
int om_step(const omech *m, const double *par, int method, double p, const double *y,
            double h, double *ynew, double *err);
int om_integrate(const omech *m, const double *par, long ncell, double *T, const double *p,
                 double *Y, double dt, double rtol, double atol, const om_opts *opt,
                 int *nacc, int *nrej, int *status, int nthreads);
/* Accepted step sizes of one cell's adaptive solve (frozen-step map). */
int om_step_sizes(const omech *m, const double *par, double T, double p, const double *Y,
                  double dt, double rtol, double atol, const om_opts *opt,
                  int cap, double *hs, int *nh);
int om_replay(const omech *m, const double *par, int method, double p, const double *y0,
              int nh, const double *hs, double *yend);

/* ---- derivatives of the frozen-step map ---- */
/* Directional derivative of y_end along (dy0, dpar), by complex step through
   the whole replay. */
int om_replay_dir(const omech *m, int method, double p, const double *y0, int nh,
                  const double *hs, const double *dy0, const double *dpar, double *dyend);
/* Discrete adjoint: per cell, gT0/gY0 = d(gT.T_end + gY.Y_end)/d(T0, Y0); the
   parameter gradients are summed over cells in ascending order. */
int om_adjoint(const omech *m, int method, long ncell, const double *T0, const double *p,
               const double *Y0, double dt, double rtol, double atol, const om_opts *opt,
               const double *gT, const double *gY, double *gT0, double *gY0,
               double *g_lnA, double *g_b, double *g_Ea, int nthreads);

#ifdef __cplusplus
}
#endif
#endif
