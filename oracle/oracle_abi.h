/*
 * oracle_abi.h -- the chemistry-step C ABI served by the CPU oracle: the
 * entry points of the GPU library (load, info, parameters, source terms,
 * fixed step, integration, discrete adjoint, last error) with the same
 * arguments, codes and conventions, on host memory and without a stream, so
 * a test can run unchanged against either library.
 *
 * TEST INFRASTRUCTURE ONLY, like the rest of the oracle: only the test suite,
 * the smoke check and the benchmark's CPU-baseline leg may load it.  It
 * declares its own codes and structures; the values are the ABI's contract:
 *
 *   return codes: 0 ok; -1 bad argument (nothing done); -2 mechanism file
 *   syntax; -3 mechanism content (element balance, ...); -6 ran, a cell has
 *   a non-OK status; -8 unsupported (sizes above the oracle's limits, h0).
 *   cell status: 0 ok, 1 max substeps, 2 step below hmin_rel dt, 3 (adjoint
 *   rerun mismatch; never produced here), 4 bad input (T <= 0, p <= 0, a
 *   non-finite value: the cell is left untouched).
 *
 * The method is the oracle's RODAS4 integration (oracle.h); the GPU-only
 * launch knobs of the options (form, block, waves per SIMD, refill, order,
 * cost, checkpoint interval, a forward's step counts) change no result and
 * are accepted and ignored, except that a checkpoint interval above 16 is a
 * bad argument as there.
 */
#ifndef CHEM_ORACLE_ABI_H
#define CHEM_ORACLE_ABI_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

typedef struct oracle_mechanism oracle_mechanism;

enum {
    ORACLE_OK = 0,
    ORACLE_E_INVAL = -1,
    ORACLE_E_PARSE = -2,
    ORACLE_E_MECH_INVALID = -3,
    ORACLE_E_CELL_FAILED = -6,
    ORACLE_E_UNSUPPORTED = -8
};

typedef struct {
    int form;
    int max_substeps;            /* attempts per cell; <= 0 means 100000 */
    double hmin_rel;             /* fail below hmin_rel * dt; <= 0 means 1e-20 */
    const double *h0;            /* must be NULL (first trial step dt) */
    int checkpoint_every;        /* adjoint: 0..16 accepted, no effect here */
    int block, waves_per_simd, refill, order;
    const int32_t *const *cost;
    const int32_t *adjoint_nacc;  /* a forward's step counts: no effect here */
} oracle_options;

typedef struct {
    int64_t cells, accepted, rejected, max_substeps, failed;
    double kernel_ms;            /* wall time of the computation */
} oracle_stats;

/* A `chemmi-mech 1` file (the oracle's reader); -1 unreadable path. */
int oracle_load_mechanism(const char *path, oracle_mechanism **out);
void oracle_free_mechanism(oracle_mechanism *m);
int oracle_mechanism_info(const oracle_mechanism *m, int *n_species, int *n_reactions);
/* ln A (SI), b, Ea (J/mol) of every reaction's main rate; set: finite values. */
int oracle_get_params(const oracle_mechanism *m, double *lnA, double *b, double *Ea);
int oracle_set_params(oracle_mechanism *m, const double *lnA, const double *b, const double *Ea);
/* f[ncell * n] and (nullable) J[ncell * n * n], row-major, analytic. */
int oracle_eval_source(const oracle_mechanism *m, int64_t ncell, const double *T, const double *p,
                       const double *Y, double *f, double *J);
/* One RODAS4 step of size h: ynew[ncell * n], the RMS error norm with
   scale atol + rtol max(|y_k|, |ynew_k|), ok = 0 if the step failed. */
int oracle_step_fixed(const oracle_mechanism *m, int64_t ncell, const double *T, const double *p,
                      const double *Y, double h, double rtol, double atol, double *ynew,
                      double *errnorm, int32_t *ok);
/* Adaptive integration over [0, dt]: T, Y in/out; p in; cell_status, nacc,
   nrej nullable out; -6 when stats is given and a cell failed. */
int oracle_integrate(const oracle_mechanism *m, int64_t ncell, double *T, const double *p,
                     double *Y, double dt, double rtol, double atol, const oracle_options *opt,
                     oracle_stats *stats, int32_t *cell_status, int32_t *nacc, int32_t *nrej);
/* Discrete adjoint of the frozen-step map; T_end/Y_end both or neither;
   -6 if a cell failed (its gT0/gY0 are NaN and it adds nothing to the
   parameter gradients). */
int oracle_integrate_adjoint(const oracle_mechanism *m, int64_t ncell, const double *T0,
                             const double *p, const double *Y0, double dt, double rtol,
                             double atol, const double *gT, const double *gY, double *gT0,
                             double *gY0, double *g_lnA, double *g_b, double *g_Ea,
                             double *T_end, double *Y_end, const oracle_options *opt,
                             oracle_stats *stats);
const char *oracle_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
