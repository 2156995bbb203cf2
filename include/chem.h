/*
 * chem.h -- C ABI of the MI355X chemistry-step library.
 *
 * The library advances, cell by cell, the temperature T and species mass
 * fractions Y_k of an adiabatic, constant-pressure, ideal-gas cell over one
 * flow time step dt under detailed finite-rate chemistry: the species
 * production rates omega_k and heat release Q of the governing equations
 * (Appendix A, eqs. (20)-(21)) with the detailed-chemistry model of Sec. 2.1,
 * integrated as the operator-split energy/species stage of the solver
 * (Sec. 2.1, PIMPLE description).  Per cell:
 *     dY_k/dt = W_k omega_k / rho,
 *     dT/dt   = -sum_k H_k omega_k / (rho c_p),      p fixed,
 * with NASA-7 thermo, modified-Arrhenius forward rates, reverse rates from
 * equilibrium constants (1 atm standard state), third-body efficiencies and
 * Lindemann/Troe falloff, integrated by RODAS4 (Hairer & Wanner) with an
 * analytic Jacobian, dense LU with partial pivoting, RMS error control
 * (scale atol + rtol max(|y|, |y_new|)) and h <- h clip(0.9 err^-1/4, 0.2, 6).
 *
 * Conventions for every function:
 *   - Return 0 (CHEM_OK) or a negative CHEM_E_* code; chem_last_error() then
 *     holds a message (thread-local).
 *   - Arrays named "device" must be device (or managed) memory on the current
 *     HIP device; host pointers there give CHEM_E_INVAL and nothing runs.
 *     The caller owns every array it passes; the library never frees them.
 *   - Layout: T[ncell], p[ncell] (Pa), Y[ncell * ns] row-major (cell-major,
 *     species fastest), all IEEE double.
 *   - Work is enqueued on `stream` (a hipStream_t; NULL = the legacy default
 *     stream) and is asynchronous, unless a stats pointer is given, which
 *     synchronises the stream before return.
 *   - ncell = 0 is a valid no-op.
 *   - A mechanism handle may be used from several host threads; calls on it
 *     are serialised internally, and the device work of each call is ordered
 *     after that of the previous call on the handle even when the two use
 *     different streams (they share the handle's device workspace).
 */
#ifndef CHEM_H
#define CHEM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CHEM_MAX_SPECIES 48

typedef struct chem_mechanism chem_mechanism;   /* opaque, library-owned */

enum chem_error {
    CHEM_OK = 0,
    CHEM_E_INVAL = -1,          /* bad argument; nothing was launched */
    CHEM_E_PARSE = -2,          /* mechanism file syntax */
    CHEM_E_MECH_INVALID = -3,   /* mechanism content (e.g. element balance) */
    CHEM_E_HIP = -4,            /* HIP runtime failure */
    CHEM_E_NOMEM = -5,          /* device allocation failed */
    CHEM_E_CELL_FAILED = -6,    /* ran; at least one cell has a non-OK status */
    CHEM_E_COMPILE = -7,        /* device code generation or compilation failed */
    CHEM_E_UNSUPPORTED = -8     /* e.g. more than CHEM_MAX_SPECIES species */
};

/* Per-cell status (int32 per cell).  A failed cell keeps its last accepted
   state; a BADINPUT cell is left untouched. */
enum chem_cell_status {
    CHEM_CELL_OK = 0,
    CHEM_CELL_MAXSTEPS = 1,     /* max_substeps attempts without reaching dt */
    CHEM_CELL_HMIN = 2,         /* step size fell below hmin_rel * dt */
    CHEM_CELL_NONFINITE = 3,    /* adjoint only: the checkpointed rerun of a cell took more
                                   accepted steps than its sizing pass or the caller's
                                   adjoint_nacc entry allows (the sizing pass runs the same
                                   code on the same input, so only a wrong entry does it) */
    CHEM_CELL_BADINPUT = 4      /* T <= 0, p <= 0 or a non-finite input */
};

enum chem_form {
    CHEM_FORM_AUTO = 0,         /* plain for a single field */
    CHEM_FORM_PLAIN = 1,        /* one cell per lane, one launch per field */
    CHEM_FORM_PERSISTENT = 2    /* persistent work-stealing launch in a HIP graph */
};

/* Order in which the persistent form starts cells (results are bitwise the
   same in every order; only the time differs). */
enum chem_order {
    CHEM_ORDER_AUTO = 0,        /* default: whichever of the two below measured faster on a
                                   sample of a field of this size (the launch-shape tuner) */
    CHEM_ORDER_COST = 1,        /* most expensive first (caller's cost, else predicted) */
    CHEM_ORDER_NATURAL = 2      /* index order */
};

typedef struct {
    int form;                   /* enum chem_form */
    int max_substeps;           /* attempts per cell; <= 0 means 100000 */
    double hmin_rel;            /* fail below hmin_rel * dt; <= 0 means 1e-20 */
    const double *h0;           /* nullable device [ncell]: first trial step; else dt */
    int checkpoint_every;       /* adjoint: accepted steps per checkpoint (1..16); <= 0: the
                                   smallest of 1, 2, 4, 8, 16 whose arena fits a quarter of
                                   the free device memory (16 if none does) */
    int block;                  /* persistent: lanes per workgroup (64..256); 0 = tuned */
    int waves_per_simd;         /* persistent: resident waves per SIMD (1..2); 0 = tuned */
    int refill;                 /* persistent: idle lanes that trigger a refill; 0 = tuned */
    int order;                  /* persistent: enum chem_order; 0 = CHEM_ORDER_AUTO */
    const int32_t *const *cost; /* nullable host array [nfield] of nullable device int32 [ncell]
                                   per-cell cost hints (e.g. nacc + nrej of the previous call);
                                   fields without one get a cost predicted from their state:
                                   the mean over the components of
                                   log2(1 + |f_k(y)| dt / (atol + rtol |y_k|)) */
    const int32_t *adjoint_nacc; /* adjoint: nullable device int32 [ncell], the accepted
                                   substeps of every cell in a forward integration of the same
                                   input with the same tolerances and limits (chem_integrate's
                                   nacc, either form); given, the adjoint skips its own sizing
                                   pass.  A cell whose rerun takes more steps than its entry
                                   fails with CHEM_CELL_NONFINITE (NaN gradients) */
} chem_options;

typedef struct {
    int64_t cells;              /* cells processed */
    int64_t accepted;           /* accepted substeps, summed over cells */
    int64_t rejected;           /* rejected substeps, summed over cells */
    int64_t max_substeps;       /* largest accepted + rejected of any cell */
    int64_t failed;             /* cells with a non-OK status */
    double kernel_ms;           /* device time of the integration launches */
} chem_stats;

/* Read and validate a `chemmi-mech 1` file, or a CHEMKIN file with its thermo
   inline (recognised by a first keyword ELEMENTS/ELEM/SPECIES/SPEC/THERMO; read
   as chem_load_chemkin does) (native format: NASA-7 species thermo;
   elementary, third-body, Lindemann, Troe, SRI and pressure-tabulated (PLOG)
   reactions, reversible at k_f / K_c or irreversible; the "reactions and
   thermo data" of Sec. 2.1), check the element balance of every reaction
   exactly, convert A from cm-mol-s to SI by (1e-6)^(order-1) and Ea from
   kJ/mol, and build the device code for it
   (generated mechanism-specific source compiled for gfx950 with hipRTC, with an
   on-disk cache in $CHEM_KERNEL_CACHE or a kcache/ folder beside the library).
   *out is owned by the caller until chem_free_mechanism.  Errors:
   CHEM_E_INVAL (unreadable path), CHEM_E_PARSE, CHEM_E_MECH_INVALID,
   CHEM_E_UNSUPPORTED, CHEM_E_COMPILE. */
int chem_load_mechanism(const char *path, chem_mechanism **out);

/* Read a mechanism in the CHEMKIN text format and build its device code as
   chem_load_mechanism does (which also takes a CHEMKIN file, recognised by
   its first keyword, with the thermo data inline).  mech_path: ELEMENTS
   (symbols, optional /weight/; standard weights for H D HE C N O F NE SI S CL
   AR KR XE), SPECIES, an optional THERMO section, REACTIONS with the unit
   keywords CAL/MOLE (default), KCAL/MOLE, JOULES/MOLE, KJOULES/MOLE, KELVINS,
   EVOLTS and MOLES.  thermo_path: NULL, or a file of NASA-7 four-line
   records (optionally opened by THERMO [ALL] and the default temperatures)
   used for species the mechanism file gives no record for.  Reactions:
   "=", "<=>" (reversible at k_f / K_c) and "=>" (irreversible); "+M" third
   bodies with species/efficiency/ pairs; "(+M)" and "(+species)" falloff with
   LOW and optional TROE (3 or 4 values) or SRI (3 or 5 values); PLOG/p A b E/
   lines (p in atm, increasing; ln k linear in ln p between them, the end
   rates outside), which replace the reaction line's own rate; DUPLICATE,
   required on every reaction that repeats another's species and third-body
   form.  Integer coefficients only.  REV, FORD/RORD, HIGH, CHEB, LT and the
   other rate forms give CHEM_E_UNSUPPORTED naming the line.  A PLOG
   reaction's parameters (chem_get_params) are a factor on its table
   (A = 1, b = 0, Ea = 0 as loaded).  Errors as chem_load_mechanism, with
   "file:line: " in chem_last_error(). */
int chem_load_chemkin(const char *mech_path, const char *thermo_path, chem_mechanism **out);

/* Read a mechanism in OpenFOAM's chemistry dictionary format (the input of
   the paper's detailed-chemistry model, Sec. 2.1) and build its device code.
   reactions_path: a dictionary file with `species (names);`, an optional
   `elements (names);` and a `reactions { name { type ...; reaction "a + b =
   c"; ... } ... }` dictionary; types (with or without a trailing "Reaction")
   reversible/irreversible + Arrhenius, ThirdBodyArrhenius,
   ArrheniusLindemannFallOff, ArrheniusTroeFallOff (F: alpha Tsss Ts Tss),
   ArrheniusSRIFallOff (F: a b c d e); rates as A beta Ta with A in
   (m^3/kmol)^(order-1)/s and Ta = Ea/R in K; k0 and kInf dictionaries for
   falloff; thirdBodyEfficiencies { coeffs N ((species value) ...); }.
   thermo_path: one dictionary per species with specie { molWeight (kg/kmol) },
   thermodynamics { Tlow Thigh Tcommon highCpCoeffs (7) lowCpCoeffs (7) } and
   elements { symbol count; ... }; species weights come from molWeight.
   Reaction orders (^), non-integer coefficients and other reaction types give
   CHEM_E_UNSUPPORTED naming the reaction.  Errors as chem_load_mechanism. */
int chem_load_openfoam(const char *reactions_path, const char *thermo_path, chem_mechanism **out);

/* Free the handle and every device resource the library holds for it. */
void chem_free_mechanism(chem_mechanism *m);

/* Species and reaction counts. */
int chem_mechanism_info(const chem_mechanism *m, int *n_species, int *n_reactions);

/* Arrhenius parameters of each reaction's main (high-pressure) rate
   k = A T^b exp(-Ea/RT): host arrays [n_reactions] of ln A (SI), b and Ea
   (J/mol).  chem_set_params replaces them for every later call (the kernels
   read them from device memory, so no recompilation happens). */
int chem_get_params(const chem_mechanism *m, double *lnA, double *b, double *Ea);
int chem_set_params(chem_mechanism *m, const double *lnA, const double *b, const double *Ea);

/* Source terms f = dy/dt (y = (T, Y_1..Y_ns), n = ns + 1) of eqs. (20)-(21) at
   constant p, and optionally their analytic Jacobian, at given states.
   Device: T, p, Y (in), f[ncell * n] (out), J[ncell * n * n] (out, row-major
   df_i/dy_j, nullable). */
int chem_eval_source(const chem_mechanism *m, int64_t ncell, const double *T, const double *p,
                     const double *Y, double *f, double *J, void *stream);

/* One RODAS4 step of fixed size h per cell (no step-size control).  Device:
   T, p, Y (in); ynew[ncell * n], errnorm[ncell] (the RMS error norm with the
   given rtol, atol), ok[ncell] int32 (0 if the step matrix was singular or a
   result not finite). */
int chem_step_fixed(const chem_mechanism *m, int64_t ncell, const double *T, const double *p,
                    const double *Y, double h, double rtol, double atol, double *ynew,
                    double *errnorm, int32_t *ok, void *stream);

/* Integrate every cell over [0, dt] (adaptive RODAS4).  Device: T, Y in/out;
   p in; cell_status[ncell] (nullable, out); nacc/nrej[ncell] (nullable, out:
   accepted and rejected substeps per cell).  opt and stats are host pointers
   and may be NULL.  dt > 0, rtol > 0, atol >= 0 or CHEM_E_INVAL.  Returns
   CHEM_E_CELL_FAILED when stats is given and a cell failed.  Without stats
   the call does not wait for the result and returns CHEM_OK: a failed cell
   then shows only in cell_status (keep it, or pass stats, to detect one). */
int chem_integrate(const chem_mechanism *m, int64_t ncell, double *T, const double *p,
                   double *Y, double dt, double rtol, double atol, const chem_options *opt,
                   chem_stats *stats, int32_t *cell_status, int32_t *nacc, int32_t *nrej,
                   void *stream);

/* Largest ncell of chem_integrate_noalloc: its scratch holds 17 bytes per
   cell plus 4 KiB, about 36 MB per device. */
#define CHEM_NOALLOC_MAX_CELLS 2097152

/* chem_integrate without any device allocation, for callers that cannot
   allocate: code under HIP graph capture, tight serving loops, harnesses that
   forbid hipMalloc.  It runs the persistent form (cells started most
   expensive first, work-stealing waves) with every temporary -- queue heads,
   cost histogram, field table, per-cell cost buckets and permutation, and
   the status/substep counters the caller does not pass -- in a fixed scratch
   area the library holds on each device (CHEM_NOALLOC_MAX_CELLS cells, kept
   until the process ends), and calls no hipMalloc, hipFree or allocating
   library routine.  Arguments as chem_integrate, without stats: T, Y (in/out)
   and p are device arrays of ncell <= CHEM_NOALLOC_MAX_CELLS cells;
   cell_status, nacc, nrej are nullable device outputs; opt may be NULL
   (order, cost, block, refill, max_substeps and hmin_rel are used; form is
   ignored; h0 must be NULL).  The work is enqueued on `stream` and the call
   returns without waiting, so failed cells show only in cell_status.
   Results are bitwise equal to chem_integrate with CHEM_FORM_PERSISTENT.
   Set-up: the mechanism's device code must be loaded on the current device
   beforehand -- chem_load_mechanism does it when a gfx950 device is current,
   and any other entry point does it on first use on a device; otherwise
   CHEM_E_INVAL.  After chem_set_params the next call copies the parameters
   and waits for that copy.  Every call on one GPU shares that GPU's scratch
   and leaves its contents behind (the kernels clear what must start at
   zero): calls that overlap on one GPU -- on unordered streams, or from
   different mechanism handles -- race.  Errors: CHEM_E_INVAL (bad argument,
   ncell above the limit, device not set up; nothing launched), CHEM_E_HIP. */
int chem_integrate_noalloc(const chem_mechanism *m, int64_t ncell, double *T, const double *p,
                           double *Y, double dt, double rtol, double atol, const chem_options *opt,
                           int32_t *cell_status, int32_t *nacc, int32_t *nrej, void *stream);

/* Integrate every cell over [0, dt] as chem_integrate does and return the
   reaction terms a flow solver adds to its species and energy equations
   (Appendix A, eqs. (21) and (20)) for an operator-split step: the mean rates
   over the step,
     wdot[cell * ns + k] = rho0 (Y_k(dt) - Y_k(0)) / dt      [kg/(m^3 s)]
     qdot[cell]          = -sum_k h_k(298.15 K) wdot_k         [W/m^3]
   where rho0 = p Wbar / (R T) of the initial state and h_k(298.15 K) the
   species' enthalpy from its NASA-7 data (J/kg; zero for the elements'
   reference species), i.e. the chemical heat release.  Device: T, Y in/out
   (advanced as by chem_integrate); p in; wdot[ncell * ns], qdot[ncell] out;
   cell_status[ncell] nullable out.  A failed cell gets NaN in wdot and qdot.
   opt (form, tolerances of the integration, ...) and stats as for
   chem_integrate. */
int chem_integrate_source(const chem_mechanism *m, int64_t ncell, double *T, const double *p,
                          double *Y, double dt, double rtol, double atol, double *wdot,
                          double *qdot, const chem_options *opt, chem_stats *stats,
                          int32_t *cell_status, void *stream);

/* The conserved state of the 1D driver (layout as chem_euler1d_step's U)
   from temperature T, pressure p (Pa), mass fractions Y [ncell][ns] and
   velocity u (NULL: at rest), all device pointers: rho = p / (R T sum Y/W),
   rho E_s = rho (e_s(T) + u^2/2).  Errors: CHEM_E_INVAL for bad arguments. */
int chem_euler1d_init(const chem_mechanism *m, int64_t ncell, const double *T, const double *p,
                      const double *Y, const double *u, double *U, void *stream);

/* One step of a minimal one-dimensional reactive-Euler solver around the
   chemistry step (the flow equations of Appendix A with the chemistry as the
   source terms of eqs. (20)-(21)): first-order finite volumes on a uniform
   grid of ncell cells of width dx with the local Lax-Friedrichs flux and
   reflecting ends, forward Euler in time, the chemistry advanced over the same
   dt by chem_integrate_source (constant pressure, each cell's own state) and
   entering as wdot_k in the species equations and qdot in the sensible-energy
   equation.
   U, U_out: device, [ncell][3 + ns] row-major conserved state rho (kg/m^3),
   rho u (kg/(m^2 s)), rho E_s (J/m^3; E_s = e_s + u^2/2, e_s = sum_k Y_k
   (h_k(T) - h_k(298.15 K)) - p/rho with h_k from the NASA-7 data), rho Y_k;
   U_out must not be U.  T: device [ncell], in: a starting guess for the
   temperature of U (<= 0: 1000 K), out: that temperature (Newton's method on
   e_s).  rtol, atol, opt: as chem_integrate (opt->h0 must be NULL).  stats:
   the chemistry step's.  max_cfl: NULL, or receives max over cells of
   (|u| + c) dt / dx with the frozen sound speed c (the step is taken whatever
   its value; it is stable for max_cfl <= 1).  The step keeps its checks on
   the device and synchronises the stream once, at its end, for one 16-byte
   readback (the bad-state flag and the largest CFL number).  Errors:
   CHEM_E_INVAL for bad arguments (nothing launched) or a cell whose state
   gives no temperature (U_out is then not written; T holds the Newton
   iterates); CHEM_E_CELL_FAILED if a cell's chemistry failed (its U_out
   entries are NaN). */
int chem_euler1d_step(const chem_mechanism *m, int64_t ncell, double dx, double dt, const double *U,
                      double *U_out, double *T, double rtol, double atol, const chem_options *opt,
                      chem_stats *stats, double *max_cfl, void *stream);

/* Integrate nfield independent fields (e.g. the cell sets of different mesh
   refinement levels) of sizes ncell[f] in one launch: the single-GPU analogue
   of the paper's dynamic load balancing on measured compute time
   (Sec. 3.3.1), with cells rather than subdomains as the unit of balance.  T, p, Y are host
   arrays of nfield device pointers.  With CHEM_FORM_PERSISTENT (the default
   here) one persistent work-stealing kernel processes all fields: waves pull
   cells from per-XCD queues, steal from the others when theirs is empty, and
   refill idle lanes at substep boundaries, so cells of very different cost
   share the machine evenly; the launch is captured once in a HIP graph and
   replayed.  Results are bitwise identical to chem_integrate on each field. */
int chem_integrate_batched(const chem_mechanism *m, int nfield, double *const *T,
                           const double *const *p, double *const *Y, const int64_t *ncell,
                           double dt, double rtol, double atol, const chem_options *opt,
                           chem_stats *stats, void *stream);

/* Discrete adjoint of the frozen-step map y0 -> y(dt) of the chemistry step
   above (the paper defines the step, eqs. (20)-(21), not its derivative; the
   construction follows the Rosenbrock adjoints of Sandu, Daescu & Carmichael,
   Atmos. Environ. 37 (2003)): the accepted step sizes of the forward solve are held fixed and every RODAS4
   step is differentiated exactly, stage by stage (transposed LU solves, the
   Jacobian at each stage point, and the derivative of the step matrix's
   Jacobian along each stage vector).  Device inputs: T0, p, Y0 (the start
   state), gT[ncell], gY[ncell * ns] (dL/dT_end, dL/dY_end).  Device outputs:
   gT0, gY0 (dL/dT0, dL/dY0 per cell) and g_lnA, g_b, g_Ea [n_reactions]: dL
   with respect to each reaction's ln A, b and Ea (J/mol) of the main rate,
   summed over cells in a fixed order (bitwise reproducible).  T_end/Y_end
   (device, both or neither) receive the forward result, bitwise equal to
   chem_integrate's.  The call first runs a sizing pass (unless
   opt->adjoint_nacc gives the step counts), then stores each cell's state
   every opt->checkpoint_every accepted steps (see chem_options; by default
   every step whenever memory allows) and recomputes in between, keeping what
   a replayed step's adjoint needs in a per-lane buffer of that many steps;
   it allocates its arena (8 bytes per accepted step plus one state per
   checkpoint per cell, and 24 n_reactions bytes per resident lane) for the
   call and synchronises the stream.  Returns
   CHEM_E_CELL_FAILED if a cell failed (stats or not): such cells get NaN
   gT0/gY0 and add nothing to the parameter gradients.  Both kernel forms
   provide it: one cell per lane, or one group of lanes per cell for the
   wave-cooperative form (mechanisms above 13 species), whose transposed
   solves and Jacobian-transpose products are group reductions.  In the one
   cell per lane form the most expensive cells (at least 0.6 of the largest
   accepted-step count; CHEM_ADJOINT_GROUP_FRAC in the environment overrides
   the fraction, 0 turns it off) run on groups of 8 lanes that evaluate the
   six second-order terms of each step side by side: the same derivative up
   to the order of that six-term sum. */
int chem_integrate_adjoint(const chem_mechanism *m, int64_t ncell, const double *T0,
                           const double *p, const double *Y0, double dt, double rtol,
                           double atol, const double *gT, const double *gY, double *gT0,
                           double *gY0, double *g_lnA, double *g_b, double *g_Ea,
                           double *T_end, double *Y_end, const chem_options *opt,
                           chem_stats *stats, void *stream);

/* Message of the last non-zero return on this thread ("" if none). */
const char *chem_last_error(void);

/* Library version string. */
const char *chem_version(void);

#ifdef __cplusplus
}
#endif
#endif /* CHEM_H */
