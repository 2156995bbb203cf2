/*
 * oracle_internal.h -- the oracle's mechanism, reaction and tableau structs and
 * limits, shared by oracle.c and the counted instantiation (count.cpp).
 *
 * TEST INFRASTRUCTURE ONLY (see oracle.h).
 */
#ifndef CHEM_ORACLE_INTERNAL_H
#define CHEM_ORACLE_INTERNAL_H

#define OM_NSMAX 64
#define OM_NRMAX 256
#define OM_NMAX (OM_NSMAX + 1)
#define OM_SMAX 6
#define OM_RU 8.314462618      /* J/(mol K), CODATA 2018 */
#define OM_PATM 101325.0       /* Pa, standard state of K_p */
#define OM_MAXSIDE 4
#define OM_NEMAX 16

#define OM_PLOGMAX 16

enum { OMR_ELEMENTARY = 0, OMR_THIRDBODY = 1, OMR_LINDEMANN = 2, OMR_TROE = 3, OMR_SRI = 4, OMR_PLOG = 5 };

typedef struct {
    int type;
    int nre, rsp[OM_MAXSIDE], rnu[OM_MAXSIDE];
    int np, psp[OM_MAXSIDE], pnu[OM_MAXSIDE];
    int dnu;
    double lnA, b, Ea;                 /* SI, J/mol */
    double lnA0, b0, Ea0;              /* low-pressure limit */
    double alpha, T3, T1, T2;
    int has_T2;
    double sri[5];                     /* SRI a, b (K), c (K), d, e */
    int nplog;                         /* PLOG: pressures (Pa), increasing, and their rates */
    double plog_p[OM_PLOGMAX], plog_lnA[OM_PLOGMAX], plog_b[OM_PLOGMAX], plog_Ea[OM_PLOGMAX];
    int irrev;                         /* no reverse reaction */
    double eff[OM_NSMAX];
} omrxn;

struct omech {
    int ns, nr, ne;
    char ename[OM_NEMAX][8];
    double ew[OM_NEMAX];               /* g/mol */
    char sname[OM_NSMAX][24];
    int comp[OM_NSMAX][OM_NEMAX];
    double W[OM_NSMAX];                /* kg/mol */
    double tmid[OM_NSMAX], lo[OM_NSMAX][7], hi[OM_NSMAX][7];
    int has_thermo[OM_NSMAX];
    omrxn rx[OM_NRMAX];
    double par[3 * OM_NRMAX];          /* lnA[nr], b[nr], Ea[nr] */
};

typedef struct {
    int s;
    double gamma;
    double a[OM_SMAX][OM_SMAX], c[OM_SMAX][OM_SMAX], m[OM_SMAX], e[OM_SMAX];
} omtab;

#endif
