// euler.hip -- a minimal one-dimensional reactive-Euler step around the
// chemistry step: the flow equations of the reacting-flow model (mass,
// momentum, sensible energy, species; Appendix A) on a uniform grid with
// reflecting ends, first-order finite volumes with the local Lax-Friedrichs
// (Rusanov) flux, and the chemistry entering as the source terms of eqs.
// (20)-(21): wdot_k in the species equations and qdot in the sensible-energy
// equation, from the operator-split reactor step over the same dt.
//
// Conserved state per cell, row-major [ncell][NV]: rho, rho u, rho E_s,
// rho Y_k (k < NS), with E_s = e_s + u^2 / 2 and the sensible internal energy
// e_s = sum_k Y_k (h_k(T) - h_k(298.15 K)) - p / rho (h_k from the NASA-7
// data, J/kg), ideal gas p = rho R T sum_k Y_k / W_k.
namespace chem_euler {

constexpr int NV = 3 + mech::NS;

// cp/R and h/(RT) of species k at T (the two-range NASA-7 polynomials)
__device__ __forceinline__ void nasa(int k, double T, double& cpR, double& hRT)
{
    const double* c = &mech::THERMO[k][T < mech::THERMO_TMID[k] ? 0 : 1][0];
    cpR = fma(T, fma(T, fma(T, fma(T, c[4], c[3]), c[2]), c[1]), c[0]);
    hRT = fma(T, fma(T, fma(T, fma(T, c[8], c[7]), c[6]), c[5]), c[0]) + c[9] / T;
}

// e_s(T) - target and its derivative c_v, for the mixture Y (J/kg, J/(kg K))
__device__ __forceinline__ void energy(const double* __restrict__ Y, double T, double Rm, double& es, double& cv)
{
    es = -Rm * T;
    double cp = 0.0;
    for (int k = 0; k < mech::NS; ++k) {
        double cpR, hRT;
        nasa(k, T, cpR, hRT);
        es = fma(Y[k], fma(hRT * T, mech::MWTAB[2 * mech::NS + k], -mech::HF298[k]), es);
        cp = fma(Y[k], cpR * mech::MWTAB[2 * mech::NS + k], cp);
    }
    cv = cp - Rm;
}

struct PrimArgs {
    const double* U;   // [ncell][NV]
    long ncell;
    double* T;         // in: starting guess (<= 0: 1000 K); out: temperature
    double* p;
    double* Y;         // [ncell][NS]
    double* u;
    double* c;         // frozen sound speed
    int* bad;          // set to 1 if a cell has no valid state
};

// Primitive variables from the conserved state: T from e_s by Newton's method
// (monotone: c_v > 0), then p and the frozen sound speed sqrt(gamma p / rho).
extern "C" __global__ void __launch_bounds__(256) chem_euler_prim(PrimArgs a)
{
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.ncell) return;
    const double* U = a.U + i * NV;
    const double rho = U[0];
    const double u = U[1] / rho;
    const double es = U[2] / rho - 0.5 * u * u;
    double Y[mech::NS];
    double sig = 0.0;
    for (int k = 0; k < mech::NS; ++k) {
        Y[k] = U[3 + k] / rho;
        sig = fma(Y[k], mech::MWTAB[mech::NS + k], sig);
    }
    const double Rm = mech::RU * sig;
    double T = a.T[i] > 0.0 ? a.T[i] : 1000.0;
    double f = 0.0, cv = 1.0;
    bool conv = false;
    for (int it = 0; it < 60 && !conv; ++it) {
        energy(Y, T, Rm, f, cv);
        f -= es;
        const double dT = -f / cv;
        double Tn = T + dT;
        Tn = fmin(fmax(Tn, 0.5 * T), 2.0 * T);   // damped far from the root
        conv = fabs(Tn - T) <= 1e-12 * T;
        T = Tn;
    }
    const bool ok = conv && rho > 0.0 && T > 0.0 && isfinite(T) && cv > 0.0;
    if (!ok) a.bad[0] = 1;
    const double p = rho * Rm * T;
    a.T[i] = T;
    a.p[i] = p;
    a.u[i] = u;
    a.c[i] = sqrt((cv + Rm) / cv * p / rho);
    for (int k = 0; k < mech::NS; ++k) a.Y[i * mech::NS + k] = Y[k];
}

struct InitArgs {
    const double* T;
    const double* p;
    const double* Y;   // [ncell][NS]
    const double* u;   // may be null (gas at rest)
    long ncell;
    double* U;         // [ncell][NV]
};

// The conserved state of cells given T, p, Y and u.
extern "C" __global__ void __launch_bounds__(256) chem_euler_init(InitArgs a)
{
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.ncell) return;
    double Y[mech::NS];
    double sig = 0.0;
    for (int k = 0; k < mech::NS; ++k) {
        Y[k] = a.Y[i * mech::NS + k];
        sig = fma(Y[k], mech::MWTAB[mech::NS + k], sig);
    }
    const double Rm = mech::RU * sig;
    const double T = a.T[i];
    const double rho = a.p[i] / (Rm * T);
    const double u = a.u ? a.u[i] : 0.0;
    double es, cv;
    energy(Y, T, Rm, es, cv);
    double* U = a.U + i * NV;
    U[0] = rho;
    U[1] = rho * u;
    U[2] = rho * (es + 0.5 * u * u);
    for (int k = 0; k < mech::NS; ++k) U[3 + k] = rho * Y[k];
}

struct UpdateArgs {
    const double* U;
    const double* p;
    const double* u;
    const double* c;
    const double* wdot;   // [ncell][NS], kg/(m^3 s)
    const double* qdot;   // [ncell], W/m^3
    long ncell;
    double dt, dx;
    double* Unew;
    unsigned long long* cflmax;   // max over cells of (|u| + c) dt / dx, as the bits of a
                                  // non-negative double (integer order = numeric order);
                                  // cleared by chem_euler_prim
    const int* bad;               // set by chem_euler_prim: write nothing if any cell is bad
};

// Rusanov flux between the states (UL, pL, uL, cL) and (UR, ...): the mean of
// the physical fluxes minus half the largest wave speed times the jump.
__device__ __forceinline__ void flux(const double* __restrict__ UL, double pL, double uL, double cL,
                                     const double* __restrict__ UR, double pR, double uR, double cR, int v,
                                     double& F)
{
    const double s = fmax(fabs(uL) + cL, fabs(uR) + cR);
    double fl = UL[v] * uL, fr = UR[v] * uR;
    if (v == 1) {
        fl += pL;
        fr += pR;
    } else if (v == 2) {
        fl += pL * uL;
        fr += pR * uR;
    }
    F = 0.5 * (fl + fr) - 0.5 * s * (UR[v] - UL[v]);
}

// U_new = U - dt/dx (F_i+1/2 - F_i-1/2) + dt S; the ends reflect (a mirror
// state with the velocity reversed), so mass, species and energy stay in the
// tube.
extern "C" __global__ void __launch_bounds__(256) chem_euler_update(UpdateArgs a)
{
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    // the block's largest CFL number, one atomic per block
    __shared__ double smax[256];
    const double cfl = i < a.ncell ? (fabs(a.u[i]) + a.c[i]) * (a.dt / a.dx) : 0.0;
    smax[threadIdx.x] = cfl;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + off]);
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicMax(a.cflmax, (unsigned long long)__double_as_longlong(smax[0]));
    if (i >= a.ncell || *a.bad) return;
    const double* Ui = a.U + i * NV;
    double mir[NV];
    const long l = i - 1, r = i + 1;
    const double r_dt = a.dt / a.dx;
    for (int v = 0; v < NV; ++v) {
        double Fl, Fr;
        // left face
        if (l < 0) {
            for (int q = 0; q < NV; ++q) mir[q] = Ui[q];
            mir[1] = -Ui[1];
            flux(mir, a.p[i], -a.u[i], a.c[i], Ui, a.p[i], a.u[i], a.c[i], v, Fl);
        } else {
            flux(a.U + l * NV, a.p[l], a.u[l], a.c[l], Ui, a.p[i], a.u[i], a.c[i], v, Fl);
        }
        // right face
        if (r >= a.ncell) {
            for (int q = 0; q < NV; ++q) mir[q] = Ui[q];
            mir[1] = -Ui[1];
            flux(Ui, a.p[i], a.u[i], a.c[i], mir, a.p[i], -a.u[i], a.c[i], v, Fr);
        } else {
            flux(Ui, a.p[i], a.u[i], a.c[i], a.U + r * NV, a.p[r], a.u[r], a.c[r], v, Fr);
        }
        double src = 0.0;
        if (v == 2) src = a.qdot[i];
        if (v >= 3) src = a.wdot[i * mech::NS + (v - 3)];
        a.Unew[i * NV + v] = Ui[v] - r_dt * (Fr - Fl) + a.dt * src;
    }
}

}  // namespace chem_euler
