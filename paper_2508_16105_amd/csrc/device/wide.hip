// wide.hip -- the chemistry step for mechanisms whose per-cell matrices do not
// fit the registers of one lane (CDNA4, gfx950).
//
// G lanes (a power of two, at least n = ns + 1) cooperate on one cell, so a
// 64-lane wave holds 64 / G cells.  Lane i of a group owns component i of
// every state-sized vector (i = 0: T, i = 1 + k: Y_k) and row i of the
// Jacobian, of the step matrix and of its LU factors: n doubles of matrix row
// and one double per vector stay in registers.  Per source-term evaluation:
//   - species thermo (NASA-7) in the species' own lanes;
//   - mixture sums (sum Y/W, c_p, heat release) as group reductions;
//   - reaction rates spread over the lanes, read from the mechanism tables
//     (reactions grouped by kind so a round of lanes mostly takes one branch);
//   - production rates gathered, and Jacobian rows assembled, by each species
//     lane from the rates and partials in the cell's LDS scratch in a fixed
//     order (reproducible results);
// and per step the LU factorisation with partial pivoting (pivot search as a
// group arg-max, the pivot row broadcast from its lane), the triangular
// solves (one broadcast per column) and the RMS error norm (a group sum).
// Reductions leave the same bits in every lane of a group, so the step-size
// controller runs identically in all of them.
//
// The equations, the RODAS4 tableau and the controller are those of the
// one-cell-per-lane integrator (the species/energy source of eqs. (20)-(21)
// at constant pressure over one flow step).

namespace chemw {

using chem::RA;
using chem::RC;
using chem::Rodas4;
using chem::StepArgs;
using chem::finite;
constexpr int N = mech::N, NS = mech::NS, NR = mech::NR, G = mech::G;
constexpr int CPW = 64 / G;
constexpr int NSLOT = mech::NSLOT, PW = mech::PW, JW = mech::JW;
constexpr int ROUNDS = (NR + G - 1) / G;
static_assert(N <= G && G <= 64 && (G & (G - 1)) == 0, "group size");

__device__ __forceinline__ int gl() { return (int)(threadIdx.x & (unsigned)(G - 1)); }

// the lane index behind an opaque zero: compares against it (i == k for
// every k of an unrolled loop) are made where used instead of being hoisted
// out of the substep loop as dozens of live lane masks
__device__ __forceinline__ int gl_local() { return gl() + mech::opaque_zero(); }
__device__ __forceinline__ int gbase() { return (int)(threadIdx.x & 63u & ~(unsigned)(G - 1)); }

// value of x in lane `src` of this group; src is the same in every lane of the group
__device__ __forceinline__ double bcast(double x, int src)
{
    if constexpr (G == 64) {
        const long long b = __double_as_longlong(x);
        const int lo = __builtin_amdgcn_readlane((int)b, src);
        const int hi = __builtin_amdgcn_readlane((int)(b >> 32), src);
        return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
    } else {
        return __shfl(x, gbase() + src, 64);
    }
}

// value of x in lane `src` of this group; src may differ per lane
__device__ __forceinline__ double gather(double x, int src) { return __shfl(x, gbase() + src, 64); }

template <int CTRL>
__device__ __forceinline__ double dpp(double x)
{
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

__device__ __forceinline__ double readlane(double x, int lane)
{
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_readlane((int)b, lane);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Group reductions.  Inside each 16-lane row a butterfly over the DPP
// patterns xor 1, xor 2, mirror-in-8 and mirror-in-16: each step adds a
// lane's value to its partner's and the partner adds the same two numbers,
// so every lane of the row ends with the same bits; rows are then combined
// in a fixed order from their last lanes.
template <class Op>
__device__ __forceinline__ double greduce(double x, Op op)
{
    x = op(x, dpp<0xB1>(x));    // quad_perm [1, 0, 3, 2]
    x = op(x, dpp<0x4E>(x));    // quad_perm [2, 3, 0, 1]
    x = op(x, dpp<0x141>(x));   // row_half_mirror
    x = op(x, dpp<0x140>(x));   // row_mirror
    if constexpr (G == 16) {
        return x;
    } else if constexpr (G == 32) {
        const double r0 = readlane(x, 15), r1 = readlane(x, 31), r2 = readlane(x, 47), r3 = readlane(x, 63);
        return gbase() == 0 ? op(r0, r1) : op(r2, r3);
    } else {
        const double r0 = readlane(x, 15), r1 = readlane(x, 31), r2 = readlane(x, 47), r3 = readlane(x, 63);
        return op(op(r0, r1), op(r2, r3));
    }
}

__device__ __forceinline__ double gsum(double x)
{
    return greduce(x, [](double a, double b) { return a + b; });
}

__device__ __forceinline__ double gmax(double x)
{
    return greduce(x, [](double a, double b) { return fmax(a, b); });
}

__device__ __forceinline__ chem_math::Dual gsum(chem_math::Dual x)
{
    return chem_math::Dual(gsum(x.v), gsum(x.d));
}

// bits of this group's lanes in a wave-wide ballot, lane 0 of the group at bit 0
__device__ __forceinline__ unsigned long long gbits(unsigned long long ballot)
{
    if constexpr (G == 64) return ballot;
    else return (ballot >> gbase()) & ((1ull << G) - 1ull);
}

// true in every lane of the group if `bad` holds in any lane of it
__device__ __forceinline__ bool gany(bool bad)
{
    return gbits(__ballot(bad)) != 0ull;
}

// LDS writes of this wave visible to its later LDS reads
__device__ __forceinline__ void lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

template <class S>
__device__ __forceinline__ S ipow(S c, int nu) { return nu == 1 ? c : (nu == 2 ? c * c : c * c * c); }

// d(c^nu)/dc
template <class S>
__device__ __forceinline__ S dipow(S c, int nu) { return nu == 1 ? S(1.0) : (nu == 2 ? 2.0 * c : 3.0 * c * c); }

// add x to an LDS word (only the lane owning the address adds to it)
__device__ __forceinline__ void lds_add(double* p, double x) { atomicAdd(p, x); }
__device__ __forceinline__ void lds_add(chem_math::Dual* p, chem_math::Dual x)
{
    atomicAdd(&p->v, x.v);
    atomicAdd(&p->d, x.d);
}

// Evaluation modes of the source terms: the rates; the rates and the
// Jacobian row; the parameter products w . df/dtheta (adjoint).
enum : int { F_ONLY = 0, F_JAC = 1, PARAM_VJP = 2 };

// Rate of progress of the reaction in slot j, written to the cell's LDS; with
// F_JAC also its partials (d q / d C of each species slot, d q / dT at fixed C,
// and the coefficient of the third-body efficiencies in d q / d C); with
// PARAM_VJP the products of w . df/dq_j with d q_j / d(ln A, b, Ea) added to g.
template <class S, int MODE>
__device__ __forceinline__ void reaction(int j, const unsigned (&pk)[3], const double* __restrict__ par,
                                         S* __restrict__ L, S T, S lnT, S iT, S lnPRT, S ctot, S irho, S rcpinv,
                                         double p, S* __restrict__ g)
{
    constexpr bool JAC = MODE == F_JAC;
    // the slot's packed table entry (loaded by the caller ahead of time)
    // kind: 0 elementary, 1 third body, 2 Lindemann, 3 Troe, 4 SRI, 5 PLOG
    const int kind = (int)(pk[2] & 7u);
    const bool irrev = mech::HAS_IRREV && ((pk[2] >> 3) & 1u);
    const int dnu = (int)((pk[2] >> 4) & 7u) - 4;
    const int er = (int)((pk[2] >> 7) & 511u) - 1;   // EFF row, or PLOG table for kind 5
    const int oj = (int)(pk[2] >> 16);
    double pb = par[NR + oj], pe = par[2 * NR + oj];
    S lnk = lnT * pb;
    lnk = fma(-iT, pe, lnk);
    lnk = lnk + par[oj];
    if (mech::HAS_PLOG && kind == 5) {
        // the Arrhenius set at this pressure: linear in ln p between the
        // tabulated pressures, the end sets outside them
        const double lnp = log(p);
        const int e0 = mech::RX_PLOG_OFF[er], e1 = mech::RX_PLOG_OFF[er + 1] - 1;
        const double* E = mech::RX_PLOG;
        int e = e0;
        double w = 0.0;
        if (lnp >= E[4 * e1]) {
            e = e1;
        } else if (lnp > E[4 * e0]) {
            while (e + 1 < e1 && lnp >= E[4 * (e + 1)]) ++e;
            w = (lnp - E[4 * e]) / (E[4 * (e + 1)] - E[4 * e]);
        }
        const int e2 = e < e1 ? e + 1 : e;
        const double pla = fma(w, E[4 * e2 + 1] - E[4 * e + 1], E[4 * e + 1]);
        const double plb = fma(w, E[4 * e2 + 2] - E[4 * e + 2], E[4 * e + 2]);
        const double ple = fma(w, E[4 * e2 + 3] - E[4 * e + 3], E[4 * e + 3]);
        lnk = lnk + (lnT * plb - iT * ple + pla);
        pb += plb;
        pe += ple;
    }
    int sp[NSLOT], nu[NSLOT];
    S c[NSLOT];
    S lnKc = 0.0, dH = 0.0, ws = 0.0;
#pragma unroll
    for (int s = 0; s < NSLOT; ++s) {
        const unsigned v = (pk[s / 4] >> (8 * (s % 4))) & 255u;
        sp[s] = (int)(v & 63u) - 1;
        nu[s] = (int)(v >> 6);
        c[s] = 1.0;
        if (sp[s] >= 0) {
            const double sgn = s < mech::MAXT ? -(double)nu[s] : (double)nu[s];
            lnKc = fma(sgn, L[mech::L_G + sp[s]], lnKc);
            if (MODE != F_ONLY) dH = fma(sgn, L[mech::L_H + sp[s]], dH);
            if (MODE == PARAM_VJP) ws = fma(sgn * mech::MWTAB[sp[s]], L[mech::L_W + 1 + sp[s]], ws);
            c[s] = L[mech::L_C + sp[s]];
        }
    }
    lnKc = fma((double)dnu, lnPRT, lnKc);
    S Mc = ctot;
    if (er >= 0 && !(mech::HAS_PLOG && kind == 5)) {
        for (int m = 0; m < NS; ++m) Mc = fma(mech::EFF[er * NS + m] - 1.0, L[mech::L_C + m], Mc);
    }
    S kf, kr, kinf = 0.0, r0 = 0.0, Fb = 1.0, ipr1 = 0.0, iKc = 0.0, Pr = 0.0;
    S dF_dPr = 0.0, dF_dFc = 0.0, dlogFc_dT = 0.0, dlnF_T = 0.0;
    if (kind < 2 || (mech::HAS_PLOG && kind == 5)) {
        kf = chem_math::exp_poly(lnk);
        kr = irrev ? S(0.0) : chem_math::exp_poly(lnk - lnKc);
    } else {
        // P_r = k0 [M] / k_inf, one exponential for the ratio
        const double* lo = &mech::RX_LOW[j * 3];
        kinf = chem_math::exp_poly(lnk);
        const S lnr0 = lo[0] + lo[1] * lnT - lo[2] * iT - lnk;
        r0 = chem_math::exp_poly(lnr0);
        Pr = r0 * Mc;
        const bool floored = !(Pr >= 1e-300);
        const S logPr = floored ? S(-300.0) : log10(Pr);
        if (kind == 3) {
            const double* tr = &mech::RX_TROE[j * 8];
            const S e3 = chem_math::exp_poly(-T * tr[2]);
            const S e1 = chem_math::exp_poly(-T * tr[3]);
            S Fc = tr[0] * e3 + tr[1] * e1;
            S dFc = tr[5] * e3 + tr[6] * e1;
            if (tr[7] != 0.0) {
                const S e2 = chem_math::exp_poly(-tr[4] * iT);
                Fc += e2;
                dFc += tr[4] * iT * iT * e2;
            }
            const S logFc = log10(Fc);
            const S tc = -0.4 - 0.67 * logFc;
            const S tn = 0.75 - 1.27 * logFc;
            const S tu = logPr + tc;
            const S tden = tn - 0.14 * tu;
            const S tx = tu / tden;
            const S opx2 = 1.0 + tx * tx;
            const S logF = logFc / opx2;
            Fb = chem_math::exp_poly(mech::LN10 * logF);
            if (MODE != F_ONLY) {
                const S tg = -logFc * 2.0 * tx / (opx2 * opx2);
                dF_dPr = floored ? S(0.0) : tg * tn / (tden * tden);
                dF_dFc = 1.0 / opx2 + tg * (-0.67 * tn + 1.27 * tu) / (tden * tden);
                dlogFc_dT = dFc / (Fc * mech::LN10);
                dlnF_T = mech::LN10 * dF_dFc * dlogFc_dT;
            }
        } else if (mech::HAS_SRI && kind == 4) {
            // SRI: F = d [a exp(-b/T) + exp(-T/c)]^X T^e, X = 1 / (1 + log10(P_r)^2);
            // row: a, -b, 1/c, b, ln d, e
            const double* sr = &mech::RX_TROE[j * 8];
            const S sea = sr[0] * chem_math::exp_poly(sr[1] * iT);
            const S sec = chem_math::exp_poly(-T * sr[2]);
            const S sY = sea + sec;
            const S lnsY = log(sY);
            const S sX = 1.0 / (1.0 + logPr * logPr);
            Fb = chem_math::exp_poly(sX * lnsY + sr[5] * lnT + sr[4]);
            if (MODE != F_ONLY) {
                dF_dPr = floored ? S(0.0) : lnsY * (-2.0 / mech::LN10) * logPr * sX * sX;
                dlnF_T = sX * (sea * sr[3] * iT * iT - sec * sr[2]) / sY + sr[5] * iT;
            }
        }
        ipr1 = 1.0 / (1.0 + Pr);
        kf = kinf * Pr * ipr1 * Fb;
        iKc = irrev ? S(0.0) : chem_math::exp_poly(-lnKc);
        kr = kf * iKc;
    }
    S pf = 1.0, pr = 1.0;
#pragma unroll
    for (int s = 0; s < NSLOT; ++s) {
        if (sp[s] >= 0) {
            if (s < mech::MAXT) pf *= ipow(c[s], nu[s]);
            else pr *= ipow(c[s], nu[s]);
        }
    }
    const S fwd = kf * pf, rev = kr * pr;
    const S q = kind == 1 ? Mc * (fwd - rev) : fwd - rev;
    if (MODE == PARAM_VJP) {
        // w . df/dq_j: species rows W_k nu_kj / rho, temperature row
        // -R T (sum nu H/RT) / (rho c_p); d q / d ln A of the main rate (k_inf
        // for falloff, through P_r = k0 [M] / k_inf)
        const S wsum = ws * irho - L[mech::L_W] * (mech::RU * T) * dH * rcpinv;
        const S qA = (kind >= 2 && !(mech::HAS_PLOG && kind == 5)) ? q * (Pr * ipr1 - dF_dPr) : q;
        const S gq = wsum * qA;
        g[0] += gq;
        g[1] += gq * lnT;
        g[2] += gq * (-iT * (1.0 / mech::RU));
        return;
    }
    L[mech::L_Q + j] = q;
    if (!JAC) return;
    S* P = L + mech::L_P + j * PW;
    const S fac = kind == 1 ? Mc : S(1.0);
    const S dlnKc = (dH - (double)dnu) * iT;
    const S dlnkinf = (pb + pe * iT) * iT;
    S dlnkf = dlnkinf;
    S dM = kind == 1 ? fwd - rev : S(0.0);
    if (kind >= 2 && !(mech::HAS_PLOG && kind == 5)) {
        const double* lo = &mech::RX_LOW[j * 3];
        const S dlnk0 = (lo[1] + lo[2] * iT) * iT;
        dlnkf = dlnkinf + (ipr1 + dF_dPr) * (dlnk0 - dlnkinf) + dlnF_T;
        const S dkdM = kinf * r0 * Fb * (ipr1 * ipr1 + dF_dPr * ipr1);
        dM = dkdM * (pf - iKc * pr);
    }
    P[NSLOT] = fac * (dlnkf * fwd - (dlnkf - dlnKc) * rev);
    P[NSLOT + 1] = dM;
#pragma unroll
    for (int s = 0; s < NSLOT; ++s) {
        // derivative of this side's product with respect to the slot's species
        S d = 0.0;
        if (sp[s] >= 0) {
            const int lo = s < mech::MAXT ? 0 : mech::MAXT;
            d = dipow(c[s], nu[s]);
#pragma unroll
            for (int t = 0; t < mech::MAXT; ++t)
                if (lo + t != s && sp[lo + t] >= 0) d *= ipow(c[lo + t], nu[lo + t]);
            d = s < mech::MAXT ? fac * kf * d : -fac * kr * d;
        }
        P[s] = d;
    }
}

// Source terms f = dy/dt of the group's cell at the state whose component i
// is yi (lane i); with F_JAC row i of the Jacobian in A; with PARAM_VJP
// (weights w, component wi in lane i) the products w . df/dtheta of the
// lane's reaction slots r G + i added to g[r].  Every lane of the group calls
// it together.  S is double, or a dual number for directional derivatives.
template <class S, int MODE>
__device__ __forceinline__ S rhs(const double* __restrict__ par, double p, double ip, S yi, S* __restrict__ L,
                                 S (&A)[N], S wi, S (&g)[ROUNDS][3])
{
    constexpr bool JAC = MODE == F_JAC;
    const int i = gl();
    const bool sp = i >= 1 && i <= NS;
    const int k = sp ? i - 1 : 0;
    // constant tables at an opaque offset: their uniform loads stay inside this
    // evaluation instead of being hoisted out of the substep loop into SGPRs
    const int z = mech::opaque_zero();
    mech::cdbl* MW = (mech::cdbl*)&mech::MWTAB[0] + z;
    // the packed table entries of the lane's reaction slots, loaded now so the
    // loads overlap the thermo phase
    unsigned pk[ROUNDS][3];
#pragma unroll
    for (int r = 0; r < ROUNDS; ++r) {
        const int j = r * G + i;
#pragma unroll
        for (int q = 0; q < 3; ++q) pk[r][q] = j < NR ? (unsigned)mech::RX_PACK[3 * j + q] : 0u;
    }
    if (i < N) {
        L[mech::L_Y + i] = yi;
        if (MODE == PARAM_VJP) L[mech::L_W + i] = wi;
    }
    lds_sync();
    const S T = L[mech::L_Y];
    const S lnT = log(T);
    const S iT = chem_math::recip(T);
    const S T2 = T * T, T3 = T2 * T, T4 = T2 * T2;
    S cpR = 0.0, HRT = 0.0, Gk = 0.0, dcpR = 0.0;
    if (sp) {
        const double* c = &mech::THERMO[k][T < mech::TMID[k] ? 0 : 1][0];
        S a = T4 * c[4];
        a = fma(T3, c[3], a);
        a = fma(T2, c[2], a);
        a = fma(T, c[1], a);
        cpR = a + c[0];
        a = T4 * c[8];
        a = fma(T3, c[7], a);
        a = fma(T2, c[6], a);
        a = fma(T, c[5], a);
        a = fma(iT, c[9], a);
        HRT = a + c[0];
        a = T4 * c[13];
        a = fma(T3, c[12], a);
        a = fma(T2, c[11], a);
        a = fma(T, c[10], a);
        a = fma(lnT, c[0], a);
        a = fma(-iT, c[9], a);
        Gk = a + c[14];
        if (JAC) {
            a = T3 * c[18];
            a = fma(T2, c[17], a);
            a = fma(T, c[16], a);
            dcpR = a + c[15];
        }
    }
    const double W = sp ? MW[k] : 0.0;
    const double iW = sp ? MW[NS + k] : 0.0;
    const S yw = sp ? yi * iW : S(0.0);
    const S sig = gsum(yw);
    const S Wbar = chem_math::recip(sig);
    const S rho = p * Wbar * iT * (1.0 / mech::RU);
    const S irho = mech::RU * T * sig * ip;
    const S ctot = p * iT * (1.0 / mech::RU);
    if (sp) {
        L[mech::L_C + k] = rho * yw;
        L[mech::L_G + k] = Gk;
        L[mech::L_H + k] = HRT;
    }
    lds_sync();
    const S lnPRT = mech::LN_PATM_R - lnT;
    if (MODE == PARAM_VJP) {
        const S rcp = T * sig * ip / gsum(cpR * yw);
#pragma unroll
        for (int r = 0; r < ROUNDS; ++r) {
            const int j = r * G + i;
            if (j < NR) reaction<S, MODE>(j, pk[r], par, L, T, lnT, iT, lnPRT, ctot, irho, rcp, p, g[r]);
        }
        return S(0.0);
    }
#pragma unroll 1
    for (int r = 0; r < ROUNDS; ++r) {
        const int j = r * G + i;
        unsigned pr[3] = {pk[0][0], pk[0][1], pk[0][2]};
#pragma unroll
        for (int q = 1; q < ROUNDS; ++q)
#pragma unroll
            for (int t = 0; t < 3; ++t) pr[t] = (q == r) ? pk[q][t] : pr[t];
        if (j < NR) reaction<S, MODE>(j, pr, par, L, T, lnT, iT, lnPRT, ctot, irho, irho, p, g[0]);
    }
    lds_sync();
    // species lists come padded to multiples of 4: four entries' loads in flight
    const S* __restrict__ Q = L + mech::L_Q;
    S wdot = 0.0;
    if (sp) {
        const int e1 = mech::SP_OFF[k + 1];
        for (int e = mech::SP_OFF[k]; e < e1; e += 4) {
            S q[4];
            double nu[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                nu[u] = (double)mech::SP_NU[e + u];
                q[u] = Q[mech::SP_RX[e + u]];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) wdot = nu[u] != 0.0 ? fma(nu[u], q[u], wdot) : wdot;
        }
    }
    const S cpm = gsum(cpR * yw);
    const S hw = gsum(HRT * wdot);
    const S icpm = chem_math::recip(cpm);
    const S rcpinv = T * sig * ip * icpm;
    const S fT = -mech::RU * T * hw * rcpinv;
    const S fk = W * (irho * wdot);
    const S fi = sp ? fk : (i == 0 ? fT : S(0.0));
    if (!JAC) return fi;

    // Row k of the concentration Jacobian: Jc_km = d wdot_k / d C_m (fixed T)
    // and wT_k = d wdot_k / dT (fixed C) in column NS.  The species partials
    // of the lane's reactions go into its own LDS row by atomic adds (one
    // lane per address, applied in program order: reproducible); the
    // third-body part, dense over m, accumulates in registers.
    S* Jr = L + mech::L_J + k * JW;
    if (sp) {
#pragma unroll
        for (int m = 0; m <= NS; ++m) Jr[m] = 0.0;
    }
    lds_sync();
    if (sp) {
        const S* __restrict__ Pb = L + mech::L_P;
        const int e1 = mech::SP_OFF[k + 1];
        for (int e = mech::SP_OFF[k]; e < e1; e += 4) {
            // one round of independent table loads per four entries (slot,
            // coefficient and slot species packed per entry), then the partials
            unsigned w[4][3];
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int q = 0; q < 3; ++q) w[u][q] = (unsigned)mech::SP_JPACK[3 * (e + u) + q];
            int j[4], ms[4][NSLOT];
            double nu[4];
            S P[4][NSLOT + 1];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                j[u] = (int)(w[u][0] & 0xffffu);
                nu[u] = (double)(signed char)(w[u][0] >> 16);
#pragma unroll
                for (int s = 0; s < NSLOT; ++s) ms[u][s] = (int)((w[u][1 + s / 4] >> (8 * (s % 4))) & 255u) - 1;
#pragma unroll
                for (int s = 0; s <= NSLOT; ++s) P[u][s] = Pb[j[u] * PW + s];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                if (nu[u] == 0.0) continue;
#pragma unroll
                for (int s = 0; s < NSLOT; ++s)
                    if (ms[u][s] >= 0) lds_add(&Jr[ms[u][s]], nu[u] * P[u][s]);
                lds_add(&Jr[NS], nu[u] * P[u][NSLOT]);
            }
        }
    }
    S R[NS + 1];
#pragma unroll
    for (int m = 0; m <= NS; ++m) R[m] = 0.0;
    // the efficiencies by scalar loads at an opaque offset, so they are loaded
    // here, one reaction at a time, not hoisted out of the substep loop
    mech::cdbl* EF = (mech::cdbl*)&mech::EFF[0] + z;
    // the lane's coefficients in all of them: one load per eight reactions,
    // ahead of the loop (4-bit fields, coefficient + 8)
    unsigned tbw[mech::NTBW];
#pragma unroll
    for (int q = 0; q < mech::NTBW; ++q) tbw[q] = sp ? (unsigned)mech::NU_TB4[k * mech::NTBW + q] : 0x88888888u;
#pragma unroll
    for (int q = 0; q < mech::NTBW; ++q) {
#pragma unroll 1
        for (int t = 8 * q; t < mech::NTB && t < 8 * q + 8; ++t) {
            const double nut = (double)((int)((tbw[q] >> (4 * (t - 8 * q))) & 15u) - 8);
            const S d = nut * L[mech::L_P + mech::TB_SLOT[t] * PW + NSLOT + 1];
            mech::cdbl* eff = EF + t * NS;
#pragma unroll
            for (int m = 0; m < NS; ++m) R[m] = fma(eff[m], d, R[m]);
        }
    }
    lds_sync();
    if (sp) {
#pragma unroll
        for (int m = 0; m <= NS; ++m) R[m] += Jr[m];
#pragma unroll
        for (int m = 0; m <= NS; ++m) Jr[m] = R[m];
    }
    lds_sync();
    // chain rule to (T, Y), with S_k = sum_l Jc_kl C_l:
    //   J_km = (W_k/W_m) Jc_km + (Wbar/W_m)(f_k - W_k S_k / rho)
    //   J_k0 = (W_k / rho)(wT_k - S_k / T) + f_k / T
    //   J_0m = -R T (rho HJ_m - Wbar HS) / (W_m rho cp) - f_T (cp_m / cp - Wbar / W_m)
    //   J_00 = -R (cpw + T HwT - HS) / (rho cp) - f_T (dcp / cp - 1/T)
    // HJ_m = sum_k H_k/RT Jc_km, HS = sum_k H_k/RT S_k, HwT = sum_k H_k/RT wT_k,
    // cpw = sum_k cp_k/R wdot_k
    S Sk = 0.0, wT = 0.0;
    if (sp) {
#pragma unroll
        for (int m = 0; m < NS; ++m) Sk = fma(R[m], L[mech::L_C + m], Sk);
        wT = R[NS];
    }
    const S HS = gsum(HRT * Sk);
    const S HwT = gsum(HRT * wT);
    const S cpw = gsum(cpR * wdot);
    const S dcpm = gsum(dcpR * yw);
    const S RT = mech::RU * T;
    const S icp = icpm * (1.0 / mech::RU);
    const S dcp = mech::RU * dcpm;
    if (sp) {
        S HJ = 0.0;
        for (int l = 0; l < NS; ++l) HJ = fma(L[mech::L_H + l], L[mech::L_J + l * JW + k], HJ);
        const S t = fma(rho, HJ, -Wbar * HS) * (-RT * rcpinv);
        const S u = fma(cpR, icp * mech::RU, -Wbar);
        L[mech::L_T0 + k] = fma(-fT, u, t) * iW;
    }
    lds_sync();
    if (sp) {
        const S gk = fma(-W, Sk * irho, fk);
        const S wg = Wbar * gk;
#pragma unroll
        for (int m = 0; m < NS; ++m) A[1 + m] = fma(R[m], W, wg) * MW[NS + m];
        A[0] = fma(W * irho, wT - Sk * iT, fk * iT);
    } else if (i == 0) {
        A[0] = -mech::RU * (cpw + T * HwT - HS) * rcpinv - fT * (dcp * icp - iT);
#pragma unroll
        for (int m = 0; m < NS; ++m) A[1 + m] = L[mech::L_T0 + m];
    } else {
#pragma unroll
        for (int m = 0; m < N; ++m) A[m] = 0.0;
    }
    return fi;
}

// LU with partial pivoting of the group's matrix (row i in lane i), in place:
// multipliers below the diagonal, U above, reciprocal pivots on the diagonal.
// PV: LDS scratch of the cell for the pivot row (N doubles) and, after it, the
// pivot indices: piv[k] is the row swapped into k at step k (LINPACK order,
// the lowest row index among equal magnitudes).  Bit k of the result: some
// group of the wave swapped at step k.
__device__ __forceinline__ unsigned long long lu(double (&A)[N], bool& ok, double* __restrict__ PV)
{
    const int i = gl_local();
    double* PR = PV;
    int* piv = (int*)(PV + N);      // read by the solves only on a swap
    unsigned long long swaps = 0ull;
    ok = true;
#pragma unroll
    for (int k = 0; k < N; ++k) {
        // the column's largest magnitude (a max is exact in any order), then the
        // lowest row that reaches it
        const double v = (i >= k && i < N) ? fabs(A[k]) : -1.0;
        const double vmax = gmax(v);
        const unsigned long long hit = gbits(__ballot(v == vmax));
        int idx = hit ? __builtin_ctzll(hit) : k;
        if (!(vmax > 0.0)) idx = k;
        if (i == 0) piv[k] = idx;
        ok = ok && (vmax > 0.0);
        if (__any(idx != k)) {
            swaps |= 1ull << k;
            const int src = (i == k) ? idx : (i == idx ? k : i);
#pragma unroll
            for (int j = k; j < N; ++j) A[j] = gather(A[j], src);
        }
        // the pivot row: with one cell per wave read straight from the pivot
        // lane into scalar registers; otherwise through LDS (one lane writes
        // it, every lane of the group reads it)
        double prow[N];
        if constexpr (G == 64) {
#pragma unroll
            for (int j = k; j < N; ++j) prow[j] = bcast(A[j], k);
        } else {
            if (i == k) {
#pragma unroll
                for (int j = k; j < N; ++j) PR[j] = A[j];
            }
            lds_sync();
#pragma unroll
            for (int j = k; j < N; ++j) prow[j] = PR[j];
            lds_sync();
        }
        const double rp = chem_math::recip(prow[k]);
        if (i == k) {
            A[k] = rp;
        } else if (i > k && i < N) {
            const double l = A[k] * rp;
            A[k] = l;
#pragma unroll
            for (int j = k + 1; j < N; ++j) A[j] = fma(-l, prow[j], A[j]);
        }
    }
    return swaps;
}

// Solve (LU) x = b for the group's vector b (component i in lane i).
__device__ __forceinline__ double solve(const double (&A)[N], const double* __restrict__ PV,
                                        unsigned long long swaps, double b)
{
    const int i = gl_local();
    const int* piv = (const int*)(PV + N);
#pragma unroll
    for (int k = 0; k < N; ++k) {
        if (swaps & (1ull << k)) {
            const int pk = piv[k];
            b = gather(b, (i == k) ? pk : (i == pk ? k : i));
        }
        const double zk = bcast(b, k);
        if (i > k && i < N) b = fma(-A[k], zk, b);
    }
#pragma unroll
    for (int k = N - 1; k >= 0; --k) {
        if (i == k) b *= A[k];
        const double zk = bcast(b, k);
        if (i < k) b = fma(-A[k], zk, b);
    }
    return b;
}

// One RODAS4 step from y (component yi) with step h; false if the step
// matrix is singular or a result is not finite.  L: the cell's scratch, PV:
// its pivot scratch.
__device__ __forceinline__ bool ros_step(const double* __restrict__ par, double p, double ip, double yi, double h,
                                         double rtol, double atol, double* __restrict__ L, double* __restrict__ PV,
                                         double& ynew, double& errn)
{
    const int i = gl_local();
    double A[N];
    double g[ROUNDS][3];
    const double f0 = rhs<double, F_JAC>(par, p, ip, yi, L, A, 0.0, g);
    const double hinv = chem_math::recip(h);
    const double ghinv = hinv * (1.0 / Rodas4::gamma);
#pragma unroll
    for (int j = 0; j < N; ++j) A[j] = (j == i ? ghinv : 0.0) - A[j];
    bool ok;
    const unsigned long long swaps = lu(A, ok, PV);
    double u[Rodas4::S];
    u[0] = solve(A, PV, swaps, f0);
#pragma unroll
    for (int s = 1; s < Rodas4::S; ++s) u[s] = 0.0;
    double dummy[N];
    // one copy of the source-term code for the five later stages (the kernel
    // stays inside the instruction cache); stage vectors stay in registers
#pragma unroll 1
    for (int s = 1; s < Rodas4::S; ++s) {
        double Ys = yi, acc = 0.0;
#pragma unroll
        for (int j = 0; j < Rodas4::S - 1; ++j) {
            if (j < s) {
                Ys = fma(RA[s][j], u[j], Ys);
                acc = fma(RC[s][j], u[j], acc);
            }
        }
        if (s == Rodas4::S - 1) ynew = Ys;
        const double fs = rhs<double, F_ONLY>(par, p, ip, Ys, L, dummy, 0.0, g);
        const double us = solve(A, PV, swaps, fma(acc, hinv, fs));
#pragma unroll
        for (int j = 1; j < Rodas4::S; ++j)
            if (j == s) u[j] = us;
    }
    ynew += u[Rodas4::S - 1];
    const double sc = atol + rtol * fmax(fabs(yi), fabs(ynew));
    const double e = u[Rodas4::S - 1] * chem_math::recip(sc);
    errn = sqrt(gsum(i < N ? e * e : 0.0) * (1.0 / N));
    const bool bad = gany(i < N && !finite(ynew));
    return ok && !bad && finite(errn);
}

// Per-group integration state (component yi in lane i, the rest replicated).
struct Cell {
    double y, p, ip, t, h;
    int nacc, nrej, status;
    bool rej_last, done;
};

__device__ __forceinline__ void cell_begin(Cell& c, double T, double p, const double* __restrict__ Y, double h0)
{
    const int i = gl();
    c.y = i == 0 ? T : (i <= NS ? Y[i - 1] : 0.0);
    c.p = p;
    c.ip = 1.0 / p;
    c.t = 0.0;
    c.h = h0;
    c.nacc = 0;
    c.nrej = 0;
    c.rej_last = false;
    const bool bad = gany(!finite(c.y)) || !(T > 0.0) || !(p > 0.0) || !finite(p);
    c.status = bad ? chem::CELL_BADINPUT : chem::CELL_OK;
    c.done = bad;
}

// One attempted substep with the controller of the one-cell-per-lane form;
// returns the step size if the step was accepted, else 0.
__device__ __forceinline__ double cell_attempt(Cell& c, const double* __restrict__ par, const StepArgs& a,
                                               double* __restrict__ L, double* __restrict__ PV)
{
    if (c.done) return 0.0;
    if (c.nacc + c.nrej >= a.max_substeps) {
        c.status = chem::CELL_MAXSTEPS;
        c.done = true;
        return 0.0;
    }
    if (c.h < a.hmin) {
        c.status = chem::CELL_HMIN;
        c.done = true;
        return 0.0;
    }
    bool last = false;
    double h = c.h;
    if (h >= a.dt - c.t) {
        h = a.dt - c.t;
        last = true;
    }
    double ynew, en;
    const bool ok = ros_step(par, c.p, c.ip, c.y, h, a.rtol, a.atol, L, PV, ynew, en);
    if (ok && en <= 1.0) {
        c.y = ynew;
        c.t = last ? a.dt : c.t + h;
        double fac = 0.9 * chem::inv_root4(fmax(en, 1e-16));
        fac = fmin(6.0, fmax(0.2, fac));
        if (c.rej_last) fac = fmin(1.0, fac);
        c.h = h * fac;
        c.rej_last = false;
        ++c.nacc;
        if (last) c.done = true;
        return h;
    }
    ++c.nrej;
    c.h = h * (ok ? fmax(0.2, 0.9 * chem::inv_root4(en)) : 0.2);
    c.rej_last = true;
    return 0.0;
}

__device__ __forceinline__ void cell_store(const Cell& c, double* __restrict__ T, double* __restrict__ Y, long cell,
                                           int* status, int* nacc, int* nrej)
{
    const int i = gl();
    if (c.status != chem::CELL_BADINPUT) {
        if (i == 0) T[cell] = c.y;
        else if (i <= NS) Y[cell * NS + i - 1] = c.y;
    }
    if (i == 0) {   // the per-cell counters only where someone reads them (null: not asked for)
        if (status) status[cell] = c.status;
        if (nacc) nacc[cell] = c.nacc;
        if (nrej) nrej[cell] = c.nrej;
    }
}

// ---- discrete adjoint of the frozen-step map (see the one-cell-per-lane form
// for the algebra); every vector one component per lane ----

// Solve M^T x = b with the factors of lu(): U^T y = b forward, then, for
// k = N-1 .. 0, y_k -= sum_{i>k} l_ik y_i and swap y_k, y_piv[k].  The row
// sums a column needs are group sums.
__device__ __forceinline__ double solve_t(const double (&A)[N], const double* __restrict__ PV,
                                          unsigned long long swaps, double b)
{
    const int i = gl_local();
    const int* piv = (const int*)(PV + N);
    double y = b;
#pragma unroll
    for (int k = 0; k < N; ++k) {
        const double s = gsum(i < k ? A[k] * y : 0.0);
        if (i == k) y = (y - s) * A[k];
    }
#pragma unroll
    for (int k = N - 1; k >= 0; --k) {
        const double s = gsum(i > k && i < N ? A[k] * y : 0.0);
        if (i == k) y -= s;
        if (swaps & (1ull << k)) {
            const int pk = piv[k];
            y = gather(y, (i == k) ? pk : (i == pk ? k : i));
        }
    }
    return y;
}

// Component i of J^T w for the group's rows of J (row i in lane i).
__device__ __forceinline__ double colsum(const double (&J)[N], double w)
{
    const int i = gl_local();
    double out = 0.0;
#pragma unroll
    for (int k = 0; k < N; ++k) {
        const double s = gsum(J[k] * w);
        out = (i == k) ? s : out;
    }
    return out;
}

// Component i of D_u[J^T w] from dual rows of J (tangent along u).
__device__ __forceinline__ double colsum_tangent(const chem_math::Dual (&J)[N], double w)
{
    const int i = gl_local();
    double out = 0.0;
#pragma unroll
    for (int k = 0; k < N; ++k) {
        const double s = gsum(J[k].d * w);
        out = (i == k) ? s : out;
    }
    return out;
}

// value of a stage-indexed register array at a run-time stage s (selects, so
// the array stays in registers)
__device__ __forceinline__ double pick(const double (&v)[Rodas4::S], int s)
{
    double r = v[0];
#pragma unroll
    for (int q = 1; q < Rodas4::S; ++q) r = (q == s) ? v[q] : r;
    return r;
}

__device__ __forceinline__ void place(double (&v)[Rodas4::S], int s, double x)
{
#pragma unroll
    for (int q = 0; q < Rodas4::S; ++q) v[q] = (q == s) ? x : v[q];
}

// The adjoint of one frozen RODAS4 step from y (component yi) with step h:
// lam (the cotangent of y_new, component in lane i) becomes the cotangent of
// y; the parameter products of the lane's reaction slots are added to g.
// L: the cell's scratch (room for dual numbers), PV: its pivot scratch.  The
// stage loops stay rolled (one copy of each source-term evaluation).
__device__ __noinline__ void step_adjoint(const double* __restrict__ par, double p, double ip, double yi, double h,
                                          double& lam, double (&g)[ROUNDS][3], double* __restrict__ L,
                                          double* __restrict__ PV)
{
    using chem_math::Dual;
    const int i = gl_local();
    double J0[N], A[N], dummy[N];
    const double f0 = rhs<double, F_JAC>(par, p, ip, yi, L, J0, 0.0, g);
    const double hinv = chem_math::recip(h);
    const double ghinv = hinv * (1.0 / Rodas4::gamma);
#pragma unroll
    for (int j = 0; j < N; ++j) A[j] = (j == i ? ghinv : 0.0) - J0[j];
    bool ok;
    const unsigned long long swaps = lu(A, ok, PV);
    double u[Rodas4::S], Ys[Rodas4::S];
#pragma unroll
    for (int s = 0; s < Rodas4::S; ++s) u[s] = Ys[s] = 0.0;
    Ys[0] = yi;
    u[0] = solve(A, PV, swaps, f0);
#pragma unroll 1
    for (int s = 1; s < Rodas4::S; ++s) {
        double Y = yi, acc = 0.0;
#pragma unroll
        for (int j = 0; j < Rodas4::S - 1; ++j) {
            if (j < s) {
                Y = fma(RA[s][j], u[j], Y);
                acc = fma(RC[s][j], u[j], acc);
            }
        }
        place(Ys, s, Y);
        const double fs = rhs<double, F_ONLY>(par, p, ip, Y, L, dummy, 0.0, g);
        place(u, s, solve(A, PV, swaps, fma(acc, hinv, fs)));
    }
    // reverse over the stages
    const double mw[Rodas4::S] = {RA[5][0], RA[5][1], RA[5][2], RA[5][3], 1.0, 1.0};
    double ub[Rodas4::S], w[Rodas4::S];
    double yb = lam;
#pragma unroll
    for (int s = 0; s < Rodas4::S; ++s) {
        ub[s] = mw[s] * lam;
        w[s] = 0.0;
    }
#pragma unroll 1
    for (int s = Rodas4::S - 1; s >= 0; --s) {
        const double ws = solve_t(A, PV, swaps, pick(ub, s));
        place(w, s, ws);
        const double Yss = pick(Ys, s);
        double Js[N];
        if (s == 0) {
#pragma unroll
            for (int j = 0; j < N; ++j) Js[j] = J0[j];
        } else {
            rhs<double, F_JAC>(par, p, ip, Yss, L, Js, 0.0, g);
        }
        const double Yb = colsum(Js, ws);
        yb += Yb;
        rhs<double, PARAM_VJP>(par, p, ip, Yss, L, dummy, ws, g);
#pragma unroll
        for (int j = 0; j < Rodas4::S - 1; ++j)
            if (j < s) ub[j] = fma(RA[s][j], Yb, fma(RC[s][j] * hinv, ws, ub[j]));
    }
    // second-order terms at y: J(y) inside M, one dual evaluation per stage direction
    Dual* Ld = (Dual*)L;
#pragma unroll 1
    for (int s = 0; s < Rodas4::S; ++s) {
        const double us = pick(u, s), ws = pick(w, s);
        Dual Jd[N];
        Dual gd[ROUNDS][3];
#pragma unroll
        for (int r = 0; r < ROUNDS; ++r) gd[r][0] = gd[r][1] = gd[r][2] = 0.0;
        rhs<Dual, F_JAC>(par, p, ip, Dual(yi, us), Ld, Jd, Dual(0.0), gd);
        yb += colsum_tangent(Jd, ws);
        rhs<Dual, PARAM_VJP>(par, p, ip, Dual(yi, us), Ld, Jd, Dual(ws), gd);
#pragma unroll
        for (int r = 0; r < ROUNDS; ++r) {
            g[r][0] += gd[r][0].d;
            g[r][1] += gd[r][1].d;
            g[r][2] += gd[r][2].d;
        }
    }
    lam = yb;
}

}  // namespace chemw

// ---- plain form: one group of G lanes per cell, cells in index order ----
extern "C" __global__ void __launch_bounds__(64, 2) chem_plain(chem::IntegrateArgs a)
{
    using namespace chemw;
    extern __shared__ double lds[];
    const int grp = (int)threadIdx.x / G;
    const long cell = (long)blockIdx.x * CPW + grp;
    if (cell >= a.ncell) return;
    double* L = lds + grp * mech::LDS_CELL;
    Cell c;
    cell_begin(c, a.T[cell], a.p[cell], a.Y + cell * NS, a.h0 ? a.h0[cell] : a.step.dt);
    while (!c.done) cell_attempt(c, a.par, a.step, L, L + mech::L_J);
    cell_store(c, a.T, a.Y, cell, a.status, a.nacc, a.nrej);
}

// ---- source terms and Jacobian at given states ----
extern "C" __global__ void __launch_bounds__(64) chem_eval(EvalArgs a)
{
    using namespace chemw;
    extern __shared__ double lds[];
    const int grp = (int)threadIdx.x / G;
    const long cell = (long)blockIdx.x * CPW + grp;
    if (cell >= a.ncell) return;
    double* L = lds + grp * mech::LDS_CELL;
    const int i = gl();
    const double p = a.p[cell];
    const double yi = i == 0 ? a.T[cell] : (i <= NS ? a.Y[cell * NS + i - 1] : 0.0);
    double A[N];
    double g[ROUNDS][3];
    double f;
    if (a.J) {
        f = rhs<double, F_JAC>(a.par, p, 1.0 / p, yi, L, A, 0.0, g);
        if (i < N) {
#pragma unroll
            for (int j = 0; j < N; ++j) a.J[(cell * N + i) * N + j] = A[j];
        }
    } else {
        f = rhs<double, F_ONLY>(a.par, p, 1.0 / p, yi, L, A, 0.0, g);
    }
    if (i < N) a.f[cell * N + i] = f;
}

// ---- one fixed RODAS4 step of size h per cell (y_new and the error norm) ----
struct FixedStepArgs {
    const double* par;
    const double* T;
    const double* p;
    const double* Y;
    long ncell;
    double h;
    double* ynew;   // [ncell][N]
    double* err;    // [ncell]
    double rtol, atol;
    int* ok;
};

extern "C" __global__ void __launch_bounds__(64) chem_fixed_step(FixedStepArgs a)
{
    using namespace chemw;
    extern __shared__ double lds[];
    const int grp = (int)threadIdx.x / G;
    const long cell = (long)blockIdx.x * CPW + grp;
    if (cell >= a.ncell) return;
    double* L = lds + grp * mech::LDS_CELL;
    const int i = gl();
    const double p = a.p[cell];
    const double yi = i == 0 ? a.T[cell] : (i <= NS ? a.Y[cell * NS + i - 1] : 0.0);
    double yn, en;
    const bool ok = ros_step(a.par, p, 1.0 / p, yi, a.h, a.rtol, a.atol, L, L + mech::L_J, yn, en);
    if (i < N) a.ynew[cell * N + i] = yn;
    if (i == 0) {
        a.err[cell] = en;
        a.ok[cell] = ok ? 1 : 0;
    }
}

// ---- persistent form: groups pull cells from one global counter ----
// Cells of all fields form one index space [0, total); each group takes the
// next cell when its current one is done, so no group idles while cells
// remain (the hardware already balances whole waves; this also balances the
// groups inside a wave and spans several fields in one launch).
extern "C" __global__ void __launch_bounds__(64, 2) chem_persistent(const PersistBlock* __restrict__ blk,
                                                                 unsigned long long* __restrict__ heads,
                                                                 const double* __restrict__ par)
{
    using namespace chemw;
    extern __shared__ double lds[];
    const int grp = (int)threadIdx.x / G;
    double* L = lds + grp * mech::LDS_CELL;
    const StepArgs step = blk->step;
    const long total = blk->total;
    Cell c;
    c.done = true;
    bool have = false, exhausted = false;
    long local = 0;
    int f = 0;
    while (true) {
        if (!have && !exhausted) {
            unsigned long long t = 0ull;
            if (gl() == 0) t = atomicAdd(heads, 1ull);
            t = (unsigned long long)__shfl((long long)t, gbase(), 64);
            if ((long)t < total) {
                f = field_of(blk, (long)t);
                const FieldDesc& fd = blk->fields[f];
                local = (long)t - fd.start;
                cell_begin(c, fd.T[local], fd.p[local], fd.Y + local * NS, step.dt);
                have = true;
            } else {
                exhausted = true;
            }
        }
        if (__all(exhausted)) break;
        if (have) {
            cell_attempt(c, par, step, L, L + mech::L_J);
            if (c.done) {
                const FieldDesc& fd = blk->fields[f];
                cell_store(c, fd.T, fd.Y, local, fd.status, fd.nacc, fd.nrej);
                have = false;
            }
        }
    }
}

// ---- discrete adjoint: one group per cell, cells in descending cost order ----
// The forward solve is rerun, storing every accepted step size and the state
// every K accepted steps; then the reverse sweep recomputes each segment from
// its checkpoint and applies the step adjoints backwards.  Per-cell parameter
// gradients go to gpar for the fixed-order reduction.
// Group s (of a.nslot) takes the cells in positions s, s + nslot, ... of the
// cost order and keeps the parameter gradients of all its cells in its lanes'
// registers (lane i holds those of its reaction slots): one row of partial
// sums per group instead of one per cell.
extern "C" __global__ void __launch_bounds__(64) chem_adjoint(AdjointArgs a)
{
    using namespace chemw;
    extern __shared__ double lds[];
    const int grp = (int)threadIdx.x / G;
    const long gslot = (long)blockIdx.x * CPW + grp;
    if (gslot >= a.nslot) return;
    double* L = lds + grp * mech::ADJ_LDS_CELL;
    double* PV = L + 2 * mech::LDS_CELL;
    const int i = gl();
    double g[ROUNDS][3];
#pragma unroll
    for (int r = 0; r < ROUNDS; ++r) g[r][0] = g[r][1] = g[r][2] = 0.0;
    for (long slot = gslot; slot < a.ncell; slot += a.nslot) {
        const long cell = a.order[slot];
        Cell c;
        cell_begin(c, a.T0[cell], a.p[cell], a.Y0 + cell * NS, a.h0 ? a.h0[cell] : a.step.dt);
        double* hs = a.hs + a.off_h[cell];
        double* ck = a.ck + a.off_ck[cell] * N;
        const int cap = a.nacc_fwd[cell];
        int stored = -1;
        while (!c.done) {
            if (c.nacc % a.K == 0 && c.nacc != stored && c.nacc < cap) {
                if (i < N) ck[(c.nacc / a.K) * N + i] = c.y;
                stored = c.nacc;
            }
            const double hacc = cell_attempt(c, a.par, a.step, L, PV);
            if (hacc > 0.0) {
                if (c.nacc > cap) {
                    c.status = chem::CELL_NONFINITE;
                    c.done = true;
                    break;
                }
                if (i == 0) hs[c.nacc - 1] = hacc;
            }
        }
        cell_store(c, a.Tend, a.Yend, cell, a.status, a.nacc, a.nrej);
        if (c.status == chem::CELL_BADINPUT) {
            if (i == 0) a.Tend[cell] = a.T0[cell];
            else if (i <= NS) a.Yend[cell * NS + i - 1] = a.Y0[cell * NS + i - 1];
        }
        if (c.status != chem::CELL_OK) {
            if (i == 0) a.gT0[cell] = __builtin_nan("");
            else if (i <= NS) a.gY0[cell * NS + i - 1] = __builtin_nan("");
            continue;                   // adds nothing to the parameter gradients
        }
        double lam = i == 0 ? a.gT[cell] : (i <= NS ? a.gY[cell * NS + i - 1] : 0.0);
        const int na = c.nacc;
        const double p = c.p, ip = c.ip;
        for (int seg = (na - 1) / a.K; seg >= 0 && na > 0; --seg) {
            const int first = seg * a.K;
            const int last = min(na, first + a.K) - 1;
            double ys[16];                        // the segment's states (K <= 16), component i
            ys[0] = i < N ? ck[seg * N + i] : 0.0;
            for (int s = first; s < last; ++s) {
                double yn, en;
                double yc = ys[0];
#pragma unroll
                for (int q = 1; q < 16; ++q) yc = (q == s - first) ? ys[q] : yc;
                ros_step(a.par, p, ip, yc, hs[s], a.step.rtol, a.step.atol, L, PV, yn, en);
#pragma unroll
                for (int q = 1; q < 16; ++q) ys[q] = (q == s - first + 1) ? yn : ys[q];
            }
            for (int s = last; s >= first; --s) {
                double yc = ys[0];
#pragma unroll
                for (int q = 1; q < 16; ++q) yc = (q == s - first) ? ys[q] : yc;
                step_adjoint(a.par, p, ip, yc, hs[s], lam, g, L, PV);
            }
        }
        if (i == 0) a.gT0[cell] = lam;
        else if (i <= NS) a.gY0[cell * NS + i - 1] = lam;
    }
    double* gp = a.gpar + gslot * 3 * NR;
#pragma unroll
    for (int r = 0; r < ROUNDS; ++r) {
        const int j = r * G + i;
        if (j < NR) {
            const int oj = mech::RX_ORIG[j];
            gp[oj] = g[r][0];
            gp[NR + oj] = g[r][1];
            gp[2 * NR + oj] = g[r][2];
        }
    }
}
