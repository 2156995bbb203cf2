// integrator.hip -- device side of the chemistry step for CDNA4 (gfx950).
//
// Compiled at mechanism-load time together with the mechanism-specific code
// (namespace mech: sizes, thermo, source terms and analytic Jacobian with
// every species index a compile-time constant), so one cell's state, its
// Jacobian and LU factors live in the registers of one lane.
//
// Contents: dense LU with partial pivoting, the RODAS4 Rosenbrock step
// (Hairer & Wanner, Solving ODEs II, Sec. IV.7 / VI.4), the step-size
// controller, and the kernels (plain one-cell-per-lane, persistent
// work-stealing with lane refill, fixed-step and source-term evaluation).
//
// The per-cell problem is the species/energy source of the governing
// equations (Appendix A, eqs. (20)-(21)) at constant pressure over one flow
// step dt, cell by cell.

namespace chem {

constexpr int N = mech::N;
constexpr int NS = mech::NS;


// ---- dense LU with partial pivoting, one matrix per lane ----
// The step matrix is eliminated in the order mech::PERM: T and the species
// some reaction changes (positions 0 .. NACT-1) first, then the species no
// reaction changes, whose rows of M = I/(gamma h) - J hold the diagonal alone.
// Their entries in the first NACT columns are zero, so they never become
// pivots there and take no row updates; when their own columns come, only
// such rows remain below the diagonal.  Skipping them is exact: this is dense
// LU with partial pivoting of the symmetrically permuted matrix, with the
// structural zeros of those rows left out.  Row interchanges are made with
// selects (the pivot row differs per lane), on the trailing columns only, and
// skipped when no lane of the wave needs one; piv[a] records the position
// swapped into position a at step a (LINPACK order) and bit a of the returned
// wave-uniform mask says whether any lane swapped at step a.  The diagonal of
// U is stored as its reciprocal.
constexpr int NACT = mech::NACT;

__device__ __forceinline__ constexpr int P(int a) { return mech::PERM[a]; }

// ---- per-lane LDS ----
// A workgroup's dynamic LDS holds, for each of its waves, kLaneWords doubles
// per lane, lane-interleaved: word w of lane l at w * 64 + l.  The 64 lanes
// of a wave touch 64 consecutive doubles (no bank conflicts) and every word
// sits at a compile-time offset from the lane's base, whatever the workgroup
// size.  The words hold the RODAS4 stage vectors u_1..u_5 (u_s component k
// at word s N + k), or, when the step matrix's factors do not fit the lane's
// registers (kFactorsInLds), the first factor entries in the order the solves
// read them, the stage vectors then going to private memory.
constexpr int kLaneStride = 64;
// entries of the LU factors the solves read: L below the diagonal of the
// first NACT positions, and per position a its diagonal and min(a, NACT) of U
constexpr int kFactorEntries = NACT * (NACT - 1) / 2 + N + (NACT * (NACT - 1)) / 2 + (N - NACT) * NACT;
// From 12 unknowns the factors no longer fit beside the source-term temporaries
// and spill to private memory (measured at 14: 1.4 KB a lane), where every
// solve waits on them; below, they stay in accumulation registers, whose two
// moves per read cost less than an LDS load in the solve's chain (m9).
constexpr bool kFactorsInLds = N >= 12;
constexpr int kLdsBudget = 80;     // doubles a lane: 160 KB over four 64-lane waves
constexpr int kFactorsLds = kFactorsInLds ? (kFactorEntries < kLdsBudget ? kFactorEntries : kLdsBudget) : 0;
constexpr int kLaneWords = kFactorsInLds ? kFactorsLds : 5 * N;

__device__ __forceinline__ double* lane_lds(double* lds)
{
    return lds + (threadIdx.x / kLaneStride) * (kLaneStride * kLaneWords) + threadIdx.x % kLaneStride;
}

// slot[i][j]: the LDS word of factor entry (i, j), or -1 if it stays in registers
struct FactorSlots {
    int slot[N][N];
};

__host__ __device__ constexpr FactorSlots factor_slots(int count)
{
    FactorSlots m{};
    for (int i = 0; i < N; ++i)
        for (int j = 0; j < N; ++j) m.slot[i][j] = -1;
    int s = 0;
    for (int a = 0; a < NACT; ++a)                 // forward substitution: L by columns
        for (int c = a + 1; c < NACT; ++c) {
            if (s < count) m.slot[mech::PERM[c]][mech::PERM[a]] = s;
            ++s;
        }
    for (int a = N - 1; a >= 0; --a) {             // back substitution: U by columns
        const int k = mech::PERM[a];
        if (s < count) m.slot[k][k] = s;
        ++s;
        for (int c = 0; c < (a < NACT ? a : NACT); ++c) {
            if (s < count) m.slot[mech::PERM[c]][k] = s;
            ++s;
        }
    }
    return m;
}

__device__ constexpr FactorSlots kFactorSlots = factor_slots(kFactorsLds);

// factor entry (i, j): from the lane's LDS words if FL and it has a slot there
template <bool FL>
__device__ __forceinline__ double factor(const double (&A)[N][N], const double* __restrict__ fl, int i, int j)
{
    if constexpr (FL) {
        if (kFactorSlots.slot[i][j] >= 0) return fl[kFactorSlots.slot[i][j] * kLaneStride];
    }
    return A[i][j];
}

__device__ __forceinline__ unsigned lu_factor(double (&A)[N][N], int (&piv)[N], bool& ok)
{
    unsigned swaps = 0u;
    ok = true;
#pragma unroll
    for (int a = 0; a < NACT; ++a) {
        const int k = P(a);
        double amax = fabs(A[k][k]);
        int p = a;
#pragma unroll
        for (int b = a + 1; b < NACT; ++b) {
            const double v = fabs(A[P(b)][k]);
            const bool c = v > amax;
            amax = c ? v : amax;
            p = c ? b : p;
        }
        piv[a] = p;
        ok = ok && (amax > 0.0);
        if (__any(p != a)) {
            swaps |= 1u << a;
#pragma unroll
            for (int b = a + 1; b < NACT; ++b) {
                const bool s = (p == b);
                const int i = P(b);
#pragma unroll
                for (int c = a; c < N; ++c) {
                    const int j = P(c);
                    const double akj = A[k][j], aij = A[i][j];
                    A[k][j] = s ? aij : akj;
                    A[i][j] = s ? akj : aij;
                }
            }
        }
        const double rp = chem_math::recip(A[k][k]);
        A[k][k] = rp;
#pragma unroll
        for (int b = a + 1; b < NACT; ++b) {
            const int i = P(b);
            const double l = A[i][k] * rp;
            A[i][k] = l;
#pragma unroll
            for (int c = a + 1; c < N; ++c) {
                const int j = P(c);
                A[i][j] = fma(-l, A[k][j], A[i][j]);
            }
        }
    }
#pragma unroll
    for (int a = NACT; a < N; ++a) {     // rows with the diagonal alone
        const int k = P(a);
        piv[a] = a;
        ok = ok && (fabs(A[k][k]) > 0.0);
        A[k][k] = chem_math::recip(A[k][k]);
    }
    return swaps;
}

// The pivot index read inside the (rare) swap branch is opaque to the
// optimiser: otherwise the row compares of every step are hoisted out of the
// branch, shared by all solves of a Rosenbrock step and kept live in scalar
// registers, which spill.  Back substitution runs by columns, so each unknown
// is one multiply after the previous one rather than a chain of N - i FMAs.
__device__ __forceinline__ int opaque_index(int p)
{
    asm volatile("" : "+v"(p));
    return p;
}

// A wave-uniform value passed through an empty asm at each use, so that the
// tests of its bits are made where they are needed (scalar instructions)
// rather than once per step as lane masks that live across all six solves.
__device__ __forceinline__ unsigned opaque_uniform(unsigned x)
{
    asm volatile("" : "+s"(x));
    return x;
}

// FL: the factor entries with an LDS slot are read from the lane's words fl.
template <bool FL = false>
__device__ __forceinline__ void lu_solve(const double (&A)[N][N], const int (&piv)[N], unsigned swaps,
                                         double (&b)[N], const double* __restrict__ fl = nullptr)
{
#pragma unroll
    for (int a = 0; a < NACT; ++a) {
        const int k = P(a);
        if (swaps & (1u << a)) {
            const int p = opaque_index(piv[a]);
#pragma unroll
            for (int c = a + 1; c < NACT; ++c) {
                const bool s = (p == c);
                const int i = P(c);
                const double bk = b[k], bi = b[i];
                b[k] = s ? bi : bk;
                b[i] = s ? bk : bi;
            }
        }
#pragma unroll
        for (int c = a + 1; c < NACT; ++c) {
            const int i = P(c);
            b[i] = fma(-factor<FL>(A, fl, i, k), b[k], b[i]);
        }
    }
#pragma unroll
    for (int a = N - 1; a >= 0; --a) {
        const int k = P(a);
        b[k] *= factor<FL>(A, fl, k, k);
#pragma unroll
        for (int c = 0; c < (a < NACT ? a : NACT); ++c) {
            const int r = P(c);
            b[r] = fma(-factor<FL>(A, fl, r, k), b[k], b[r]);
        }
    }
}


// What one step leaves for its adjoint, per lane and step: the factors of M
// (N x N, as lu_factor leaves them), the pivot positions, the swap mask, and
// the stage vectors u_1..u_6.
struct StashLayout {
    static constexpr int WORDS = N * N + N + 1 + Rodas4::S * N;
    __device__ static constexpr int lu(int i, int j) { return i * N + j; }
    __device__ static constexpr int piv(int a) { return N * N + a; }
    __device__ static constexpr int swaps() { return N * N + N; }
    __device__ static constexpr int u(int s, int k) { return N * N + N + 1 + s * N + k; }
};

// One RODAS4 step from y with step h.  Returns false if the step matrix is
// singular or anything is not finite; otherwise ynew and the RMS error norm.
// The stage vectors u_1..u_5 live in the lane's LDS words ul (lane_lds); the
// matrix factors, y and the current stage stay in registers.
// With STASH the step also leaves what its adjoint needs in `stash` (see
// StashLayout; nothing if it is null): the factors of M, the pivots, the swap
// mask and u_1..u_6, bitwise the values the adjoint would recompute.
template <bool STASH>
__device__ __forceinline__ bool ros_step_impl(const double* __restrict__ par, double p, double ip,
                                              const double (&y)[N], double h, double rtol,
                                              double atol, double (&ynew)[N], double& errn,
                                              double* __restrict__ ul, double* __restrict__ stash)
{
    double M[N][N], f[N];
    mech::rhs_jac(par, p, ip, y, f, M);
    const double hinv = chem_math::recip(h);
    const double ghinv = hinv * (1.0 / Rodas4::gamma);
#pragma unroll
    for (int i = 0; i < N; ++i) {
#pragma unroll
        for (int j = 0; j < N; ++j) M[i][j] = -M[i][j];
        M[i][i] += ghinv;
    }
    int piv[N];
    bool ok;
    // the swap mask is the same in every active lane (lu_factor builds it from
    // __any), so it is read into a scalar register once
    const unsigned swaps = __builtin_amdgcn_readfirstlane(lu_factor(M, piv, ok));
    if constexpr (kFactorsInLds) {
#pragma unroll
        for (int i = 0; i < N; ++i)
#pragma unroll
            for (int j = 0; j < N; ++j)
                if (kFactorSlots.slot[i][j] >= 0) ul[kFactorSlots.slot[i][j] * kLaneStride] = M[i][j];
    }
    if constexpr (STASH) {
        if (stash) {
#pragma unroll
        for (int i = 0; i < N; ++i)
#pragma unroll
            for (int j = 0; j < N; ++j) stash[StashLayout::lu(i, j)] = M[i][j];
#pragma unroll
        for (int a = 0; a < N; ++a) stash[StashLayout::piv(a)] = (double)piv[a];
        stash[StashLayout::swaps()] = (double)swaps;
        }
    }

    // the stage vectors when the factors take the LDS words: private memory
    // (the indices pass through an empty asm so the array is not promoted to
    // registers, which the factors need)
    double us[kFactorsInLds ? Rodas4::S - 1 : 1][N];
    lu_solve<kFactorsInLds>(M, piv, opaque_uniform(swaps), f, ul);
#pragma unroll
    for (int k = 0; k < N; ++k) {
        if constexpr (kFactorsInLds) us[opaque_index(0)][k] = f[k];
        else ul[k * kLaneStride] = f[k];
    }
    if constexpr (STASH) {
        if (stash)
#pragma unroll
            for (int k = 0; k < N; ++k) stash[StashLayout::u(0, k)] = f[k];
    }
    double u[N];
#pragma unroll
    for (int s = 1; s < Rodas4::S; ++s) {
        double Ys[N], acc[N];
#pragma unroll
        for (int k = 0; k < N; ++k) {
            double v = y[k], w = 0.0;
#pragma unroll
            for (int j = 0; j < s; ++j) {
                double uj;
                if constexpr (kFactorsInLds) uj = us[opaque_index(j)][k];
                else uj = ul[(j * N + k) * kLaneStride];
                v = fma(RA[s][j], uj, v);
                w = fma(RC[s][j], uj, w);
            }
            Ys[k] = v;
            acc[k] = w;
        }
        if (s == Rodas4::S - 1) {
#pragma unroll
            for (int k = 0; k < N; ++k) ynew[k] = Ys[k];     // stiffly accurate: y_new = Y_6 + u_6
        }
        mech::rhs(par, p, ip, Ys, u);
#pragma unroll
        for (int k = 0; k < N; ++k) u[k] = fma(acc[k], hinv, u[k]);
        lu_solve<kFactorsInLds>(M, piv, opaque_uniform(swaps), u, ul);
        if (s < Rodas4::S - 1) {
#pragma unroll
            for (int k = 0; k < N; ++k) {
                if constexpr (kFactorsInLds) us[opaque_index(s)][k] = u[k];
                else ul[(s * N + k) * kLaneStride] = u[k];
            }
        }
        if constexpr (STASH) {
            if (stash)
#pragma unroll
                for (int k = 0; k < N; ++k) stash[StashLayout::u(s, k)] = u[k];
        }
    }
    double acc = 0.0;
#pragma unroll
    for (int k = 0; k < N; ++k) {
        ynew[k] += u[k];
        const double sc = atol + rtol * fmax(fabs(y[k]), fabs(ynew[k]));
        const double e = u[k] * chem_math::recip(sc);
        acc = fma(e, e, acc);
        ok = ok && finite(ynew[k]);
    }
    errn = sqrt(acc * (1.0 / N));
    return ok && finite(errn);
}

__device__ __forceinline__ bool ros_step(const double* __restrict__ par, double p, double ip,
                                         const double (&y)[N], double h, double rtol,
                                         double atol, double (&ynew)[N], double& errn,
                                         double* __restrict__ ul)
{
    return ros_step_impl<false>(par, p, ip, y, h, rtol, atol, ynew, errn, ul, nullptr);
}

// Per-lane integration state.
struct Cell {
    double y[N];
    double p, ip, t, h;
    int nacc, nrej, status;
    bool rej_last, done;
};

__device__ __forceinline__ void cell_begin(Cell& c, double T, double p, const double* __restrict__ Y,
                                           long stride, double h0)
{
    c.y[0] = T;
#pragma unroll
    for (int k = 0; k < NS; ++k) c.y[1 + k] = Y[k * stride];
    c.p = p;
    c.ip = 1.0 / p;
    c.t = 0.0;
    c.h = h0;
    c.nacc = 0;
    c.nrej = 0;
    c.rej_last = false;
    bool bad = !(T > 0.0) || !(p > 0.0) || !finite(p);
#pragma unroll
    for (int k = 0; k < N; ++k) bad = bad || !finite(c.y[k]);
    c.status = bad ? CELL_BADINPUT : CELL_OK;
    c.done = bad;
}

// One attempted substep (accepted or rejected), with the controller:
// accept if err <= 1; h <- h * clip(0.9 err^-1/4, 0.2, 6), no growth right after
// a rejection; a rejected or failed step shrinks h by max(0.2, 0.9 err^-1/4)
// or 0.2; the final step is truncated to land on dt.
// STASH: the attempt also leaves its step's factors and stage vectors in
// `stash` (nullable), see ros_step_impl.
template <bool STASH = false>
__device__ __forceinline__ double cell_attempt(Cell& c, const double* __restrict__ par, const StepArgs& a,
                                               double* __restrict__ ul, double* __restrict__ stash = nullptr)
{
    if (c.done) return 0.0;
    if (c.nacc + c.nrej >= a.max_substeps) { c.status = CELL_MAXSTEPS; c.done = true; return 0.0; }
    if (c.h < a.hmin) { c.status = CELL_HMIN; c.done = true; return 0.0; }
    bool last = false;
    double h = c.h;
    if (h >= a.dt - c.t) { h = a.dt - c.t; last = true; }
    double ynew[N], en;
    const bool ok = ros_step_impl<STASH>(par, c.p, c.ip, c.y, h, a.rtol, a.atol, ynew, en, ul, stash);
    if (ok && en <= 1.0) {
#pragma unroll
        for (int k = 0; k < N; ++k) c.y[k] = ynew[k];
        c.t = last ? a.dt : c.t + h;
        double fac = 0.9 * inv_root4(fmax(en, 1e-16));
        fac = fmin(6.0, fmax(0.2, fac));
        if (c.rej_last) fac = fmin(1.0, fac);
        c.h = h * fac;
        c.rej_last = false;
        ++c.nacc;
        if (last) c.done = true;
        return h;
    }
    ++c.nrej;
    c.h = h * (ok ? fmax(0.2, 0.9 * inv_root4(en)) : 0.2);
    c.rej_last = true;
    return 0.0;
}


__device__ __forceinline__ void cell_store(const Cell& c, double* __restrict__ T, double* __restrict__ Y,
                                           long cell, int* status, int* nacc, int* nrej)
{
    if (c.status != CELL_BADINPUT) {
        T[cell] = c.y[0];
#pragma unroll
        for (int k = 0; k < NS; ++k) Y[cell * NS + k] = c.y[1 + k];
    }
    // the per-cell counters only where someone reads them (null: not asked for)
    if (status) status[cell] = c.status;
    if (nacc) nacc[cell] = c.nacc;
    if (nrej) nrej[cell] = c.nrej;
}

}  // namespace chem

// ---- plain form: one cell per lane, cells in index order ----
extern "C" __global__ void __launch_bounds__(64, 1) chem_plain(chem::IntegrateArgs a)
{
    using namespace chem;
    const long cell = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (cell >= a.ncell) return;
    extern __shared__ double lds[];
    Cell c;
    cell_begin(c, a.T[cell], a.p[cell], a.Y + cell * NS, 1, a.h0 ? a.h0[cell] : a.step.dt);
    double* const ul = lane_lds(lds);
    while (!c.done) cell_attempt(c, a.par, a.step, ul);
    cell_store(c, a.T, a.Y, cell, a.status, a.nacc, a.nrej);
}


// ---- source terms and Jacobian at given states (no integration) ----
extern "C" __global__ void __launch_bounds__(64, 1) chem_eval(EvalArgs a)
{
    using namespace chem;
    const long cell = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (cell >= a.ncell) return;
    double y[N], f[N];
    y[0] = a.T[cell];
#pragma unroll
    for (int k = 0; k < NS; ++k) y[1 + k] = a.Y[cell * NS + k];
    const double p = a.p[cell];
    if (a.J) {
        double J[N][N];
        mech::rhs_jac(a.par, p, 1.0 / p, y, f, J);
#pragma unroll
        for (int i = 0; i < N; ++i)
#pragma unroll
            for (int j = 0; j < N; ++j) a.J[(cell * N + i) * N + j] = J[i][j];
    } else {
        mech::rhs(a.par, p, 1.0 / p, y, f);
    }
#pragma unroll
    for (int i = 0; i < N; ++i) a.f[cell * N + i] = f[i];
}

// ---- one fixed step of size h per cell (y_new and the error vector) ----
struct FixedStepArgs {
    const double* par;
    const double* T;
    const double* p;
    const double* Y;
    long ncell;
    double h;
    double* ynew;   // [ncell][N]
    double* err;    // [ncell] RMS norm with rtol = 1, atol = 0 ... see host
    double rtol, atol;
    int* ok;
};

extern "C" __global__ void __launch_bounds__(64, 1) chem_fixed_step(FixedStepArgs a)
{
    using namespace chem;
    const long cell = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (cell >= a.ncell) return;
    extern __shared__ double lds[];
    double y[N], yn[N], en;
    y[0] = a.T[cell];
#pragma unroll
    for (int k = 0; k < NS; ++k) y[1 + k] = a.Y[cell * NS + k];
    const double p = a.p[cell];
    const bool ok = ros_step(a.par, p, 1.0 / p, y, a.h, a.rtol, a.atol, yn, en, lane_lds(lds));
#pragma unroll
    for (int k = 0; k < N; ++k) a.ynew[cell * N + k] = yn[k];
    a.err[cell] = en;
    a.ok[cell] = ok ? 1 : 0;
}


// ---- persistent form ----
// Cells of all fields form one global index space [0, total).  Optionally the
// cells are first ordered by predicted cost, most expensive first (a counting
// sort over 256 cost buckets): the cost of a cell is either given by the
// caller (e.g. its substep count in the previous call, the measured load the
// paper balances on) or predicted from its state by one source-term
// evaluation: the mean over the components of log2(1 + |f_k| dt / (atol +
// rtol |y_k|)), i.e. by how many factors of two each component would move,
// in tolerance units, over dt.  A log-average weighs every component; an RMS
// is set by the fastest-changing trace species alone and ranks the costs of
// reacting cells far worse (rank correlation 0.38 against 0.69 on the RDE
// field's reacting cells).  Positions are dealt to
// nq queues (one per XCD) interleaved, so every queue sees the same cost mix.
// Each wave pulls cells from the queue of its XCD (workgroups are dealt to
// the XCDs round-robin), moves on to the next queue when its own is empty,
// and refills idle lanes at substep boundaries, so a lane never waits for the
// slowest cell of its wave.

extern "C" __global__ void __launch_bounds__(256) chem_order_key(const PersistBlock* __restrict__ blk,
                                                                const double* __restrict__ par)
{
    using namespace chem;
    __shared__ unsigned h[kCostBuckets];
    for (int b = threadIdx.x; b < kCostBuckets; b += blockDim.x) h[b] = 0u;
    __syncthreads();
    if (blk->order) {
        const StepArgs st = blk->step;
        for (long g = (long)blockIdx.x * blockDim.x + threadIdx.x; g < blk->total;
             g += (long)gridDim.x * blockDim.x) {
            const FieldDesc& fd = blk->fields[field_of(blk, g)];
            const long l = g - fd.start;
            double key;
            if (fd.cost) {
                key = 12.0 * log2(1.0 + (double)max(fd.cost[l], 0));
            } else {
                double y[N], f[N];
                y[0] = fd.T[l];
#pragma unroll
                for (int k = 0; k < NS; ++k) y[1 + k] = fd.Y[l * NS + k];
                const double p = fd.p[l];
                mech::rhs(par, p, 1.0 / p, y, f);
                double s = 0.0;
#pragma unroll
                for (int k = 0; k < N; ++k) s += log2(1.0 + fabs(f[k]) * st.dt / (st.atol + st.rtol * fabs(y[k])));
                key = 6.0 * s * (1.0 / N);
            }
            const int b = (key >= 0.0) ? (key < kCostBuckets - 1 ? (int)key : kCostBuckets - 1)
                                       : kCostBuckets - 1;    // NaN: schedule early
            blk->bucket[g] = (unsigned char)b;
            atomicAdd(&h[b], 1u);
        }
    }
    __syncthreads();
    for (int b = threadIdx.x; b < kCostBuckets; b += blockDim.x)
        if (h[b]) atomicAdd(&blk->hist[b], h[b]);
}

// start positions of the buckets, most expensive bucket first
extern "C" __global__ void __launch_bounds__(kCostBuckets) chem_order_scan(const PersistBlock* __restrict__ blk)
{
    __shared__ unsigned s[kCostBuckets];
    const int t = threadIdx.x;
    s[t] = blk->hist[kCostBuckets - 1 - t];
    __syncthreads();
    for (int off = 1; off < kCostBuckets; off <<= 1) {
        const unsigned v = t >= off ? s[t - off] : 0u;
        __syncthreads();
        s[t] += v;
        __syncthreads();
    }
    const int b = kCostBuckets - 1 - t;
    blk->cursor[b] = s[t] - blk->hist[b];         // exclusive
}

// Cells to their positions: within each chunk of blockDim cells, ranks come
// from LDS atomics and one global atomic per bucket reserves the chunk's
// share (the cheap cells of a field mostly share one bucket, so per-cell
// global atomics would serialise on it).
extern "C" __global__ void __launch_bounds__(256) chem_order_scatter(const PersistBlock* __restrict__ blk)
{
    if (!blk->order) return;
    __shared__ unsigned cnt[kCostBuckets], off[kCostBuckets];
    const long total = blk->total;
    for (long base = (long)blockIdx.x * blockDim.x; base < total; base += (long)gridDim.x * blockDim.x) {
        for (int b = threadIdx.x; b < kCostBuckets; b += blockDim.x) cnt[b] = 0u;
        __syncthreads();
        const long g = base + threadIdx.x;
        const int b = g < total ? (int)blk->bucket[g] : -1;
        const unsigned r = b >= 0 ? atomicAdd(&cnt[b], 1u) : 0u;
        __syncthreads();
        for (int k = threadIdx.x; k < kCostBuckets; k += blockDim.x)
            if (cnt[k]) off[k] = atomicAdd(&blk->cursor[k], cnt[k]);
        __syncthreads();
        if (b >= 0) blk->perm[off[b] + r] = (int)g;
        __syncthreads();
    }
}

__device__ __forceinline__ void persistent_body(const PersistBlock* __restrict__ blk,
                                                unsigned long long* __restrict__ heads,
                                                const double* __restrict__ par)
{
    using namespace chem;
    extern __shared__ double lds[];
    double* const ul = lane_lds(lds);
    const int lane = threadIdx.x & 63;
    const long total = blk->total;
    const int nq = blk->nq;
    const int refill = blk->refill;
    const bool ordered = blk->order != 0;
    const int* __restrict__ perm = blk->perm;
    const StepArgs step = blk->step;
    const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));

    int q = (int)(blockIdx.x % (unsigned)nq);     // home queue: this workgroup's XCD
    int tried = 0;
    bool exhausted = false;
    bool have = false;
    int fidx = 0;
    long local = 0;
    Cell c;
    c.done = true;

    while (true) {
        const unsigned long long idle = __ballot(!have);
        const int nidle = __popcll(idle);
        if (!exhausted && (nidle >= refill || nidle == 64)) {
            int need = nidle;
            int assigned = 0;
            const int rank = __popcll(idle & below);
            long my_g = -1;
            while (need > 0 && !exhausted) {
                const int leader = __ffsll((long long)idle) - 1;
                unsigned long long old = 0;
                if (lane == leader) old = atomicAdd(&heads[q], (unsigned long long)need);
                old = __shfl(old, leader);
                // queue q holds positions q, q + nq, q + 2 nq, ... below total
                const long qsize = (total - q + nq - 1) / nq;
                const long avail = qsize - (long)old;
                const int got = avail <= 0 ? 0 : (avail < (long)need ? (int)avail : need);
                if (!have && rank >= assigned && rank < assigned + got) {
                    const long pos = ((long)old + (rank - assigned)) * nq + q;
                    my_g = ordered ? (long)perm[pos] : pos;
                }
                assigned += got;
                if (got < need) {
                    q = (q + 1 == nq) ? 0 : q + 1;
                    if (++tried >= nq) exhausted = true;
                }
                need -= got;
            }
            if (my_g >= 0) {
                fidx = field_of(blk, my_g);
                const FieldDesc& fd = blk->fields[fidx];
                local = my_g - fd.start;
                cell_begin(c, fd.T[local], fd.p[local], fd.Y + local * NS, 1, step.dt);
                have = true;
            }
        }
        if (!__any(have)) {
            if (exhausted) break;
            continue;
        }
        if (have) {
            cell_attempt(c, par, step, ul);
            if (c.done) {
                const FieldDesc& fd = blk->fields[fidx];
                cell_store(c, fd.T, fd.Y, local, fd.status, fd.nacc, fd.nrej);
                have = false;
            }
        }
    }
}

extern "C" __global__ void __launch_bounds__(256, 1)
chem_persistent(const PersistBlock* __restrict__ blk, unsigned long long* __restrict__ heads,
                const double* __restrict__ par)
{
    persistent_body(blk, heads, par);
}

// gather every stride-th cell of the global index space into contiguous
// buffers (the autotuner's sample)
extern "C" __global__ void __launch_bounds__(256) chem_gather_sample(const PersistBlock* __restrict__ blk,
                                                                    long stride, long count,
                                                                    double* __restrict__ T,
                                                                    double* __restrict__ p,
                                                                    double* __restrict__ Y)
{
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const long g = i * stride;
    const FieldDesc& fd = blk->fields[field_of(blk, g)];
    const long l = g - fd.start;
    T[i] = fd.T[l];
    p[i] = fd.p[l];
    for (int k = 0; k < chem::NS; ++k) Y[i * chem::NS + k] = fd.Y[l * chem::NS + k];
}


// ---- discrete adjoint of the frozen-step map ----
// For one RODAS4 step y -> y_new with M = I/(gamma h) - J(y), M u_s = f(Y_s) +
// sum_{j<s} (c_sj/h) u_j, Y_s = y + sum_{j<s} a_sj u_j, y_new = y + sum m_s u_s,
// the cotangent lambda of y_new gives, with u-bar_s = m_s lambda and stages in
// reverse order,
//     w_s = M^-T u-bar_s,   Ybar_s = J(Y_s)^T w_s,
//     y-bar += Ybar_s,  u-bar_j += a_sj Ybar_s + (c_sj/h) w_s  (j < s),
//     theta-bar += f_theta(Y_s)^T w_s,
// and, through J(y) inside M, y-bar += sum_s D_{u_s}[J(y)^T w_s] and
// theta-bar += sum_s D_{u_s}[f_theta(y)^T w_s] (dual numbers along u_s).
// Those six second-order terms are independent of one another once every w_s
// is known, so a group of kAdjGroup lanes holding the same cell (all of them
// repeating the rest of the step) evaluates one direction per lane and sums
// the group's results; on the critical path of the most expensive cells that
// replaces six evaluations by one.
namespace chem {

__device__ __forceinline__ void lu_solve_t(const double (&A)[N][N], const int (&piv)[N], unsigned swaps,
                                           double (&b)[N])
{
    // U^T (only the first NACT rows of U have entries off the diagonal)
#pragma unroll
    for (int a = 0; a < N; ++a) {
        const int i = P(a);
        double v = b[i];
#pragma unroll
        for (int c = 0; c < (a < NACT ? a : NACT); ++c) {
            const int j = P(c);
            v = fma(-A[j][i], b[j], v);
        }
        b[i] = v * A[i][i];
    }
    // L^T and the interchanges in reverse (L has entries below the diagonal in
    // the first NACT rows and columns only)
#pragma unroll
    for (int a = NACT - 1; a >= 0; --a) {
        const int k = P(a);
        double v = b[k];
#pragma unroll
        for (int c = a + 1; c < NACT; ++c) {
            const int i = P(c);
            v = fma(-A[i][k], b[i], v);
        }
        b[k] = v;
        if (swaps & (1u << a)) {
            const int p = opaque_index(piv[a]);
#pragma unroll
            for (int c = a + 1; c < NACT; ++c) {
                const bool s = (p == c);
                const int i = P(c);
                const double bk = b[k], bi = b[i];
                b[k] = s ? bi : bk;
                b[i] = s ? bk : bi;
            }
        }
    }
}

// jd: -1 for a lane of its own (all six directions), else this lane's place
// in its group (direction jd; lanes 6 and 7 evaluate a zero direction); only
// lanes with jd <= 0 add the first-order parameter products.
// FROM_STASH: the factors, pivots and stage vectors of the step come from
// what ros_step_impl<true> left for it (the same values, bitwise), and only
// the stage states are formed again from them.
// gA, gb, gE: the lane's parameter-gradient accumulators (private memory).
// While the step runs they are held in the lane's LDS words instead, when the
// 3 NR of them fit (kAdjParamsInLds): the step's dozen Jacobian-transpose
// products each add to all of them, and a read-modify-write of private memory
// waits on the cache hierarchy while one of LDS does not; the caller launches
// the adjoint with that much LDS per lane (max(5 N, 3 NR) words), and the
// stage-vector words are free during a step adjoint.
constexpr bool kAdjParamsInLds = 3 * mech::NR <= 80;
constexpr int kAdjParamStride = kAdjParamsInLds ? kLaneStride : 1;

template <bool FROM_STASH>
__device__ __noinline__ void step_adjoint(const double* __restrict__ par, double p, double ip,
                                          const double (&y)[N], double h, double (&lam)[N],
                                          double* __restrict__ gA, double* __restrict__ gb,
                                          double* __restrict__ gE, int jd, const double* __restrict__ stash)
{
    using chem_math::Dual;
    double M[N][N];
    int piv[N];
    unsigned swaps;
    const double hinv = chem_math::recip(h);
    double u[Rodas4::S][N], Ys[Rodas4::S][N];
    if constexpr (FROM_STASH) {
        for (int i = 0; i < N; ++i)
            for (int j = 0; j < N; ++j) M[i][j] = stash[StashLayout::lu(i, j)];
        for (int a = 0; a < N; ++a) piv[a] = (int)stash[StashLayout::piv(a)];
        swaps = (unsigned)stash[StashLayout::swaps()];
        for (int s = 0; s < Rodas4::S; ++s)
            for (int k = 0; k < N; ++k) u[s][k] = stash[StashLayout::u(s, k)];
        for (int k = 0; k < N; ++k) Ys[0][k] = y[k];
        for (int s = 1; s < Rodas4::S; ++s)
            for (int k = 0; k < N; ++k) {
                double v = y[k];
                for (int j = 0; j < s; ++j) v = fma(RA[s][j], u[j][k], v);
                Ys[s][k] = v;
            }
    } else {
        double f[N];
        mech::rhs_jac(par, p, ip, y, f, M);
        const double ghinv = hinv * (1.0 / Rodas4::gamma);
        for (int i = 0; i < N; ++i) {
            for (int j = 0; j < N; ++j) M[i][j] = -M[i][j];
            M[i][i] += ghinv;
        }
        bool ok;
        swaps = lu_factor(M, piv, ok);
        for (int k = 0; k < N; ++k) { Ys[0][k] = y[k]; u[0][k] = f[k]; }
        lu_solve(M, piv, swaps, u[0]);
        for (int s = 1; s < Rodas4::S; ++s) {
            double acc[N], fs[N];
            for (int k = 0; k < N; ++k) {
                double v = y[k], w = 0.0;
                for (int j = 0; j < s; ++j) {
                    v = fma(RA[s][j], u[j][k], v);
                    w = fma(RC[s][j], u[j][k], w);
                }
                Ys[s][k] = v;
                acc[k] = w;
            }
            mech::rhs(par, p, ip, Ys[s], fs);
            for (int k = 0; k < N; ++k) u[s][k] = fma(acc[k], hinv, fs[k]);
            lu_solve(M, piv, swaps, u[s]);
        }
    }
    double *qA = gA, *qb = gb, *qE = gE;
    if constexpr (kAdjParamsInLds) {
        extern __shared__ double lds[];
        double* const gl = lane_lds(lds);
        qA = gl;
        qb = gl + mech::NR * kAdjParamStride;
        qE = gl + 2 * mech::NR * kAdjParamStride;
        for (int j = 0; j < mech::NR; ++j) {
            qA[j * kAdjParamStride] = gA[j];
            qb[j * kAdjParamStride] = gb[j];
            qE[j * kAdjParamStride] = gE[j];
        }
    }
    // reverse over the stages: Ybar_s = J(Y_s)^T w_s and the parameter products
    // in one pass of the generated Jacobian-transpose product
    const double mw[Rodas4::S] = {RA[5][0], RA[5][1], RA[5][2], RA[5][3], 1.0, 1.0};
    double ub[Rodas4::S][N], w[Rodas4::S][N], yb[N];
    for (int k = 0; k < N; ++k) {
        yb[k] = lam[k];
        for (int s = 0; s < Rodas4::S; ++s) ub[s][k] = mw[s] * lam[k];
    }
    const double gsc = jd <= 0 ? 1.0 : 0.0;
    for (int s = Rodas4::S - 1; s >= 0; --s) {
        for (int k = 0; k < N; ++k) w[s][k] = ub[s][k];
        lu_solve_t(M, piv, swaps, w[s]);
        double Yb[N];
        mech::jtv_param<double, kAdjParamStride>(par, p, ip, Ys[s], w[s], Yb, qA, qb, qE, gsc);
        for (int k = 0; k < N; ++k) yb[k] += Yb[k];
        for (int j = 0; j < s; ++j)
            for (int k = 0; k < N; ++k) ub[j][k] = fma(RA[s][j], Yb[k], fma(RC[s][j] * hinv, w[s][k], ub[j][k]));
    }
    // second-order terms at y (J(y) inside M): D_{u_s}[J(y)^T w_s] and the
    // parameter products' derivative, one dual evaluation per stage direction
    // (the parameter products add only their tangent, see param_acc), all six
    // on a lane of its own, direction jd on a lane of a group
    double sec[N];
    for (int k = 0; k < N; ++k) sec[k] = 0.0;
    const int nd = jd < 0 ? Rodas4::S : 1;
    for (int t = 0; t < nd; ++t) {
        Dual yd[N], vd[N];
        double wd[N];
        if (jd < 0) {
            for (int k = 0; k < N; ++k) { yd[k] = Dual(y[k], u[t][k]); wd[k] = w[t][k]; }
        } else {
            for (int k = 0; k < N; ++k) {
                double ud = 0.0, ws = 0.0;
#pragma unroll
                for (int s = 0; s < Rodas4::S; ++s) {
                    ud = jd == s ? u[s][k] : ud;
                    ws = jd == s ? w[s][k] : ws;
                }
                yd[k] = Dual(y[k], ud);
                wd[k] = ws;
            }
        }
        mech::jtv_param<Dual, kAdjParamStride>(par, p, ip, yd, wd, vd, qA, qb, qE, 1.0);
        for (int k = 0; k < N; ++k) sec[k] += vd[k].d;
    }
    if (jd >= 0) {
        // butterfly over the group: every lane adds the same pairs, so all
        // lanes of the group hold the same sums, bit for bit
#pragma unroll
        for (int m = 1; m < kAdjGroup; m <<= 1)
            for (int k = 0; k < N; ++k) sec[k] += __shfl_xor(sec[k], m, kAdjGroup);
    }
    for (int k = 0; k < N; ++k) lam[k] = yb[k] + sec[k];
    if constexpr (kAdjParamsInLds) {
        for (int j = 0; j < mech::NR; ++j) {
            gA[j] = qA[j * kAdjParamStride];
            gb[j] = qb[j * kAdjParamStride];
            gE[j] = qE[j * kAdjParamStride];
        }
    }
}

}  // namespace chem



// The cells in cost order (descending accepted steps): the first a.gcells go
// to the a.ngroup lane groups (group g: positions g, g + ngroup, ...), whose
// lanes all run the cell and split the second-order terms of each step (see
// step_adjoint); the others to the remaining lanes, lane s taking the
// positions gcells + s, gcells + s + nlane, ...  The lanes of a wave thus work
// on cells of similar cost, and each keeps the parameter gradients of all its
// cells in registers: one row of partial sums per lane instead of one per
// cell.  Within a group only the first lane writes the cell's results.
extern "C" __global__ void __launch_bounds__(64, 1) chem_adjoint(AdjointArgs a)
{
    using namespace chem;
    const long lane = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (lane >= a.nslot) return;
    extern __shared__ double lds[];
    double* const ul = lane_lds(lds);
    double gA[mech::NR], gb[mech::NR], gE[mech::NR];
    for (int j = 0; j < mech::NR; ++j) { gA[j] = 0.0; gb[j] = 0.0; gE[j] = 0.0; }
    const long glanes = (long)kAdjGroup * a.ngroup;
    int jd;
    long pos0, pstride, pend;
    if (lane < glanes) {
        jd = (int)(lane % kAdjGroup);
        pos0 = lane / kAdjGroup;
        pstride = a.ngroup;
        pend = a.gcells;
    } else {
        jd = -1;
        pos0 = a.gcells + (lane - glanes);
        pstride = a.nslot - glanes;
        pend = a.ncell;
    }
    if (pstride <= 0) pend = pos0;      // no lanes of this kind (the host never launches so)
    const bool lead = jd <= 0;
    for (long slot = pos0; slot < pend; slot += pstride) {
        const long cell = a.order[slot];
        Cell c;
        cell_begin(c, a.T0[cell], a.p[cell], a.Y0 + cell * NS, 1, a.h0 ? a.h0[cell] : a.step.dt);
        double* hs = a.hs + a.off_h[cell];
        double* ck = a.ck + a.off_ck[cell] * N;
        const int cap = a.nacc_fwd[cell];
        int stored = -1;
        while (!c.done) {
            if (c.nacc % a.K == 0 && c.nacc != stored && c.nacc < cap) {
                if (lead)
                    for (int k = 0; k < N; ++k) ck[(c.nacc / a.K) * N + k] = c.y[k];
                stored = c.nacc;
            }
            // with a trail, the attempt leaves its factors and stage vectors
            // in the slot of the step it would be (the lanes of a group write
            // the same values to the same words and each reads back its own)
            double* slot = a.trail && c.nacc <= cap
                               ? a.trail + (a.off_h[cell] + cell + c.nacc) * (long)StashLayout::WORDS
                               : nullptr;
            const double hacc = cell_attempt<true>(c, a.par, a.step, ul, slot);
            if (hacc > 0.0) {
                if (c.nacc > cap) { c.status = CELL_NONFINITE; c.done = true; break; }
                if (lead) hs[c.nacc - 1] = hacc;
            }
        }
        if (lead) {
            cell_store(c, a.Tend, a.Yend, cell, a.status, a.nacc, a.nrej);
            if (c.status == CELL_BADINPUT) {
                a.Tend[cell] = a.T0[cell];
                for (int k = 0; k < NS; ++k) a.Yend[cell * NS + k] = a.Y0[cell * NS + k];
            }
        }
        if (c.status != CELL_OK) {
            if (lead) {
                a.gT0[cell] = __builtin_nan("");
                for (int k = 0; k < NS; ++k) a.gY0[cell * NS + k] = __builtin_nan("");
            }
            continue;                   // adds nothing to the parameter gradients
        }
        double lam[N];
        lam[0] = a.gT[cell];
        for (int k = 0; k < NS; ++k) lam[1 + k] = a.gY[cell * NS + k];
        const int na = c.nacc;
        const double p = c.p, ip = c.ip;
        for (int seg = (na - 1) / a.K; seg >= 0 && na > 0; --seg) {
            const int first = seg * a.K;
            const int last = min(na, first + a.K) - 1;
            double ys[16][N];                     // the segment's states (K <= 16)
            for (int k = 0; k < N; ++k) ys[0][k] = ck[seg * N + k];
            if (a.trail) {
                // checkpoints at every step (K = 1): the forward rerun left each
                // step's factors and stage vectors in the trail
                step_adjoint<true>(a.par, p, ip, ys[0], hs[first], lam, gA, gb, gE, jd,
                                   a.trail + (a.off_h[cell] + cell + first) * (long)StashLayout::WORDS);
            } else if (a.stash) {
                // replay every step of the segment, leaving each step's factors
                // and stage vectors for its adjoint in this lane's stash
                double* st = a.stash + lane * (long)a.K * StashLayout::WORDS;
                for (int i = first; i <= last; ++i) {
                    double yn[N], en;
                    ros_step_impl<true>(a.par, p, ip, ys[i - first], hs[i], a.step.rtol, a.step.atol, yn, en, ul,
                                        st + (i - first) * StashLayout::WORDS);
                    if (i < last)
                        for (int k = 0; k < N; ++k) ys[i - first + 1][k] = yn[k];
                }
                for (int i = last; i >= first; --i)
                    step_adjoint<true>(a.par, p, ip, ys[i - first], hs[i], lam, gA, gb, gE, jd,
                                       st + (i - first) * StashLayout::WORDS);
            } else {
                for (int i = first; i < last; ++i) {
                    double yn[N], en;
                    ros_step(a.par, p, ip, ys[i - first], hs[i], a.step.rtol, a.step.atol, yn, en, ul);
                    for (int k = 0; k < N; ++k) ys[i - first + 1][k] = yn[k];
                }
                for (int i = last; i >= first; --i)
                    step_adjoint<false>(a.par, p, ip, ys[i - first], hs[i], lam, gA, gb, gE, jd, nullptr);
            }
        }
        if (lead) {
            a.gT0[cell] = lam[0];
            for (int k = 0; k < NS; ++k) a.gY0[cell * NS + k] = lam[1 + k];
        }
    }
    double* g = a.gpar + lane * 3 * mech::NR;
    for (int j = 0; j < mech::NR; ++j) {
        g[j] = gA[j];
        g[mech::NR + j] = gb[j];
        g[2 * mech::NR + j] = gE[j];
    }
}
