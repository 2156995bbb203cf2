// common.hip -- device declarations shared by the per-lane and the
// wave-cooperative integrators: the RODAS4 tableau, cell status codes, kernel
// argument structs, the field table of the persistent launches, and the
// counter kernels.

namespace chem {

// ---- RODAS4 in the transformed variables u_i ----
struct Rodas4 {
    static constexpr int S = 6;
    static constexpr double gamma = 0.25;
};
__device__ constexpr double RA[6][5] = {
    {0, 0, 0, 0, 0},
    {1.544, 0, 0, 0, 0},
    {0.9466785280815826, 0.2557011698983284, 0, 0, 0},
    {3.314825187068521, 2.896124015972201, 0.9986419139977817, 0, 0},
    {1.221224509226641, 6.019134481288629, 12.53708332932087, -0.687886036105895, 0},
    {1.221224509226641, 6.019134481288629, 12.53708332932087, -0.687886036105895, 1.0}};
__device__ constexpr double RC[6][5] = {
    {0, 0, 0, 0, 0},
    {-5.6688, 0, 0, 0, 0},
    {-2.430093356833875, -0.2063599157091915, 0, 0, 0},
    {-0.1073529058151375, -9.594562251023355, -20.47028614809616, 0, 0},
    {7.496443313967647, -10.24680431464352, -33.99990352819905, 11.7089089320616, 0},
    {8.083246795921522, -7.981132988064893, -31.52159432874371, 16.31930543123136,
     -6.058818238834054}};
// y_new = y + sum_i m_i u_i with m = (a_51, a_52, a_53, a_54, 1, 1): the stage-6
// argument plus u_6 (stiffly accurate); the error estimate is u_6.

enum : int { CELL_OK = 0, CELL_MAXSTEPS = 1, CELL_HMIN = 2, CELL_NONFINITE = 3, CELL_BADINPUT = 4 };

struct StepArgs {
    double dt, rtol, atol, hmin;
    int max_substeps;
};

__device__ __forceinline__ bool finite(double x) { return __builtin_isfinite(x); }

// x^(-1/4) for the step-size controller, as the reciprocal of two square roots
__device__ __forceinline__ double inv_root4(double x) { return chem_math::recip(sqrt(sqrt(x))); }

struct IntegrateArgs {
    const double* par;
    double* T;
    const double* p;
    double* Y;
    long ncell;
    const double* h0;          // nullable: per-cell first step, else dt
    int* status;
    int* nacc;
    int* nrej;
    StepArgs step;
};

}  // namespace chem

// source terms and Jacobian at given states (no integration)
struct EvalArgs {
    const double* par;
    const double* T;
    const double* p;
    const double* Y;
    long ncell;
    double* f;      // [ncell][N]
    double* J;      // [ncell][N][N] or null
};

// ---- counters: sums of accepted / rejected substeps, failed cells, max attempts ----
extern "C" __global__ void __launch_bounds__(256) chem_zero_u64(unsigned long long* p, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

extern "C" __global__ void __launch_bounds__(256) chem_reduce_stats(const int* __restrict__ status,
                                                                    const int* __restrict__ nacc,
                                                                    const int* __restrict__ nrej,
                                                                    long ncell,
                                                                    unsigned long long* __restrict__ out)
{
    unsigned long long acc = 0, rej = 0, fail = 0, mx = 0;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < ncell; i += (long)gridDim.x * blockDim.x) {
        const int a = nacc[i], r = nrej[i];
        acc += (unsigned long long)a;
        rej += (unsigned long long)r;
        fail += status[i] != 0 ? 1ull : 0ull;
        const unsigned long long t = (unsigned long long)(a + r);
        mx = t > mx ? t : mx;
    }
    __shared__ unsigned long long s[4][256];
    s[0][threadIdx.x] = acc;
    s[1][threadIdx.x] = rej;
    s[2][threadIdx.x] = fail;
    s[3][threadIdx.x] = mx;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            s[0][threadIdx.x] += s[0][threadIdx.x + w];
            s[1][threadIdx.x] += s[1][threadIdx.x + w];
            s[2][threadIdx.x] += s[2][threadIdx.x + w];
            s[3][threadIdx.x] = s[3][threadIdx.x] > s[3][threadIdx.x + w] ? s[3][threadIdx.x] : s[3][threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        atomicAdd(&out[0], s[0][0]);
        atomicAdd(&out[1], s[1][0]);
        atomicAdd(&out[2], s[2][0]);
        atomicMax(&out[3], s[3][0]);
    }
}

// ---- field table of the persistent launches ----
constexpr int kCostBuckets = 256;

struct FieldDesc {
    double* T;
    const double* p;
    double* Y;
    int* status;
    int* nacc;
    int* nrej;
    const int* cost;          // nullable: per-cell cost hint
    long ncell;
    long start;               // first global index of this field
};

struct PersistBlock {
    long total;
    int nfield;
    int nq;
    int refill;
    int order;                // 1: cost-ordered
    chem::StepArgs step;
    unsigned char* bucket;    // [total] cost bucket per cell
    int* perm;                // [total] cells by descending cost
    unsigned* hist;           // [kCostBuckets]
    unsigned* cursor;         // [kCostBuckets]
    FieldDesc fields[1];      // nfield entries
};

__device__ __forceinline__ int field_of(const PersistBlock* __restrict__ blk, long g)
{
    int f = 0;
    while (f + 1 < blk->nfield && blk->fields[f + 1].start <= g) ++f;
    return f;
}

extern "C" __global__ void chem_reset_heads(const PersistBlock* __restrict__ blk, unsigned long long* heads)
{
    const int i = threadIdx.x;
    if (i < 64) heads[i] = 0ull;
    for (int b = i; b < kCostBuckets; b += blockDim.x) blk->hist[b] = 0u;
}

// ---- discrete adjoint: arguments (both forms) and the parameter-gradient reduction ----
struct AdjointArgs {
    const double* par;
    const double* T0;
    const double* p;
    const double* Y0;
    long ncell;
    const double* gT;
    const double* gY;
    double* gT0;
    double* gY0;
    double* gpar;          // [nslot][3 NR]: parameter gradients (ln A, b, Ea) summed over the
                           // cells of each lane (lane form) or lane group (wave-cooperative form)
    long nslot;            // lanes (groups) of the launch: slot s takes cells s, s + nslot, ...
    double* Tend;
    double* Yend;
    const long* off_h;     // first step size of each cell in hs
    const long* off_ck;    // first checkpoint of each cell (in states of N doubles)
    const int* nacc_fwd;   // accepted steps of the sizing pass
    const int* order;      // cells by descending accepted steps (slot g takes cell order[g])
    const double* h0;      // nullable: per-cell first step, else dt
    double* hs;
    double* ck;
    int* status;
    int* nacc;
    int* nrej;
    chem::StepArgs step;
    int K;                 // accepted steps per checkpoint
    // one cell per lane form: the first kAdjGroup * ngroup lanes form ngroup
    // groups of kAdjGroup lanes that take the order positions [0, gcells) (the
    // most expensive cells), group g the positions g, g + ngroup, ...; the
    // other lanes take the positions from gcells on, one cell per lane
    long ngroup;
    long gcells;
    // nullable: K steps' worth of per-lane stash (one cell per lane form), so
    // a segment's replay leaves each step's factors and stage vectors for its
    // adjoint instead of the adjoint forming them again
    double* stash;
    // nullable, K = 1 only: every accepted step's factors and stage vectors
    // from the forward rerun, slot off_h[cell] + cell + step (one spare slot
    // per cell for an attempt past its count)
    double* trail;
};

// lanes per group of the grouped adjoint (a power of two >= the RODAS4 stages)
constexpr int kAdjGroup = 8;

// Parameter gradients summed in a fixed order: one workgroup per parameter;
// thread t adds rows t, t + 256, ... in turn, then a fixed tree.  The rows are
// the partial sums of the adjoint kernel's lanes (groups), each over its cells
// in its own fixed order, so the result is bitwise reproducible.
extern "C" __global__ void __launch_bounds__(256) chem_reduce_params(const double* __restrict__ gpar, long ncell,
                                                                    int nparam, double* __restrict__ gA,
                                                                    double* __restrict__ gb, double* __restrict__ gE)
{
    __shared__ double s[256];
    const int q = blockIdx.x;
    double v = 0.0;
    for (long c = threadIdx.x; c < ncell; c += 256) v += gpar[c * nparam + q];
    s[threadIdx.x] = v;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const int nr = nparam / 3;
        if (q < nr) gA[q] = s[0];
        else if (q < 2 * nr) gb[q - nr] = s[0];
        else gE[q - 2 * nr] = s[0];
    }
}


// ---- operator-split source terms (the coupling to the flow equations) ----
// The flow solver's species and energy equations (Appendix A, eqs. (20)-(21))
// take the reaction terms of the split chemistry step as the mean rates over
// the step: wdot_k = rho0 (Y_k(dt) - Y_k(0)) / dt and qdot = -sum_k h_k(298.15 K)
// wdot_k, with rho0 the density of the initial state.  Around an integration:
// chem_source_begin keeps Y(0) in wdot and rho0 in qdot; chem_source_end turns
// them into the rates (NaN for a cell whose integration failed).
struct SourceArgs {
    const double* T;
    const double* p;
    const double* Y;
    long ncell;
    double dt;
    const int* status;
    double* wdot;   // [ncell][NS]
    double* qdot;   // [ncell]
};

extern "C" __global__ void __launch_bounds__(256) chem_source_begin(SourceArgs a)
{
    const long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= a.ncell) return;
    double sig = 0.0;
    for (int k = 0; k < mech::NS; ++k) {
        const double y = a.Y[c * mech::NS + k];
        sig = fma(y, mech::MWTAB[mech::NS + k], sig);
        a.wdot[c * mech::NS + k] = y;
    }
    a.qdot[c] = a.p[c] / (mech::RU * a.T[c] * sig);
}

extern "C" __global__ void __launch_bounds__(256) chem_source_end(SourceArgs a)
{
    const long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= a.ncell) return;
    const bool ok = a.status[c] == chem::CELL_OK;
    const double r = a.qdot[c] / a.dt;
    double q = 0.0;
    for (int k = 0; k < mech::NS; ++k) {
        const double w = r * (a.Y[c * mech::NS + k] - a.wdot[c * mech::NS + k]);
        a.wdot[c * mech::NS + k] = ok ? w : __builtin_nan("");
        q = fma(-mech::HF298[k], w, q);
    }
    a.qdot[c] = ok ? q : __builtin_nan("");
}
