// driver.cpp -- runs the library's per-lane device code (generated mechanism
// code + integrator, compiled for the host through shim.h) one cell at a
// time, exactly as the kernels do on one lane: the plain integration kernel,
// the fixed-step kernel, the source/Jacobian kernel and the discrete adjoint
// (sizing pass, arena offsets, checkpointed adjoint kernel, parameter sums in
// cell order).  Built with the host sanitizers by tests/test_hostemu.py.
//
// usage: driver IN OUT.  IN: int32 mode (0 integrate, 1 fixed step, 2 source
// terms + Jacobian, 3 adjoint), int32 ncell, int32 ns, int32 nr, then
// doubles: dt (or h), rtol, atol, par[3 nr] (ln A, b, Ea/R), T[ncell],
// p[ncell], Y[ncell ns], and for mode 3 gT[ncell], gY[ncell ns].
#include "shim.h"
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

emu_dim3 threadIdx, blockIdx, blockDim, gridDim;
double* emu_lds;

#include EMU_SOURCE

static void die(const char* m) { fprintf(stderr, "driver: %s\n", m); exit(2); }

template <class T> static T* rd(FILE* f, size_t n)
{
    T* p = (T*)malloc(sizeof(T) * (n ? n : 1));
    if (!p || fread(p, sizeof(T), n, f) != n) die("short input");
    return p;
}

template <class T> static void wr(FILE* f, const T* p, size_t n)
{
    if (fwrite(p, sizeof(T), n, f) != n) die("write failed");
}

// one lane per workgroup; the LDS of one lane is what the library gives it:
// its LDS words (the stage vectors or the LU factor entries), or in the
// adjoint the 3 NR parameter accumulators if they are more (an exact heap
// block, so the address sanitizer sees any access beyond it)
static void launch_lanes(long n, void (*body)(), bool adjoint = false)
{
    const int words = adjoint && chem::kAdjParamsInLds && 3 * mech::NR > chem::kLaneWords ? 3 * mech::NR
                                                                                           : chem::kLaneWords;
    double* lds = (double*)malloc(sizeof(double) * words);
    emu_lds = lds;
    blockDim = {1, 1, 1};
    threadIdx = {0, 0, 0};
    gridDim = {(unsigned)n, 1, 1};
    for (long b = 0; b < n; ++b) {
        blockIdx = {(unsigned)b, 0, 0};
        body();
    }
    free(lds);
}

static chem::IntegrateArgs g_ia;
static EvalArgs g_ea;
static FixedStepArgs g_fa;
static AdjointArgs g_aa;

int main(int argc, char** argv)
{
    if (argc != 3) die("usage: driver IN OUT");
    FILE* in = fopen(argv[1], "rb");
    if (!in) die("cannot open input");
    const int32_t* hdr = rd<int32_t>(in, 4);
    const int mode = hdr[0], ns = hdr[2], nr = hdr[3];
    const long n = hdr[1];
    if (ns != mech::NS || nr != mech::NR) die("mechanism size mismatch");
    const int N = ns + 1;
    const double* sc = rd<double>(in, 3);
    double* par = rd<double>(in, 3 * (size_t)nr);
    double* T = rd<double>(in, n);
    double* p = rd<double>(in, n);
    double* Y = rd<double>(in, n * ns);
    FILE* out = fopen(argv[2], "wb");
    if (!out) die("cannot open output");
    const chem::StepArgs step{sc[0], sc[1], sc[2], 1e-20 * sc[0], 100000};
    if (mode == 0) {
        int* st = (int*)calloc(3 * n + 1, sizeof(int));
        g_ia = chem::IntegrateArgs{par, T, p, Y, n, nullptr, st, st + n, st + 2 * n, step};
        launch_lanes(n, [] { chem_plain(g_ia); });
        wr(out, T, n);
        wr(out, Y, n * ns);
        wr(out, st, 3 * n);
    } else if (mode == 1) {
        double* yn = (double*)calloc(n * N + 1, sizeof(double));
        double* en = (double*)calloc(n + 1, sizeof(double));
        int* ok = (int*)calloc(n + 1, sizeof(int));
        g_fa = FixedStepArgs{par, T, p, Y, n, sc[0], yn, en, sc[1], sc[2], ok};
        launch_lanes(n, [] { chem_fixed_step(g_fa); });
        wr(out, yn, n * N);
        wr(out, en, n);
        wr(out, ok, n);
    } else if (mode == 2) {
        double* f = (double*)calloc(n * N + 1, sizeof(double));
        double* J = (double*)calloc(n * N * N + 1, sizeof(double));
        g_ea = EvalArgs{par, T, p, Y, n, f, J};
        launch_lanes(n, [] { chem_eval(g_ea); });
        wr(out, f, n * N);
        wr(out, J, n * N * N);
    } else if (mode == 3) {
        double* gT = rd<double>(in, n);
        double* gY = rd<double>(in, n * ns);
        // checkpoint interval: 4, or EMU_ADJ_K (1 runs the trail path)
        const int K = getenv("EMU_ADJ_K") ? atoi(getenv("EMU_ADJ_K")) : 4;
        // sizing pass: the plain kernel on copies gives every cell's accepted steps
        double* Tw = (double*)malloc(sizeof(double) * n);
        double* Yw = (double*)malloc(sizeof(double) * n * ns);
        memcpy(Tw, T, sizeof(double) * n);
        memcpy(Yw, Y, sizeof(double) * n * ns);
        int* i32 = (int*)calloc(6 * n + 1, sizeof(int));
        int *st = i32, *na_fwd = i32 + n, *na = i32 + 2 * n, *nj = i32 + 3 * n, *order = i32 + 4 * n;
        g_ia = chem::IntegrateArgs{par, Tw, p, Yw, n, nullptr, st, na_fwd, nj, step};
        launch_lanes(n, [] { chem_plain(g_ia); });
        long* off = (long*)malloc(sizeof(long) * 2 * n + 1);
        long th = 0, tc = 0;
        for (long c = 0; c < n; ++c) {
            off[c] = th;
            off[n + c] = tc;
            const long k = na_fwd[c] > 0 ? na_fwd[c] : 0;
            th += k;
            tc += (k + K - 1) / K;
            order[c] = (int)c;
        }
        double* hs = (double*)calloc(th + 1, sizeof(double));
        double* ck = (double*)calloc(tc * N + 1, sizeof(double));
        // fewer lanes than cells, so each lane takes several cells in turn and
        // keeps one row of partial parameter sums, as on the GPU for large fields
        const long nslot = (n + 2) / 3;
        double* gpar = (double*)calloc(nslot * 3 * nr + 1, sizeof(double));
        double* gT0 = (double*)calloc(n + 1, sizeof(double));
        double* gY0 = (double*)calloc(n * ns + 1, sizeof(double));
        double* Te = (double*)calloc(n + 1, sizeof(double));
        double* Ye = (double*)calloc(n * ns + 1, sizeof(double));
        // the K-step stash of every lane (K > 1) or the trail of every step
        // (K = 1), as the library gives the lane form
        double* stash = K > 1 ? (double*)calloc((size_t)nslot * K * chem::StashLayout::WORDS, sizeof(double)) : nullptr;
        double* trail = K == 1 ? (double*)calloc((size_t)(th + n) * chem::StashLayout::WORDS, sizeof(double)) : nullptr;
        g_aa = AdjointArgs{par, T, p, Y, n, gT, gY, gT0, gY0, gpar, nslot, Te, Ye, off, off + n, na_fwd, order,
                           nullptr, hs, ck, st, na, nj, step, K, 0, 0, stash, trail};
        launch_lanes(nslot, [] { chem_adjoint(g_aa); }, true);
        double* gp = (double*)calloc(3 * nr, sizeof(double));
        for (long c = 0; c < nslot; ++c)
            for (int j = 0; j < 3 * nr; ++j) gp[j] += gpar[c * 3 * nr + j];
        wr(out, gT0, n);
        wr(out, gY0, n * ns);
        wr(out, gp, 3 * nr);
        wr(out, Te, n);
        wr(out, Ye, n * ns);
        wr(out, st, n);
    } else {
        die("unknown mode");
    }
    fclose(out);
    return 0;
}
