// runtime.hpp -- per-device state of a mechanism and the launch paths.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/chem.h"
#include "codegen.hpp"
#include "mechanism.hpp"

namespace chemmi {

// Host mirrors of the kernel argument structs (same field order and types as
// in device/integrator.hip).
struct StepArgs {
    double dt, rtol, atol, hmin;
    int max_substeps;
};

struct IntegrateArgs {
    const double* par;
    double* T;
    const double* p;
    double* Y;
    long ncell;
    const double* h0;
    int* status;
    int* nacc;
    int* nrej;
    StepArgs step;
};

struct EvalArgs {
    const double* par;
    const double* T;
    const double* p;
    const double* Y;
    long ncell;
    double* f;
    double* J;
};

struct FixedStepArgs {
    const double* par;
    const double* T;
    const double* p;
    const double* Y;
    long ncell;
    double h;
    double* ynew;
    double* err;
    double rtol, atol;
    int* ok;
};

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
    double* gpar;      // [nslot][3 nr] partial sums of the parameter gradients
    long nslot;        // lanes (groups) of the adjoint launch
    double* Tend;
    double* Yend;
    const long* off_h;
    const long* off_ck;
    const int* nacc_fwd;
    const int* order;
    const double* h0;
    double* hs;
    double* ck;
    int* status;
    int* nacc;
    int* nrej;
    StepArgs step;
    int K;
    long ngroup;       // lane groups of the one-cell-per-lane adjoint (see kAdjGroup)
    long gcells;       // cells (first positions of the cost order) the groups take
    double* stash;     // nullable: [nslot][K][stash words] (see StashLayout)
    double* trail;     // nullable, K = 1: [accepted steps + ncell][stash words]
};

// lanes per group of the grouped one-cell-per-lane adjoint (device: kAdjGroup)
constexpr int kAdjGroupLanes = 8;

struct FieldDesc {
    double* T;
    const double* p;
    double* Y;
    int* status;
    int* nacc;
    int* nrej;
    const int* cost;
    long ncell;
    long start;
};

constexpr int kCostBuckets = 256;

struct PersistHeader {
    long total;
    int nfield;
    int nq;
    int refill;
    int order;
    StepArgs step;
    unsigned char* bucket;
    int* perm;
    unsigned* hist;
    unsigned* cursor;
};

// Scratch of the allocation-free entry point (noalloc.hip), per device:
// queue heads (64 u64), cost histogram and cursors (2 x 256 u32), the field
// table (header + one field), then per cell the status and substep counters
// (3 int32, used when the caller passes none), the cost permutation (int32)
// and the cost bucket (uint8), for up to kNoallocMaxCells cells.
constexpr size_t kNoallocMaxCells = CHEM_NOALLOC_MAX_CELLS;
constexpr int kNoallocMaxDevices = 64;
constexpr size_t kNoallocHeadsOff = 0;
constexpr size_t kNoallocHistOff = 512;
constexpr size_t kNoallocBlockOff = 2560;
constexpr size_t kNoallocCountersOff = 4096;
constexpr size_t kNoallocPermOff = kNoallocCountersOff + 12 * kNoallocMaxCells;
constexpr size_t kNoallocBucketOff = kNoallocPermOff + 4 * kNoallocMaxCells;
constexpr size_t kNoallocBytes = kNoallocBucketOff + kNoallocMaxCells;

struct Options {
    int form = CHEM_FORM_AUTO;
    int max_substeps = 100000;
    double hmin_rel = 1e-20;
    const double* h0 = nullptr;
    int checkpoint_every = 0;   // adjoint: 0 = chosen per call (see run_adjoint)
    const int32_t* adjoint_nacc = nullptr;   // adjoint: a forward's accepted steps (skips the sizing pass)
    int block = 0;
    int waves_per_simd = 0;
    int refill = 0;
    int order = CHEM_ORDER_AUTO;
    const int32_t* const* cost = nullptr;
};

// One field of cells as the caller passed it.
struct FieldView {
    double* T;
    const double* p;
    double* Y;
    int64_t ncell;
    int32_t* status;
    int32_t* nacc;
    int32_t* nrej;
    const double* h0;
    const int32_t* cost;
};

struct LaunchConfig {
    int block = 64;            // lanes per workgroup
    int waves_per_simd = 1;
    int refill = 16;
    int div = 1;               // launch 1/div of the resident workgroups (the tuner's
                               // sample runs, so a 1/div sample sees the lanes per cell
                               // of the whole field)
    bool operator<(const LaunchConfig& o) const
    {
        return std::tie(block, waves_per_simd, refill, div) < std::tie(o.block, o.waves_per_simd, o.refill, o.div);
    }
};

struct DeviceState {
    int device = -1;
    int num_cu = 256;
    hipModule_t module = nullptr;
    hipFunction_t f_plain = nullptr, f_eval = nullptr, f_fixed = nullptr, f_zero = nullptr,
                  f_stats = nullptr, f_persistent = nullptr, f_reset = nullptr, f_gather = nullptr,
                  f_okey = nullptr, f_oscan = nullptr, f_oscatter = nullptr, f_adjoint = nullptr,
                  f_rparams = nullptr, f_src_begin = nullptr, f_src_end = nullptr, f_euler_prim = nullptr,
                  f_euler_update = nullptr, f_euler_init = nullptr;
    double* par = nullptr;               // 3 * nr device doubles
    uint64_t par_version = 0;
    unsigned long long* stats = nullptr; // 4 counters
    unsigned long long* heads = nullptr; // queue heads (persistent)
    char* block_buf = nullptr;           // PersistBlock (header + fields)
    size_t block_cap = 0;                // fields capacity
    int32_t* cells_i32 = nullptr;        // status, nacc, nrej workspace [3 * cap]
    size_t cells_cap = 0;
    double* sample = nullptr;            // autotune sample buffers
    size_t sample_cap = 0;
    unsigned char* bucket = nullptr;     // cost ordering: bucket per cell
    size_t bucket_cap = 0;
    int* perm = nullptr;                 // cost ordering: cells by descending cost
    size_t perm_cap = 0;
    unsigned* hist = nullptr;            // [2 * kCostBuckets]: histogram, cursors
    hipStream_t capture_stream = nullptr;
    std::map<LaunchConfig, hipGraphExec_t> graphs;
    std::map<int64_t, hipGraphExec_t> wide_graphs;   // wave-cooperative launch, by grid size
    // by log2 bucket of the total cell count: the tuned launch shape and cell
    // order (CHEM_ORDER_COST or CHEM_ORDER_NATURAL)
    std::map<int64_t, std::pair<LaunchConfig, int>> tuned;
    std::string arch;                    // gcnArchName
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    // recorded after every API call's work: the next call's stream waits on
    // it, so the shared workspace is reused in order even across streams
    hipEvent_t done = nullptr;
    bool done_recorded = false;
    size_t lds_per_block = 65536;
    unsigned char* noalloc = nullptr;    // this device's allocation-free scratch (see noalloc.hip)
    double* euler = nullptr;             // 1D driver buffers, [cap][2 ns + 7] doubles
    size_t euler_cap = 0;                // cells
    unsigned long long* euler_flags = nullptr;   // 1D driver: bad flag, max CFL (bits)
    int n = 0;                           // state size ns + 1
    // LDS doubles a lane of the one-cell-per-lane kernels holds: the RODAS4
    // stage vectors u_1..u_5, or from 12 unknowns on up to 80 entries of the
    // LU factors (the device code's kLaneWords never exceeds this)
    int lane_words() const { return n >= 12 ? 80 : 5 * n; }
    unsigned stage_lds(int block) const { return (unsigned)(block * lane_words() * sizeof(double)); }
};

}  // namespace chemmi

struct chem_mechanism {
    chemmi::MechanismData data;
    bool wide = false;                   // wave-cooperative kernels (else one cell per lane)
    chemmi::WideLayout layout;           // of the wave-cooperative form
    std::vector<double> params;          // lnA[nr], b[nr], Ea/R[nr]
    uint64_t params_version = 1;
    std::string source;
    std::vector<char> code;
    std::string cache_file;
    std::mutex mu;
    std::map<int, chemmi::DeviceState> devices;
};

namespace chemmi {

int set_error(int code, const std::string& msg);
int hip_error(hipError_t e, const char* what);
bool is_device_ptr(const void* p);

// Device state for the current device (module loaded, parameters current).
int device_state(chem_mechanism* m, hipStream_t stream, DeviceState** out);
// Record the end of an API call's work on `stream` (see DeviceState::done).
void mark_done(chem_mechanism* m, hipStream_t stream);
void release_device_state(chem_mechanism* m);

int launch_1d(hipFunction_t f, int64_t n, int block, void* args, size_t size, hipStream_t stream,
              const char* what, unsigned shmem = 0);

// Device address of this device's allocation-free scratch (hipGetSymbolAddress
// once per device, with `device` current), and the field-table writer.
int noalloc_scratch(int device, void** out);
int noalloc_write_block(char* dst, const PersistHeader& h, const FieldDesc& f, hipStream_t stream);

// chem_integrate_noalloc: the persistent form with every temporary in the
// device's fixed scratch; needs the device state set up already.
int run_noalloc(chem_mechanism* m, int64_t ncell, double* T, const double* p, double* Y, double dt,
                double rtol, double atol, const Options& o, int32_t* status, int32_t* nacc, int32_t* nrej,
                hipStream_t stream);

// Set up the device state on the current device if a gfx950 device is
// current (at mechanism load); no effect without a usable device.
void prepare_current_device(chem_mechanism* m);

int run_plain(chem_mechanism* m, int64_t ncell, double* T, const double* p, double* Y, double dt,
              double rtol, double atol, const Options& o, chem_stats* stats, int32_t* status,
              int32_t* nacc, int32_t* nrej, hipStream_t stream);

int run_persistent(chem_mechanism* m, const FieldView* fields, int nfield, double dt, double rtol,
                   double atol, const Options& o, chem_stats* stats, hipStream_t stream);

// Integration with the operator-split source terms (see chem_integrate_source):
// the initial density and state are kept in wdot/qdot, the cells integrated in
// the form o asks for, and the mean rates over the step written back.
// Conserved 1D state U from T, p, Y and u (u may be null).
int run_euler1d_init(chem_mechanism* m, int64_t ncell, const double* T, const double* p, const double* Y,
                     const double* u, double* U, hipStream_t stream);

// One step of the 1D reactive-Euler driver: primitive recovery, the coupled
// chemistry step over dt (run_source), and the finite-volume update with the
// chemistry's source terms; *max_cfl gets the largest (|u| + c) dt / dx.
int run_euler1d(chem_mechanism* m, int64_t ncell, double dx, double dt, const double* U, double* U_out,
                double* T, double rtol, double atol, const Options& o, chem_stats* stats, double* max_cfl,
                hipStream_t stream);

int run_source(chem_mechanism* m, int64_t ncell, double* T, const double* p, double* Y, double dt,
               double rtol, double atol, const Options& o, chem_stats* stats, int32_t* status,
               double* wdot, double* qdot, hipStream_t stream);

// Discrete adjoint (see chem_integrate_adjoint); the arrays are as there, with
// T_end/Y_end non-null.
int run_adjoint(chem_mechanism* m, int64_t ncell, const double* T0, const double* p, const double* Y0,
                double dt, double rtol, double atol, const double* gT, const double* gY, double* gT0,
                double* gY0, double* g_lnA, double* g_b, double* g_Ea, double* T_end, double* Y_end,
                const Options& o, chem_stats* stats, hipStream_t stream);

}  // namespace chemmi
