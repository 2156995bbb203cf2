// runtime.cpp -- per-device module and workspace, plain and persistent launches,
// the HIP-graph cache and the launch-shape autotuner.
#include "runtime.hpp"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <sstream>
#include <tuple>

#include <unistd.h>

#include "module.hpp"

namespace chemmi {

namespace {

#define HIPCHECK(expr, what)                          \
    do {                                              \
        hipError_t e_ = (expr);                       \
        if (e_ != hipSuccess) return hip_error(e_, what); \
    } while (0)

int load_function(hipModule_t mod, const char* name, hipFunction_t* f)
{
    hipError_t e = hipModuleGetFunction(f, mod, name);
    if (e != hipSuccess) return hip_error(e, name);
    return 0;
}

template <class T>
int grow(T** ptr, size_t* cap, size_t want, const char* what)
{
    if (*cap >= want && *ptr) return 0;
    if (*ptr) (void)hipFree(*ptr);
    *ptr = nullptr;
    *cap = 0;
    size_t n = std::max<size_t>(want, 1);
    HIPCHECK(hipMalloc((void**)ptr, n * sizeof(T)), what);
    *cap = n;
    return 0;
}

int64_t size_bucket(int64_t total)
{
    int64_t b = 0;
    while ((int64_t(1) << (b + 1)) <= total) ++b;
    return b;
}

}  // namespace

int launch_1d(hipFunction_t f, int64_t n, int block, void* args, size_t size, hipStream_t stream,
              const char* what, unsigned shmem)
{
    void* cfg[] = {HIP_LAUNCH_PARAM_BUFFER_POINTER, args, HIP_LAUNCH_PARAM_BUFFER_SIZE, &size,
                   HIP_LAUNCH_PARAM_END};
    const int64_t grid = (n + block - 1) / block;
    if (grid > 0x7fffffff) return set_error(CHEM_E_INVAL, "too many cells for one launch");
    HIPCHECK(hipModuleLaunchKernel(f, (unsigned)grid, 1, 1, block, 1, 1, shmem, stream, nullptr, cfg), what);
    return 0;
}

int state_ready(chem_mechanism* m, DeviceState& d, hipStream_t stream, DeviceState** out);

int device_state(chem_mechanism* m, hipStream_t stream, DeviceState** out)
{
    (void)stream;
    int dev = 0;
    HIPCHECK(hipGetDevice(&dev), "hipGetDevice");
    DeviceState& d = m->devices[dev];
    if (!d.module) {
        d.device = dev;
        hipDeviceProp_t prop;
        HIPCHECK(hipGetDeviceProperties(&prop, dev), "hipGetDeviceProperties");
        if (std::string(prop.gcnArchName).rfind("gfx950", 0) != 0)
            return set_error(CHEM_E_UNSUPPORTED, std::string("device is ") + prop.gcnArchName +
                                                     "; this library is built for gfx950");
        d.num_cu = prop.multiProcessorCount;
        d.arch = prop.gcnArchName;
        d.lds_per_block = prop.sharedMemPerBlock;
        d.n = m->data.ns() + 1;
        HIPCHECK(hipModuleLoadData(&d.module, m->code.data()), "hipModuleLoadData");
        int rc = 0;
        rc = rc ? rc : load_function(d.module, "chem_plain", &d.f_plain);
        rc = rc ? rc : load_function(d.module, "chem_eval", &d.f_eval);
        rc = rc ? rc : load_function(d.module, "chem_zero_u64", &d.f_zero);
        rc = rc ? rc : load_function(d.module, "chem_reduce_stats", &d.f_stats);
        rc = rc ? rc : load_function(d.module, "chem_persistent", &d.f_persistent);
        rc = rc ? rc : load_function(d.module, "chem_reset_heads", &d.f_reset);
        rc = rc ? rc : load_function(d.module, "chem_adjoint", &d.f_adjoint);
        rc = rc ? rc : load_function(d.module, "chem_reduce_params", &d.f_rparams);
        rc = rc ? rc : load_function(d.module, "chem_source_begin", &d.f_src_begin);
        rc = rc ? rc : load_function(d.module, "chem_source_end", &d.f_src_end);
        rc = rc ? rc : load_function(d.module, "chem_euler_prim", &d.f_euler_prim);
        rc = rc ? rc : load_function(d.module, "chem_euler_update", &d.f_euler_update);
        rc = rc ? rc : load_function(d.module, "chem_euler_init", &d.f_euler_init);
        rc = rc ? rc : load_function(d.module, "chem_fixed_step", &d.f_fixed);
        if (!m->wide) {   // one-cell-per-lane module only
            rc = rc ? rc : load_function(d.module, "chem_gather_sample", &d.f_gather);
            rc = rc ? rc : load_function(d.module, "chem_order_key", &d.f_okey);
            rc = rc ? rc : load_function(d.module, "chem_order_scan", &d.f_oscan);
            rc = rc ? rc : load_function(d.module, "chem_order_scatter", &d.f_oscatter);
        }
        if (rc) return rc;
        HIPCHECK(hipMalloc((void**)&d.par, sizeof(double) * std::max<size_t>(m->params.size(), 1)), "hipMalloc par");
        HIPCHECK(hipMalloc((void**)&d.stats, sizeof(unsigned long long) * 4), "hipMalloc stats");
        HIPCHECK(hipMalloc((void**)&d.heads, sizeof(unsigned long long) * 64), "hipMalloc heads");
        HIPCHECK(hipMalloc((void**)&d.hist, sizeof(unsigned) * 2 * kCostBuckets), "hipMalloc hist");
        HIPCHECK(hipEventCreate(&d.ev0), "hipEventCreate");
        HIPCHECK(hipEventCreate(&d.ev1), "hipEventCreate");
        HIPCHECK(hipEventCreateWithFlags(&d.done, hipEventDisableTiming), "hipEventCreate");
        void* na = nullptr;
        if (int rc2 = noalloc_scratch(dev, &na)) return rc2;
        d.noalloc = static_cast<unsigned char*>(na);
        d.par_version = 0;
    }
    return state_ready(m, d, stream, out);
}

int state_ready(chem_mechanism* m, DeviceState& d, hipStream_t stream, DeviceState** out)
{
    // the previous call's work may still run on another stream
    if (d.done_recorded) HIPCHECK(hipStreamWaitEvent(stream, d.done, 0), "order after the previous call");
    if (d.par_version != m->params_version) {
        // stream-ordered after earlier work that read the old parameters
        HIPCHECK(hipMemcpyAsync(d.par, m->params.data(), sizeof(double) * m->params.size(),
                                hipMemcpyHostToDevice, stream),
                 "copy parameters");
        HIPCHECK(hipStreamSynchronize(stream), "sync parameters");
        d.par_version = m->params_version;
    }
    *out = &d;
    return 0;
}

void prepare_current_device(chem_mechanism* m)
{
    int count = 0, dev = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count == 0 || hipGetDevice(&dev) != hipSuccess) {
        (void)hipGetLastError();
        return;
    }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess ||
        std::string(prop.gcnArchName).rfind("gfx950", 0) != 0) {
        (void)hipGetLastError();
        return;
    }
    DeviceState* d;
    if (device_state(m, nullptr, &d)) {
        // left for the first call on the device to report
        release_device_state(m);
        (void)hipGetLastError();
    }
}

void mark_done(chem_mechanism* m, hipStream_t stream)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return;
    auto it = m->devices.find(dev);
    if (it == m->devices.end() || !it->second.done) return;
    if (hipEventRecord(it->second.done, stream) == hipSuccess) it->second.done_recorded = true;
}

void release_device_state(chem_mechanism* m)
{
    int cur = 0;
    (void)hipGetDevice(&cur);
    for (auto& kv : m->devices) {
        DeviceState& d = kv.second;
        (void)hipSetDevice(d.device);
        for (auto& g : d.graphs) (void)hipGraphExecDestroy(g.second);
        for (auto& g : d.wide_graphs) (void)hipGraphExecDestroy(g.second);
        if (d.capture_stream) (void)hipStreamDestroy(d.capture_stream);
        for (void* p : {(void*)d.par, (void*)d.stats, (void*)d.heads, (void*)d.block_buf,
                        (void*)d.cells_i32, (void*)d.sample, (void*)d.bucket, (void*)d.perm, (void*)d.hist,
                        (void*)d.euler, (void*)d.euler_flags})
            if (p) (void)hipFree(p);
        if (d.ev0) (void)hipEventDestroy(d.ev0);
        if (d.ev1) (void)hipEventDestroy(d.ev1);
        if (d.done) (void)hipEventDestroy(d.done);
        if (d.module) (void)hipModuleUnload(d.module);
    }
    m->devices.clear();
    (void)hipSetDevice(cur);
}

namespace {

// Reduce per-cell counters into stats (synchronises the stream).
int collect_stats(DeviceState& d, const int32_t* status, const int32_t* nacc, const int32_t* nrej,
                  int64_t ncell, float ms, chem_stats* stats, hipStream_t stream)
{
    int n4 = 4;
    unsigned long long* sp = d.stats;
    struct { unsigned long long* p; int n; } za{sp, n4};
    if (int rc = launch_1d(d.f_zero, 4, 64, &za, sizeof za, stream, "chem_zero_u64")) return rc;
    struct {
        const int32_t* s;
        const int32_t* a;
        const int32_t* r;
        long n;
        unsigned long long* out;
    } ra{status, nacc, nrej, (long)ncell, sp};
    const int64_t threads = std::min<int64_t>(ncell, (int64_t)d.num_cu * 4 * 256);
    if (int rc = launch_1d(d.f_stats, threads, 256, &ra, sizeof ra, stream, "chem_reduce_stats")) return rc;
    unsigned long long h[4];
    HIPCHECK(hipMemcpyAsync(h, sp, sizeof h, hipMemcpyDeviceToHost, stream), "copy stats");
    HIPCHECK(hipStreamSynchronize(stream), "sync stats");
    stats->cells = ncell;
    stats->accepted = (int64_t)h[0];
    stats->rejected = (int64_t)h[1];
    stats->failed = (int64_t)h[2];
    stats->max_substeps = (int64_t)h[3];
    stats->kernel_ms = ms;
    if (stats->failed) return set_error(CHEM_E_CELL_FAILED, std::to_string(stats->failed) + " cells failed");
    return 0;
}

StepArgs step_args(double dt, double rtol, double atol, const Options& o)
{
    return StepArgs{dt, rtol, atol, o.hmin_rel * dt, o.max_substeps};
}

}  // namespace

int run_plain(chem_mechanism* m, int64_t ncell, double* T, const double* p, double* Y, double dt,
              double rtol, double atol, const Options& o, chem_stats* stats, int32_t* status,
              int32_t* nacc, int32_t* nrej, hipStream_t stream)
{
    DeviceState* d;
    if (int rc = device_state(m, stream, &d)) return rc;
    // per-cell counters the caller did not ask for go to the workspace when the
    // statistics need them, and are not written otherwise
    if (stats && (!status || !nacc || !nrej))
        if (int rc = grow(&d->cells_i32, &d->cells_cap, 3 * (size_t)ncell, "workspace")) return rc;
    int32_t* st = status ? status : stats ? d->cells_i32 : nullptr;
    int32_t* na = nacc ? nacc : stats ? d->cells_i32 + ncell : nullptr;
    int32_t* nr = nrej ? nrej : stats ? d->cells_i32 + 2 * ncell : nullptr;
    IntegrateArgs a{d->par, T, p, Y, (long)ncell, o.h0, st, na, nr, step_args(dt, rtol, atol, o)};
    if (stats) HIPCHECK(hipEventRecord(d->ev0, stream), "event");
    // one lane per cell, or one group of G lanes per cell in the wave-cooperative form
    const int64_t lanes = m->wide ? ncell * m->layout.G : ncell;
    const unsigned shmem = m->wide ? m->layout.lds_bytes() : d->stage_lds(64);
    if (int rc = launch_1d(d->f_plain, lanes, 64, &a, sizeof a, stream, "chem_plain", shmem)) return rc;
    if (!stats) return 0;
    HIPCHECK(hipEventRecord(d->ev1, stream), "event");
    HIPCHECK(hipEventSynchronize(d->ev1), "event sync");
    float ms = 0.f;
    HIPCHECK(hipEventElapsedTime(&ms, d->ev0, d->ev1), "elapsed");
    return collect_stats(*d, st, na, nr, ncell, ms, stats, stream);
}

// ---------------- persistent form ----------------

namespace {

int write_block(DeviceState& d, const std::vector<FieldDesc>& fields, const PersistHeader& h,
                hipStream_t stream)
{
    const size_t bytes = sizeof(PersistHeader) + fields.size() * sizeof(FieldDesc);
    if (d.block_cap < bytes || !d.block_buf) {
        if (d.block_buf) (void)hipFree(d.block_buf);
        d.block_buf = nullptr;
        d.block_cap = 0;
        // graphs hold the old address
        for (auto& g : d.graphs) (void)hipGraphExecDestroy(g.second);
        d.graphs.clear();
        for (auto& g : d.wide_graphs) (void)hipGraphExecDestroy(g.second);
        d.wide_graphs.clear();
        const size_t cap = std::max<size_t>(bytes, sizeof(PersistHeader) + 64 * sizeof(FieldDesc));
        HIPCHECK(hipMalloc((void**)&d.block_buf, cap), "hipMalloc field table");
        d.block_cap = cap;
    }
    std::vector<char> host(bytes);
    std::memcpy(host.data(), &h, sizeof h);
    std::memcpy(host.data() + sizeof h, fields.data(), fields.size() * sizeof(FieldDesc));
    // pageable source: the copy is staged before this call returns
    HIPCHECK(hipMemcpyAsync(d.block_buf, host.data(), bytes, hipMemcpyHostToDevice, stream),
             "copy field table");
    return 0;
}

int grid_of(const DeviceState& d, const LaunchConfig& c)
{
    // resident workgroups: CUs x 4 SIMDs x waves per SIMD, 64-lane waves
    const int waves = d.num_cu * 4 * c.waves_per_simd;
    return std::max(1, waves * 64 / c.block / std::max(1, c.div));
}

// Launch [reset -> cost keys -> bucket offsets -> permutation -> persistent
// kernel] as a graph built once per launch shape (the kernels read everything
// call-specific from the field table, whose device address is fixed).
int launch_graph(DeviceState& d, const LaunchConfig& c, hipStream_t stream)
{
    auto it = d.graphs.find(c);
    if (it == d.graphs.end()) {
        if (!d.capture_stream) HIPCHECK(hipStreamCreateWithFlags(&d.capture_stream, hipStreamNonBlocking), "stream");
        hipGraph_t g;
        HIPCHECK(hipStreamBeginCapture(d.capture_stream, hipStreamCaptureModeThreadLocal), "begin capture");
        struct { const char* blk; unsigned long long* h; } ra{d.block_buf, d.heads};
        struct { const char* blk; const double* par; } ka{d.block_buf, d.par};
        struct { const char* blk; } sa{d.block_buf};
        struct { const char* blk; unsigned long long* heads; const double* par; } pa{d.block_buf, d.heads, d.par};
        auto launch = [&](hipFunction_t f, unsigned grid, unsigned block, unsigned shmem, void* args,
                          size_t size) {
            void* cfg[] = {HIP_LAUNCH_PARAM_BUFFER_POINTER, args, HIP_LAUNCH_PARAM_BUFFER_SIZE, &size,
                           HIP_LAUNCH_PARAM_END};
            return hipModuleLaunchKernel(f, grid, 1, 1, block, 1, 1, shmem, d.capture_stream, nullptr, cfg);
        };
        const unsigned sweep = (unsigned)d.num_cu * 4;   // grid-stride sweeps over all cells
        hipError_t e = launch(d.f_reset, 1, 256, 0, &ra, sizeof ra);
        if (e == hipSuccess) e = launch(d.f_okey, sweep, 256, 0, &ka, sizeof ka);
        if (e == hipSuccess) e = launch(d.f_oscan, 1, kCostBuckets, 0, &sa, sizeof sa);
        if (e == hipSuccess) e = launch(d.f_oscatter, sweep, 256, 0, &sa, sizeof sa);
        if (e == hipSuccess)
            e = launch(d.f_persistent, grid_of(d, c), c.block, d.stage_lds(c.block), &pa, sizeof pa);
        hipError_t e2 = hipStreamEndCapture(d.capture_stream, &g);
        if (e != hipSuccess) return hip_error(e, "capture persistent launch");
        if (e2 != hipSuccess) return hip_error(e2, "end capture");
        hipGraphExec_t ex;
        hipError_t e3 = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e3 != hipSuccess) return hip_error(e3, "graph instantiate");
        it = d.graphs.emplace(c, ex).first;
    }
    HIPCHECK(hipGraphLaunch(it->second, stream), "graph launch");
    return 0;
}

// counts: the launch's statistics are wanted, so the per-cell counters the
// caller did not ask for go to the workspace; otherwise they are not written.
int fill_fields(DeviceState& d, const FieldView* fv, int nfield, std::vector<FieldDesc>& out,
                int64_t& total, bool counts)
{
    total = 0;
    for (int f = 0; f < nfield; ++f) total += fv[f].ncell;
    if (total >= (int64_t(1) << 31)) return set_error(CHEM_E_INVAL, "more than 2^31 - 1 cells in one launch");
    if (int rc = grow(&d.cells_i32, &d.cells_cap, 3 * (size_t)total, "workspace")) return rc;
    if (int rc = grow(&d.bucket, &d.bucket_cap, (size_t)total, "workspace")) return rc;
    if (int rc = grow(&d.perm, &d.perm_cap, (size_t)total, "workspace")) return rc;
    out.clear();
    int64_t start = 0;
    for (int f = 0; f < nfield; ++f) {
        FieldDesc x;
        x.T = fv[f].T;
        x.p = fv[f].p;
        x.Y = fv[f].Y;
        x.status = fv[f].status ? fv[f].status : counts ? d.cells_i32 + start : nullptr;
        x.nacc = fv[f].nacc ? fv[f].nacc : counts ? d.cells_i32 + total + start : nullptr;
        x.nrej = fv[f].nrej ? fv[f].nrej : counts ? d.cells_i32 + 2 * total + start : nullptr;
        x.cost = fv[f].cost;
        x.ncell = (long)fv[f].ncell;
        x.start = (long)start;
        out.push_back(x);
        start += fv[f].ncell;
    }
    return 0;
}

PersistHeader header_for(const DeviceState& d, int64_t total, int nfield, const LaunchConfig& c,
                         const StepArgs& s, int order)
{
    PersistHeader h{};
    h.total = (long)total;
    h.nq = 8;                                        // one queue per XCD
    h.nfield = nfield;
    h.refill = std::max(1, std::min(64, c.refill));
    h.order = order == CHEM_ORDER_NATURAL ? 0 : 1;
    h.step = s;
    h.bucket = d.bucket;
    h.perm = d.perm;
    h.hist = d.hist;
    h.cursor = d.hist + kCostBuckets;
    return h;
}

// The on-disk record of a tuning result: one line "block refill order" in
// $CHEM_TUNE_CACHE (else the kernel cache folder) under a name that hashes the
// mechanism's code object (which names its source, options and compiler), the
// device's architecture and compute-unit count, the size bucket and any shape
// the caller fixed.
std::string tune_file(const chem_mechanism* m, const DeviceState& d, int64_t bucket, const Options& o)
{
    std::ostringstream k;
    const std::string& cf = m->cache_file;
    k << cf.substr(cf.find_last_of('/') + 1) << ' ' << d.arch << ' ' << d.num_cu << ' ' << bucket << ' ' << o.block
      << ' ' << o.refill << ' ' << o.order;
    char name[48];
    std::snprintf(name, sizeof name, "/tune-%016llx.txt", (unsigned long long)fnv1a(k.str()));
    const char* env = std::getenv("CHEM_TUNE_CACHE");
    return (env && *env ? std::string(env) : cache_dir()) + name;
}

bool read_tuned(const std::string& path, LaunchConfig* c, int* order)
{
    std::ifstream in(path);
    int b = 0, r = 0, od = 0;
    if (!(in >> b >> r >> od)) return false;
    if (b < 64 || b > 256 || b % 64 || r < 1 || r > 64 || (od != CHEM_ORDER_COST && od != CHEM_ORDER_NATURAL))
        return false;
    *c = LaunchConfig{b, 1, r};
    *order = od;
    return true;
}

void write_tuned(const std::string& path, const LaunchConfig& c, int order, float ms)
{
    const std::string tmp = path + ".tmp" + std::to_string(getpid());
    {
        std::ofstream out(tmp);
        if (!out) return;
        out << c.block << ' ' << c.refill << ' ' << order << '\n' << "# sample time " << ms << " ms\n";
        if (!out) return;
    }
    std::rename(tmp.c_str(), path.c_str());
}

// The wave-cooperative persistent launch [reset -> persistent kernel] as a
// graph built once per grid size (everything call-specific is in the field
// table, whose device address is fixed).
int launch_graph_wide(DeviceState& d, const chem_mechanism* m, int64_t waves, hipStream_t stream)
{
    auto it = d.wide_graphs.find(waves);
    if (it == d.wide_graphs.end()) {
        if (!d.capture_stream) HIPCHECK(hipStreamCreateWithFlags(&d.capture_stream, hipStreamNonBlocking), "stream");
        hipGraph_t g;
        HIPCHECK(hipStreamBeginCapture(d.capture_stream, hipStreamCaptureModeThreadLocal), "begin capture");
        struct { const char* blk; unsigned long long* h; } ra{d.block_buf, d.heads};
        struct { const char* blk; unsigned long long* heads; const double* par; } pa{d.block_buf, d.heads, d.par};
        size_t rs = sizeof ra, ps = sizeof pa;
        void* rcfg[] = {HIP_LAUNCH_PARAM_BUFFER_POINTER, &ra, HIP_LAUNCH_PARAM_BUFFER_SIZE, &rs, HIP_LAUNCH_PARAM_END};
        void* pcfg[] = {HIP_LAUNCH_PARAM_BUFFER_POINTER, &pa, HIP_LAUNCH_PARAM_BUFFER_SIZE, &ps, HIP_LAUNCH_PARAM_END};
        hipError_t e = hipModuleLaunchKernel(d.f_reset, 1, 1, 1, 256, 1, 1, 0, d.capture_stream, nullptr, rcfg);
        if (e == hipSuccess)
            e = hipModuleLaunchKernel(d.f_persistent, (unsigned)waves, 1, 1, 64, 1, 1, m->layout.lds_bytes(),
                                      d.capture_stream, nullptr, pcfg);
        hipError_t e2 = hipStreamEndCapture(d.capture_stream, &g);
        if (e != hipSuccess) return hip_error(e, "capture wave-cooperative launch");
        if (e2 != hipSuccess) return hip_error(e2, "end capture");
        hipGraphExec_t ex;
        hipError_t e3 = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e3 != hipSuccess) return hip_error(e3, "graph instantiate");
        it = d.wide_graphs.emplace(waves, ex).first;
    }
    HIPCHECK(hipGraphLaunch(it->second, stream), "graph launch");
    return 0;
}

// Time candidate launch shapes and cell orders on a strided sample of the input
// (copied, so the caller's data is untouched) and keep the fastest per size
// bucket, in memory and on disk.  Every candidate gives bitwise the same
// results; only the time differs.  The order is a candidate only when the
// caller left it to the tuner (CHEM_ORDER_AUTO).
int autotune(chem_mechanism* m, DeviceState& d, const std::vector<FieldDesc>& fields, int64_t total,
             const StepArgs& s, const Options& o, hipStream_t stream, LaunchConfig* best, int* best_order)
{
    const int64_t bucket = size_bucket(total);
    auto hit = d.tuned.find(bucket);
    if (hit != d.tuned.end()) {
        *best = hit->second.first;
        *best_order = hit->second.second;
        return 0;
    }
    const std::string record = tune_file(m, d, bucket, o);
    if (read_tuned(record, best, best_order)) {
        if (std::getenv("CHEM_LOG"))
            std::fprintf(stderr, "[chem] autotune cache hit %s: block=%d refill=%d order=%d\n", record.c_str(),
                         best->block, best->refill, *best_order);
        d.tuned[bucket] = {*best, *best_order};
        return 0;
    }
    const int ns = m->data.ns();
    const int64_t want = std::min<int64_t>(total, std::max<int64_t>(65536, total / 16));
    const int64_t stride = std::max<int64_t>(1, total / want);
    const int64_t count = (total + stride - 1) / stride;
    const size_t per = (size_t)count * (ns + 2);
    if (int rc = grow(&d.sample, &d.sample_cap, 2 * per, "autotune sample")) return rc;
    double* sT = d.sample;
    double* sp = sT + count;
    double* sY = sp + count;
    double* wT = d.sample + per;                      // working copy
    PersistHeader h = header_for(d, total, (int)fields.size(), LaunchConfig{}, s, CHEM_ORDER_NATURAL);
    if (int rc = write_block(d, fields, h, stream)) return rc;
    struct { const char* blk; long stride; long count; double* T; double* p; double* Y; } ga{
        d.block_buf, (long)stride, (long)count, sT, sp, sY};
    if (int rc = launch_1d(d.f_gather, count, 256, &ga, sizeof ga, stream, "chem_gather_sample")) return rc;

    // the sample runs on 1/stride of the workgroups, so its lanes take as many
    // cells each as the whole field's will (the cell order matters only then)
    // (a sample run then takes about as long as the whole field, so the shapes
    // are a short list: the block sizes at one refill threshold and the
    // thresholds at one block size; the other order is tried with the best shape)
    std::vector<LaunchConfig> cands;
    for (auto br : {std::make_pair(64, 16), std::make_pair(128, 16), std::make_pair(256, 16), std::make_pair(64, 4),
                    std::make_pair(64, 32)})
        if (d.stage_lds(br.first) <= d.lds_per_block) cands.push_back(LaunchConfig{br.first, 1, br.second, (int)stride});
    if (o.block) for (auto& c : cands) c.block = o.block;
    if (o.refill) for (auto& c : cands) c.refill = o.refill;
    const int first_order = o.order == CHEM_ORDER_AUTO ? CHEM_ORDER_COST : o.order;
    float best_ms = 1e30f;
    *best = cands[0];
    *best_order = first_order;
    // count <= total, so the per-cell workspace (3 * total) already fits the sample
    std::vector<FieldDesc> sf(1);
    sf[0] = FieldDesc{wT, sp, wT + count, d.cells_i32, d.cells_i32 + count, d.cells_i32 + 2 * count,
                      nullptr, (long)count, 0};
    for (int pass = 0; pass < (o.order == CHEM_ORDER_AUTO ? 2 : 1); ++pass) {
        const int od = pass == 0 ? first_order : CHEM_ORDER_NATURAL;
        const std::vector<LaunchConfig> these = pass == 0 ? cands : std::vector<LaunchConfig>{*best};
        for (const auto& c : these) {
            HIPCHECK(hipMemcpyAsync(wT, sT, sizeof(double) * count, hipMemcpyDeviceToDevice, stream), "sample copy");
            HIPCHECK(hipMemcpyAsync(wT + count, sY, sizeof(double) * count * ns, hipMemcpyDeviceToDevice, stream),
                     "sample copy");
            PersistHeader hs = header_for(d, count, 1, c, s, od);
            if (int rc = write_block(d, sf, hs, stream)) return rc;
            HIPCHECK(hipEventRecord(d.ev0, stream), "event");
            if (int rc = launch_graph(d, c, stream)) return rc;
            HIPCHECK(hipEventRecord(d.ev1, stream), "event");
            HIPCHECK(hipEventSynchronize(d.ev1), "event sync");
            float ms = 0.f;
            HIPCHECK(hipEventElapsedTime(&ms, d.ev0, d.ev1), "elapsed");
            if (std::getenv("CHEM_LOG"))
                std::fprintf(stderr, "[chem] autotune block=%d refill=%d order=%d: %.3f ms\n", c.block, c.refill,
                             od, ms);
            if (ms < best_ms) {
                best_ms = ms;
                *best = c;
                *best_order = od;
            }
        }
    }
    best->div = 1;
    d.tuned[bucket] = {*best, *best_order};
    write_tuned(record, *best, *best_order, best_ms);
    return 0;
}

}  // namespace

// Wave-cooperative form: groups of lanes pull cells from one counter (no
// cost ordering: a whole wave serves one to four cells, so the hardware's
// dispatch of waves and the refill of groups already balance the load).
int run_persistent_wide(chem_mechanism* m, const FieldView* fv, int nfield, double dt, double rtol,
                        double atol, const Options& o, chem_stats* stats, hipStream_t stream)
{
    DeviceState* d;
    if (int rc = device_state(m, stream, &d)) return rc;
    for (int f = 0; f < nfield; ++f)
        if (fv[f].h0) return set_error(CHEM_E_INVAL, "h0 is not supported by the persistent form");
    std::vector<FieldDesc> fields;
    int64_t total = 0;
    if (int rc = fill_fields(*d, fv, nfield, fields, total, stats != nullptr)) return rc;
    const StepArgs s = step_args(dt, rtol, atol, o);
    LaunchConfig c{64, 1, 1};
    if (int rc = write_block(*d, fields, header_for(*d, total, nfield, c, s, CHEM_ORDER_NATURAL), stream)) return rc;
    if (stats) HIPCHECK(hipEventRecord(d->ev0, stream), "event");
    // resident waves: as many as the LDS scratch allows, at most 8 per CU
    const unsigned per_cu = std::max<unsigned>(1u, std::min<unsigned>(8u, (unsigned)(160u * 1024u / std::max(1u, m->layout.lds_bytes()))));
    const int64_t waves = std::min<int64_t>((int64_t)d->num_cu * per_cu, (total + m->layout.cells_per_wave() - 1) / m->layout.cells_per_wave());
    if (int rc = launch_graph_wide(*d, m, waves, stream)) return rc;
    if (!stats) return 0;
    HIPCHECK(hipEventRecord(d->ev1, stream), "event");
    HIPCHECK(hipEventSynchronize(d->ev1), "event sync");
    float ms = 0.f;
    HIPCHECK(hipEventElapsedTime(&ms, d->ev0, d->ev1), "elapsed");
    chem_stats tot{};
    tot.kernel_ms = ms;
    for (int f = 0; f < nfield; ++f) {
        chem_stats sf{};
        int rc = collect_stats(*d, fields[f].status, fields[f].nacc, fields[f].nrej, fields[f].ncell, ms, &sf, stream);
        if (rc && rc != CHEM_E_CELL_FAILED) return rc;
        tot.cells += sf.cells;
        tot.accepted += sf.accepted;
        tot.rejected += sf.rejected;
        tot.failed += sf.failed;
        tot.max_substeps = std::max(tot.max_substeps, sf.max_substeps);
    }
    *stats = tot;
    if (tot.failed) return set_error(CHEM_E_CELL_FAILED, std::to_string(tot.failed) + " cells failed");
    return 0;
}

int run_persistent(chem_mechanism* m, const FieldView* fv, int nfield, double dt, double rtol,
                   double atol, const Options& o, chem_stats* stats, hipStream_t stream)
{
    if (m->wide) return run_persistent_wide(m, fv, nfield, dt, rtol, atol, o, stats, stream);
    DeviceState* d;
    if (int rc = device_state(m, stream, &d)) return rc;
    for (int f = 0; f < nfield; ++f)
        if (fv[f].h0) return set_error(CHEM_E_INVAL, "h0 is not supported by the persistent form");
    std::vector<FieldDesc> fields;
    int64_t total = 0;
    if (int rc = fill_fields(*d, fv, nfield, fields, total, stats != nullptr)) return rc;
    const StepArgs s = step_args(dt, rtol, atol, o);
    LaunchConfig c;
    int order = o.order;
    if (o.block && o.refill && o.order != CHEM_ORDER_AUTO) {
        c = LaunchConfig{o.block, std::max(1, o.waves_per_simd), o.refill};
    } else if (int rc = autotune(m, *d, fields, total, s, o, stream, &c, &order)) {
        return rc;
    }
    if (o.order != CHEM_ORDER_AUTO) order = o.order;   // the caller's order, whatever a cached tuning chose
    if (c.block < 64 || c.block > 256 || c.block % 64) return set_error(CHEM_E_INVAL, "block must be 64..256, a multiple of 64");
    if (d->stage_lds(c.block) > d->lds_per_block)
        return set_error(CHEM_E_INVAL, "block too large for the stage vectors in LDS");
    if (int rc = write_block(*d, fields, header_for(*d, total, nfield, c, s, order), stream)) return rc;
    if (stats) HIPCHECK(hipEventRecord(d->ev0, stream), "event");
    if (int rc = launch_graph(*d, c, stream)) return rc;
    if (!stats) return 0;
    HIPCHECK(hipEventRecord(d->ev1, stream), "event");
    HIPCHECK(hipEventSynchronize(d->ev1), "event sync");
    float ms = 0.f;
    HIPCHECK(hipEventElapsedTime(&ms, d->ev0, d->ev1), "elapsed");
    if (nfield == 1)
        return collect_stats(*d, fields[0].status, fields[0].nacc, fields[0].nrej, total, ms, stats, stream);
    bool all_ws = true;
    for (int f = 0; f < nfield; ++f) all_ws = all_ws && !fv[f].status && !fv[f].nacc && !fv[f].nrej;
    if (all_ws)   // workspace counters are contiguous over the global index space
        return collect_stats(*d, d->cells_i32, d->cells_i32 + total, d->cells_i32 + 2 * total, total, ms,
                             stats, stream);
    chem_stats tot{};
    tot.kernel_ms = ms;
    for (int f = 0; f < nfield; ++f) {
        chem_stats sf{};
        int rc = collect_stats(*d, fields[f].status, fields[f].nacc, fields[f].nrej, fields[f].ncell, ms, &sf, stream);
        if (rc && rc != CHEM_E_CELL_FAILED) return rc;
        tot.cells += sf.cells;
        tot.accepted += sf.accepted;
        tot.rejected += sf.rejected;
        tot.failed += sf.failed;
        tot.max_substeps = std::max(tot.max_substeps, sf.max_substeps);
    }
    *stats = tot;
    if (tot.failed) return set_error(CHEM_E_CELL_FAILED, std::to_string(tot.failed) + " cells failed");
    return 0;
}

// ---------------- allocation-free persistent launch ----------------

int run_noalloc(chem_mechanism* m, int64_t ncell, double* T, const double* p, double* Y, double dt,
                double rtol, double atol, const Options& o, int32_t* status, int32_t* nacc, int32_t* nrej,
                hipStream_t stream)
{
    if ((uint64_t)ncell > kNoallocMaxCells)
        return set_error(CHEM_E_INVAL, "ncell " + std::to_string(ncell) + " exceeds CHEM_NOALLOC_MAX_CELLS (" +
                                           std::to_string(kNoallocMaxCells) + ")");
    if (o.h0) return set_error(CHEM_E_INVAL, "h0 is not supported by the persistent form");
    int dev = 0;
    HIPCHECK(hipGetDevice(&dev), "hipGetDevice");
    auto it = m->devices.find(dev);
    if (it == m->devices.end() || !it->second.module || !it->second.noalloc)
        return set_error(CHEM_E_INVAL, "the mechanism's device code is not set up on device " + std::to_string(dev) +
                                           " (load the mechanism with that device current, or call another entry "
                                           "point on it first)");
    DeviceState* d;
    if (int rc = state_ready(m, it->second, stream, &d)) return rc;
    unsigned char* base = d->noalloc;
    auto* heads = reinterpret_cast<unsigned long long*>(base + kNoallocHeadsOff);
    auto* hist = reinterpret_cast<unsigned*>(base + kNoallocHistOff);
    char* blk = reinterpret_cast<char*>(base + kNoallocBlockOff);
    auto* counters = reinterpret_cast<int32_t*>(base + kNoallocCountersOff);
    FieldDesc f;
    f.T = T;
    f.p = p;
    f.Y = Y;
    f.status = status ? status : counters;
    f.nacc = nacc ? nacc : counters + kNoallocMaxCells;
    f.nrej = nrej ? nrej : counters + 2 * kNoallocMaxCells;
    f.cost = o.cost ? o.cost[0] : nullptr;
    f.ncell = (long)ncell;
    f.start = 0;
    const StepArgs s = step_args(dt, rtol, atol, o);
    LaunchConfig c;
    int order = o.order == CHEM_ORDER_AUTO ? CHEM_ORDER_COST : o.order;
    if (m->wide) {
        c = LaunchConfig{64, 1, 1};
    } else {
        // the shape and order the tuner chose earlier for this size, else the defaults
        auto t = d->tuned.find(size_bucket(ncell));
        if (t != d->tuned.end()) {
            c = t->second.first;
            if (o.order == CHEM_ORDER_AUTO) order = t->second.second;
        }
        if (o.block && o.refill) c = LaunchConfig{o.block, std::max(1, o.waves_per_simd), o.refill};
    }
    if (c.block < 64 || c.block > 256 || c.block % 64) return set_error(CHEM_E_INVAL, "block must be 64..256, a multiple of 64");
    if (!m->wide && d->stage_lds(c.block) > d->lds_per_block)
        return set_error(CHEM_E_INVAL, "block too large for the stage vectors in LDS");
    PersistHeader h = header_for(*d, ncell, 1, c, s, m->wide ? CHEM_ORDER_NATURAL : order);
    h.bucket = base + kNoallocBucketOff;
    h.perm = reinterpret_cast<int*>(base + kNoallocPermOff);
    h.hist = hist;
    h.cursor = hist + kCostBuckets;
    if (int rc = noalloc_write_block(blk, h, f, stream)) return rc;
    struct { const char* blk; unsigned long long* h; } ra{blk, heads};
    struct { const char* blk; unsigned long long* heads; const double* par; } pa{blk, heads, d->par};
    if (m->wide) {
        if (int rc = launch_1d(d->f_reset, 256, 256, &ra, sizeof ra, stream, "chem_reset_heads")) return rc;
        const unsigned per_cu = std::max<unsigned>(
            1u, std::min<unsigned>(8u, (unsigned)(160u * 1024u / std::max(1u, m->layout.lds_bytes()))));
        const int64_t waves = std::min<int64_t>((int64_t)d->num_cu * per_cu,
                                                (ncell + m->layout.cells_per_wave() - 1) / m->layout.cells_per_wave());
        return launch_1d(d->f_persistent, waves * 64, 64, &pa, sizeof pa, stream, "chem_persistent",
                         m->layout.lds_bytes());
    }
    auto launch = [&](hipFunction_t fn, unsigned grid, unsigned block, unsigned shmem, void* args, size_t size,
                      const char* what) {
        void* cfg[] = {HIP_LAUNCH_PARAM_BUFFER_POINTER, args, HIP_LAUNCH_PARAM_BUFFER_SIZE, &size,
                       HIP_LAUNCH_PARAM_END};
        const hipError_t e = hipModuleLaunchKernel(fn, grid, 1, 1, block, 1, 1, shmem, stream, nullptr, cfg);
        return e == hipSuccess ? 0 : hip_error(e, what);
    };
    struct { const char* blk; const double* par; } ka{blk, d->par};
    struct { const char* blk; } sa{blk};
    const unsigned sweep = (unsigned)d->num_cu * 4;
    int rc = launch(d->f_reset, 1, 256, 0, &ra, sizeof ra, "chem_reset_heads");
    if (!rc) rc = launch(d->f_okey, sweep, 256, 0, &ka, sizeof ka, "chem_order_key");
    if (!rc) rc = launch(d->f_oscan, 1, kCostBuckets, 0, &sa, sizeof sa, "chem_order_scan");
    if (!rc) rc = launch(d->f_oscatter, sweep, 256, 0, &sa, sizeof sa, "chem_order_scatter");
    if (!rc) rc = launch(d->f_persistent, grid_of(*d, c), c.block, d->stage_lds(c.block), &pa, sizeof pa,
                         "chem_persistent");
    return rc;
}

// ---------------- discrete adjoint ----------------

namespace {

// Device temporaries of one adjoint call; freed after the stream drains.
struct Scratch {
    hipStream_t stream;
    std::vector<void*> ptrs;
    explicit Scratch(hipStream_t s) : stream(s) {}
    ~Scratch()
    {
        (void)hipStreamSynchronize(stream);
        for (void* p : ptrs) (void)hipFree(p);
    }
    template <class T>
    int alloc(T** out, size_t count, const char* what)
    {
        *out = nullptr;
        void* p = nullptr;
        HIPCHECK(hipMalloc(&p, std::max<size_t>(count, 1) * sizeof(T)), what);
        ptrs.push_back(p);
        *out = (T*)p;
        return 0;
    }
};

// Cells with at least this fraction of the largest accepted-step count run
// the adjoint in lane groups (one cell per lane form).  0.6: a grouped step
// costs about 0.7 of a lane's, so cells below 0.6 of the maximum finish
// before the grouped ones anyway.  CHEM_ADJOINT_GROUP_FRAC overrides it (0
// turns the groups off).
double adjoint_group_fraction()
{
    if (const char* e = std::getenv("CHEM_ADJOINT_GROUP_FRAC")) {
        char* end = nullptr;
        const double v = std::strtod(e, &end);
        if (end != e && v >= 0.0 && v <= 1.0) return v;
    }
    return 0.6;
}

}  // namespace

int run_source(chem_mechanism* m, int64_t ncell, double* T, const double* p, double* Y, double dt,
               double rtol, double atol, const Options& o, chem_stats* stats, int32_t* status,
               double* wdot, double* qdot, hipStream_t stream)
{
    DeviceState* d;
    if (int rc = device_state(m, stream, &d)) return rc;
    // the status buffer of the integration (the caller's, else the workspace's
    // first ncell entries, sized now so the integration does not move it)
    if (int rc = grow(&d->cells_i32, &d->cells_cap, 3 * (size_t)ncell, "workspace")) return rc;
    int32_t* st = status ? status : d->cells_i32;
    struct {
        const double* T; const double* p; const double* Y; long ncell; double dt; const int* status;
        double* wdot; double* qdot;
    } a{T, p, Y, (long)ncell, dt, st, wdot, qdot};
    if (int rc = launch_1d(d->f_src_begin, ncell, 256, &a, sizeof a, stream, "chem_source_begin")) return rc;
    int rc;
    if (o.form == CHEM_FORM_PERSISTENT) {
        FieldView fv{T, p, Y, ncell, st, nullptr, nullptr, o.h0, o.cost ? o.cost[0] : nullptr};
        rc = run_persistent(m, &fv, 1, dt, rtol, atol, o, stats, stream);
    } else {
        rc = run_plain(m, ncell, T, p, Y, dt, rtol, atol, o, stats, st, nullptr, nullptr, stream);
    }
    if (rc && rc != CHEM_E_CELL_FAILED) return rc;
    if (int rc2 = launch_1d(d->f_src_end, ncell, 256, &a, sizeof a, stream, "chem_source_end")) return rc2;
    return rc;
}

int run_euler1d_init(chem_mechanism* m, int64_t ncell, const double* T, const double* p, const double* Y,
                     const double* u, double* U, hipStream_t stream)
{
    DeviceState* d;
    if (int rc = device_state(m, stream, &d)) return rc;
    struct {
        const double *T, *p, *Y, *u; long n; double* U;
    } a{T, p, Y, u, (long)ncell, U};
    return launch_1d(d->f_euler_init, ncell, 256, &a, sizeof a, stream, "chem_euler_init");
}

int run_euler1d(chem_mechanism* m, int64_t ncell, double dx, double dt, const double* U, double* U_out,
                double* T, double rtol, double atol, const Options& o, chem_stats* stats, double* max_cfl,
                hipStream_t stream)
{
    DeviceState* d;
    if (int rc = device_state(m, stream, &d)) return rc;
    const int ns = m->data.ns();
    // buffers kept per device between steps: p, Y, u, c, wdot, qdot, T (chemistry copy)
    const size_t per = 2 * (size_t)ns + 5;
    if (int rc = grow(&d->euler, &d->euler_cap, per * (size_t)ncell, "1D driver buffers")) return rc;
    if (!d->euler_flags) HIPCHECK(hipMalloc((void**)&d->euler_flags, 2 * sizeof(unsigned long long)), "1D driver flags");
    double* p = d->euler;
    double* Y = p + ncell;
    double* u = Y + (size_t)ncell * ns;
    double* c = u + ncell;
    double* wdot = c + ncell;
    double* qdot = wdot + (size_t)ncell * ns;
    double* Tc = qdot + ncell;
    unsigned long long* flags = d->euler_flags;   // [0]: bad (int in the low word), [1]: max CFL bits
    int* bad = reinterpret_cast<int*>(flags);
    struct { unsigned long long* p; int n; } za{flags, 2};
    if (int rc = launch_1d(d->f_zero, 2, 64, &za, sizeof za, stream, "chem_zero_u64")) return rc;
    struct {
        const double* U; long n; double *T, *p, *Y, *u, *c; int* bad;
    } pa{U, (long)ncell, T, p, Y, u, c, bad};
    if (int rc = launch_1d(d->f_euler_prim, ncell, 256, &pa, sizeof pa, stream, "chem_euler_prim")) return rc;
    // the chemistry advances its own copy of T; Y is a scratch copy already
    HIPCHECK(hipMemcpyAsync(Tc, T, sizeof(double) * ncell, hipMemcpyDeviceToDevice, stream), "copy T");
    const int rc = run_source(m, ncell, Tc, p, Y, dt, rtol, atol, o, stats, nullptr, wdot, qdot, stream);
    if (rc && rc != CHEM_E_CELL_FAILED) return rc;
    // the update writes nothing if a cell had no valid state
    struct {
        const double *U, *p, *u, *c, *wdot, *qdot; long n; double dt, dx; double* Unew;
        unsigned long long* cflmax; const int* bad;
    } ua{U, p, u, c, wdot, qdot, (long)ncell, dt, dx, U_out, flags + 1, bad};
    if (int rc2 = launch_1d(d->f_euler_update, ncell, 256, &ua, sizeof ua, stream, "chem_euler_update")) return rc2;
    // one small readback: the bad flag and the largest CFL number
    unsigned long long h[2] = {0ull, 0ull};
    HIPCHECK(hipMemcpyAsync(h, flags, sizeof h, hipMemcpyDeviceToHost, stream), "flag copy");
    HIPCHECK(hipStreamSynchronize(stream), "flag sync");
    if ((int)(h[0] & 0xffffffffull))
        return set_error(CHEM_E_INVAL, "a cell's conserved state gives no temperature (rho <= 0 or no root)");
    if (max_cfl) {
        double mx;
        std::memcpy(&mx, &h[1], sizeof mx);
        *max_cfl = mx;
    }
    return rc;
}

int run_adjoint(chem_mechanism* m, int64_t ncell, const double* T0, const double* p, const double* Y0,
                double dt, double rtol, double atol, const double* gT, const double* gY, double* gT0,
                double* gY0, double* g_lnA, double* g_b, double* g_Ea, double* T_end, double* Y_end,
                const Options& o, chem_stats* stats, hipStream_t stream)
{
    DeviceState* d;
    if (int rc = device_state(m, stream, &d)) return rc;
    const int ns = m->data.ns(), n = ns + 1, nr = m->data.nr();
    int K = o.checkpoint_every;
    if (K < 0 || K > 16) return set_error(CHEM_E_INVAL, "checkpoint_every must be 1..16");
    if (ncell == 0) {   // parameter gradients are zero; nothing else to do
        struct {
            const double* g;
            long n;
            int np;
            double *a, *b, *e;
        } rp{nullptr, 0, 3 * nr, g_lnA, g_b, g_Ea};
        return launch_1d(d->f_rparams, (int64_t)3 * nr * 256, 256, &rp, sizeof rp, stream, "chem_reduce_params");
    }
    Scratch s(stream);
    double *Tw, *Yw;
    int32_t* i32;
    if (int rc = s.alloc(&Tw, ncell, "adjoint T")) return rc;
    if (int rc = s.alloc(&Yw, (size_t)ncell * ns, "adjoint Y")) return rc;
    if (int rc = s.alloc(&i32, 4 * (size_t)ncell, "adjoint counters")) return rc;
    int32_t *st = i32, *na_fwd = i32 + ncell, *na = i32 + 2 * ncell, *nj = i32 + 3 * ncell;
    // sizing pass: the accepted steps of every cell fix the arena offsets
    HIPCHECK(hipMemcpyAsync(Tw, T0, sizeof(double) * ncell, hipMemcpyDeviceToDevice, stream), "copy T0");
    HIPCHECK(hipMemcpyAsync(Yw, Y0, sizeof(double) * ncell * ns, hipMemcpyDeviceToDevice, stream), "copy Y0");
    const StepArgs step = step_args(dt, rtol, atol, o);
    if (o.adjoint_nacc) {   // the caller's forward already counted the steps
        HIPCHECK(hipMemcpyAsync(na_fwd, o.adjoint_nacc, sizeof(int32_t) * ncell, hipMemcpyDeviceToDevice, stream),
                 "copy the forward's step counts");
    } else if (o.h0) {
        IntegrateArgs ia{d->par, Tw, p, Yw, (long)ncell, o.h0, st, na_fwd, nj, step};
        const int64_t lanes = m->wide ? ncell * m->layout.G : ncell;
        const unsigned shmem = m->wide ? m->layout.lds_bytes() : d->stage_lds(64);
        if (int rc = launch_1d(d->f_plain, lanes, 64, &ia, sizeof ia, stream, "chem_plain", shmem)) return rc;
    } else {   // the persistent form takes the same steps, bitwise, sooner
        FieldView fv{Tw, p, Yw, ncell, st, na_fwd, nj, nullptr, nullptr};
        Options po = o;
        po.form = CHEM_FORM_PERSISTENT;
        if (int rc = run_persistent(m, &fv, 1, dt, rtol, atol, po, nullptr, stream)) return rc;
    }
    std::vector<int32_t> nacc_h(ncell);
    HIPCHECK(hipMemcpyAsync(nacc_h.data(), na_fwd, sizeof(int32_t) * ncell, hipMemcpyDeviceToHost, stream),
             "copy step counts");
    HIPCHECK(hipStreamSynchronize(stream), "sync sizing pass");
    if (K == 0) {
        // the densest checkpoints whose arena fits a quarter of the free device
        // memory: every step stored means no recomputation in the reverse sweep
        size_t freeb = 0, totalb = 0;
        HIPCHECK(hipMemGetInfo(&freeb, &totalb), "device memory info");
        K = 16;
        for (int k : {1, 2, 4, 8, 16}) {
            double bytes = 0.0;
            for (int64_t c = 0; c < ncell; ++c) bytes += (double)((std::max<int32_t>(nacc_h[c], 0) + k - 1) / k);
            if (bytes * n * sizeof(double) <= 0.25 * (double)freeb) {
                K = k;
                break;
            }
        }
    }
    std::vector<long> off(2 * (size_t)ncell);
    long th = 0, tc = 0;
    for (int64_t c = 0; c < ncell; ++c) {
        off[c] = th;
        off[ncell + c] = tc;
        const long k = std::max<int32_t>(nacc_h[c], 0);
        th += k;
        tc += (k + K - 1) / K;
    }
    // cells by descending accepted steps (a counting sort, stable in cell index)
    std::vector<int32_t> order(ncell);
    {
        int32_t mx = 0;
        for (int64_t c = 0; c < ncell; ++c) mx = std::max(mx, std::max<int32_t>(nacc_h[c], 0));
        std::vector<int64_t> start(mx + 2, 0);
        for (int64_t c = 0; c < ncell; ++c) ++start[mx - std::max<int32_t>(nacc_h[c], 0) + 1];
        for (int32_t b = 0; b <= mx; ++b) start[b + 1] += start[b];
        for (int64_t c = 0; c < ncell; ++c) order[start[mx - std::max<int32_t>(nacc_h[c], 0)]++] = (int32_t)c;
    }
    int32_t* order_d;
    if (int rc = s.alloc(&order_d, (size_t)ncell, "adjoint order")) return rc;
    HIPCHECK(hipMemcpyAsync(order_d, order.data(), sizeof(int32_t) * ncell, hipMemcpyHostToDevice, stream),
             "copy order");
    // as many lanes (lane groups) as the device keeps resident; each takes the
    // cells s, s + nslot, ... of the cost order and keeps one row of partial
    // parameter sums, reduced in a fixed order afterwards
    int64_t nslot;
    unsigned ashmem;
    if (m->wide) {
        ashmem = m->layout.adj_lds_bytes();
        const int64_t waves_per_cu = std::max<int64_t>(1, std::min<int64_t>(8, (160 * 1024) / std::max(1u, ashmem)));
        nslot = std::min<int64_t>(ncell, (int64_t)d->num_cu * waves_per_cu * m->layout.cells_per_wave());
    } else {
        // the stage vectors (5 n doubles a lane), and during a step adjoint the
        // 3 nr parameter accumulators when they fit 80 doubles a lane (the
        // device code's kAdjParamsInLds)
        const int words = std::max(d->lane_words(), 3 * nr <= 80 ? 3 * nr : 0);
        ashmem = (unsigned)(64 * words * sizeof(double));
        nslot = std::min<int64_t>(ncell, (int64_t)d->num_cu * 4 * 64);
    }
    // One cell per lane: the most expensive cells (those within a fraction of
    // the largest step count) go to groups of kAdjGroupLanes lanes, which split
    // the six second-order evaluations of each step and so shorten the
    // kernel's critical path; whole waves of groups, at most a quarter of the
    // resident waves, the rest of the lanes one cell each.
    long ngroup = 0, gcells = 0;
    if (!m->wide && ncell > 0) {
        const int64_t cap = (int64_t)d->num_cu * 4 * 64;
        const double frac = adjoint_group_fraction();
        const int32_t top = std::max<int32_t>(nacc_h[order[0]], 0);
        int64_t cand = 0;
        if (frac > 0.0 && top > 0)
            while (cand < ncell && std::max<int32_t>(nacc_h[order[cand]], 0) >= frac * top) ++cand;
        const int64_t per_wave = 64 / kAdjGroupLanes;
        const int64_t gw = std::min<int64_t>((cand + per_wave - 1) / per_wave, cap / 64 / 4);
        if (gw > 0) {
            ngroup = (long)(gw * per_wave);
            gcells = (long)std::min<int64_t>(ncell, ngroup);
            nslot = gw * 64 + std::min<int64_t>(ncell - gcells, cap - gw * 64);
        }
    }
    long* off_d;
    double *hs, *ck, *gpar;
    if (int rc = s.alloc(&off_d, 2 * (size_t)ncell, "adjoint offsets")) return rc;
    if (int rc = s.alloc(&hs, (size_t)th, "adjoint step sizes")) return rc;
    if (int rc = s.alloc(&ck, (size_t)tc * n, "adjoint checkpoints")) return rc;
    if (int rc = s.alloc(&gpar, (size_t)nslot * 3 * nr, "adjoint parameter partial sums")) return rc;
    HIPCHECK(hipMemcpyAsync(off_d, off.data(), sizeof(long) * off.size(), hipMemcpyHostToDevice, stream),
             "copy offsets");
    // one cell per lane with checkpoints K > 1 apart: each lane's stash for
    // the K steps of a segment (see StashLayout), unless it would take more
    // than an eighth of the free device memory or CHEM_ADJOINT_STASH=0
    double* stash = nullptr;
    if (!m->wide && K > 1) {
        const char* e = std::getenv("CHEM_ADJOINT_STASH");
        const size_t words = (size_t)n * n + n + 1 + 6 * (size_t)n;
        const size_t bytes = (size_t)nslot * K * words * sizeof(double);
        size_t freeb = 0, totalb = 0;
        HIPCHECK(hipMemGetInfo(&freeb, &totalb), "device memory info");
        if (!(e && std::atoi(e) == 0) && bytes <= freeb / 8)
            if (int rc = s.alloc(&stash, (size_t)nslot * K * words, "adjoint stash")) return rc;
    }
    // checkpoints at every step: the forward rerun keeps every step's factors
    // and stage vectors (a trail), so the reverse sweep forms none of them
    // again, if that fits an eighth of the free device memory
    double* trail = nullptr;
    if (!m->wide && K == 1) {
        const char* e = std::getenv("CHEM_ADJOINT_STASH");
        const size_t words = (size_t)n * n + n + 1 + 6 * (size_t)n;
        const size_t slots = (size_t)th + (size_t)ncell;
        size_t freeb = 0, totalb = 0;
        HIPCHECK(hipMemGetInfo(&freeb, &totalb), "device memory info");
        if (!(e && std::atoi(e) == 0) && slots * words * sizeof(double) <= freeb / 8)
            if (int rc = s.alloc(&trail, slots * words, "adjoint trail")) return rc;
    }
    AdjointArgs aa{d->par, T0, p, Y0, (long)ncell, gT, gY, gT0, gY0, gpar, (long)nslot, T_end, Y_end, off_d,
                   off_d + ncell, na_fwd, order_d, o.h0, hs, ck, st, na, nj, step, K, ngroup, gcells, stash, trail};
    HIPCHECK(hipEventRecord(d->ev0, stream), "event");
    const int64_t alanes = m->wide ? nslot * m->layout.G : nslot;
    if (int rc = launch_1d(d->f_adjoint, alanes, 64, &aa, sizeof aa, stream, "chem_adjoint", ashmem)) return rc;
    HIPCHECK(hipEventRecord(d->ev1, stream), "event");
    struct {
        const double* g;
        long n;
        int np;
        double *a, *b, *e;
    } rp{gpar, (long)nslot, 3 * nr, g_lnA, g_b, g_Ea};
    if (int rc = launch_1d(d->f_rparams, (int64_t)3 * nr * 256, 256, &rp, sizeof rp, stream,
                           "chem_reduce_params"))
        return rc;
    HIPCHECK(hipEventSynchronize(d->ev1), "event sync");
    float ms = 0.f;
    HIPCHECK(hipEventElapsedTime(&ms, d->ev0, d->ev1), "elapsed");
    chem_stats local{};
    return collect_stats(*d, st, na, nj, ncell, ms, stats ? stats : &local, stream);
}

}  // namespace chemmi
