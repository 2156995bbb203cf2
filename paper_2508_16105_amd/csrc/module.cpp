// module.cpp -- hipRTC compilation with an on-disk code-object cache.
#include "module.hpp"

#include <dlfcn.h>
#include <hip/hip_runtime.h>
#include <hip/hiprtc.h>
#include <link.h>
#include <sys/stat.h>
#include <utime.h>
#include <unistd.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <sstream>

#include "../../include/chem.h"

namespace chemmi {

#include "_device_source.inc"   // kMathSource, kCommonSource, kIntegratorSource, kWideSource, kEulerSource

std::string device_source(const std::string& mechanism_code, bool wide, bool exp_saturating)
{
    const std::string config = std::string("namespace chem_config {\nconstexpr bool kExpSaturatingConvert = ") +
                               (exp_saturating ? "true" : "false") + ";\n}\n";
    return config + std::string(kMathSource) + "\n" + mechanism_code + "\n" + std::string(kCommonSource) + "\n" +
           std::string(wide ? kWideSource : kIntegratorSource) + "\n" + std::string(kEulerSource);
}

const std::vector<std::string>& compile_options()
{
    static const std::vector<std::string> opts = {
        "--offload-arch=gfx950", "-O3", "-std=c++17", "-ffp-contract=on",
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"};
    return opts;
}

uint64_t fnv1a(const std::string& s, uint64_t h)
{
    for (unsigned char c : s) {
        h ^= c;
        h *= 1099511628211ull;
    }
    return h;
}

std::string cache_dir()
{
    if (const char* env = std::getenv("CHEM_KERNEL_CACHE")) return env;
    Dl_info info;
    if (dladdr((void*)&cache_dir, &info) && info.dli_fname) {
        std::string p(info.dli_fname);
        auto slash = p.rfind('/');
        if (slash != std::string::npos) return p.substr(0, slash) + "/kcache";
    }
    return "kcache";
}

namespace {

// The path (with its full version suffix), size and modification time of a
// loaded shared library whose file name contains `part`, or "" if none is.
std::string loaded_library(const char* part)
{
    struct Q {
        const char* part;
        std::string found;
    } q{part, {}};
    dl_iterate_phdr(
        [](struct dl_phdr_info* info, size_t, void* data) -> int {
            auto* qq = static_cast<Q*>(data);
            if (info->dlpi_name && std::strstr(info->dlpi_name, qq->part)) {
                char real[4096];
                const char* path = realpath(info->dlpi_name, real) ? real : info->dlpi_name;
                struct stat st{};
                std::ostringstream o;
                o << path;
                if (stat(path, &st) == 0) o << " size " << st.st_size << " mtime " << st.st_mtime;
                qq->found = o.str();
                return 1;
            }
            return 0;
        },
        &q);
    return q.found;
}

}  // namespace

// Everything that decides the machine code hipRTC makes from a source: the
// hipRTC and HIP runtime versions and the exact hipRTC and code-object
// compiler (comgr) libraries this process loaded.  Part of every cache key,
// so a host with another compiler build compiles afresh instead of running
// code objects another compiler made.
const std::string& compiler_identity()
{
    static const std::string id = [] {
        int vmaj = 0, vmin = 0, rt = 0;
        hiprtcVersion(&vmaj, &vmin);
        (void)hipRuntimeGetVersion(&rt);
        // hipRTC loads comgr on first use; load it now (it is the library hipRTC
        // itself loads) so its identity is known before the first compile
        if (!dlopen("libamd_comgr.so.3", RTLD_LAZY | RTLD_NOLOAD)) (void)dlopen("libamd_comgr.so.3", RTLD_LAZY);
        std::ostringstream o;
        o << "hiprtc " << vmaj << "." << vmin << "; hip runtime " << rt << "; " << loaded_library("libhiprtc.so")
          << "; " << loaded_library("libamd_comgr.so");
        return o.str();
    }();
    return id;
}

namespace {

bool read_file(const std::string& path, std::vector<char>& out)
{
    std::ifstream in(path, std::ios::binary);
    if (!in) return false;
    out.assign(std::istreambuf_iterator<char>(in), std::istreambuf_iterator<char>());
    return !out.empty();
}

void write_file_atomic(const std::string& path, const std::vector<char>& data)
{
    std::string tmp = path + ".tmp" + std::to_string(getpid());
    {
        std::ofstream out(tmp, std::ios::binary);
        if (!out) return;
        out.write(data.data(), (std::streamsize)data.size());
        if (!out) return;
    }
    std::rename(tmp.c_str(), path.c_str());
}

}  // namespace

int build_code_object(const std::string& source, std::vector<char>& code, std::string& err,
                      std::string* cache_file)
{
    std::string key_text = source;
    for (auto& o : compile_options()) key_text += "\n" + o;
    key_text += "\n" + compiler_identity();
    if (std::getenv("CHEM_LOG")) std::fprintf(stderr, "[chem] compiler: %s\n", compiler_identity().c_str());
    char name[40];
    std::snprintf(name, sizeof name, "%016llx.co", (unsigned long long)fnv1a(key_text));
    const std::string dir = cache_dir();
    const std::string path = dir + "/" + name;
    if (cache_file) *cache_file = path;
    if (const char* dump = std::getenv("CHEM_DUMP_SOURCE")) {   // for offline inspection
        std::ofstream out(dump);
        out << source;
    }
    if (read_file(path, code)) {
        utime(path.c_str(), nullptr);   // mark as in use (stale entries are pruned by the build)
        return 0;
    }

    hiprtcProgram prog;
    if (hiprtcCreateProgram(&prog, source.c_str(), "chem_mechanism.hip", 0, nullptr, nullptr) !=
        HIPRTC_SUCCESS) {
        err = "hiprtcCreateProgram failed";
        return CHEM_E_COMPILE;
    }
    std::vector<const char*> opts;
    for (auto& o : compile_options()) opts.push_back(o.c_str());
    hiprtcResult rc = hiprtcCompileProgram(prog, (int)opts.size(), opts.data());
    if (rc != HIPRTC_SUCCESS) {
        size_t n = 0;
        hiprtcGetProgramLogSize(prog, &n);
        std::string log(n, '\0');
        if (n) hiprtcGetProgramLog(prog, &log[0]);
        err = "device compilation failed: " + log.substr(0, 4000);
        hiprtcDestroyProgram(&prog);
        return CHEM_E_COMPILE;
    }
    size_t n = 0;
    hiprtcGetCodeSize(prog, &n);
    code.resize(n);
    hiprtcGetCode(prog, code.data());
    hiprtcDestroyProgram(&prog);
    mkdir(dir.c_str(), 0755);
    write_file_atomic(path, code);
    return 0;
}

}  // namespace chemmi
