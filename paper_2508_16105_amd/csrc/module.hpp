// module.hpp -- building and loading the device code of a mechanism.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

namespace chemmi {

// Full device source for a mechanism: the generated mechanism code followed by
// the hand-written integrator and kernels (one cell per lane, or with `wide`
// the wave-cooperative form).
// The complete device source of a mechanism: the math, the generated
// mechanism code, the shared and form-specific kernels.  exp_saturating picks
// how exp_poly converts its exponent to int (see math.hip).
std::string device_source(const std::string& mechanism_code, bool wide, bool exp_saturating);

// Compile options used for every device build (gfx950, FP64, contraction of
// a*b+c into FMA only within an expression, no packed-FP32 instructions).
const std::vector<std::string>& compile_options();

// Code object for `source`, from the on-disk cache or compiled with hipRTC
// (and then stored).  Returns 0 or a chem error code with err set.
int build_code_object(const std::string& source, std::vector<char>& code, std::string& err,
                      std::string* cache_file = nullptr);

// hipRTC/HIP versions and the loaded hipRTC and comgr libraries (path with
// version suffix, size, mtime): part of every code-object cache key.
const std::string& compiler_identity();

// Directory of the kernel cache.
std::string cache_dir();

uint64_t fnv1a(const std::string& s, uint64_t h = 1469598103934665603ull);

}  // namespace chemmi
