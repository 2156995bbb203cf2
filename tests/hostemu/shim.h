// shim.h -- host (x86-64) stand-ins for the HIP device builtins that the
// library's generated device source uses, so that source can be compiled as
// plain C++ and run one lane at a time under the host sanitizers (address,
// undefined behaviour, memory) and with trivial-auto-var-init patterns.
//
// Semantics: a "wave" of one lane.  Cross-lane votes reduce to the lane's own
// predicate, shuffles return the lane's own value, atomics are plain
// read-modify-writes, barriers do nothing.  Launch geometry is a set of
// globals that the driver sets before calling a kernel function.  Test
// infrastructure only: nothing in the library includes this file.
#pragma once
#include <math.h>
#include <stdint.h>

#define __device__
#define __host__
#define __forceinline__ inline
#define __noinline__ __attribute__((noinline))
#define __global__
#define __constant__
#define __shared__ static
#define __launch_bounds__(...)
#define __restrict__

struct emu_dim3 { unsigned x, y, z; };
extern emu_dim3 threadIdx, blockIdx, blockDim, gridDim;
extern double* emu_lds;   // dynamic LDS of the current "workgroup"

static inline bool __any(bool p) { return p; }
static inline bool __all(bool p) { return p; }
static inline unsigned long long __ballot(bool p) { return p ? 1ull : 0ull; }
static inline int __popcll(unsigned long long x) { return __builtin_popcountll(x); }
static inline int __ffsll(long long x) { return __builtin_ffsll(x); }
template <class T> static inline T __shfl(T v, int) { return v; }
// lanes run one at a time here, so nothing across lanes can be emulated; the
// grouped adjoint (the only user) is never launched by the driver
template <class T> static inline T __shfl_xor(T, int, int) { __builtin_trap(); }
template <class T, class U> static inline T atomicAdd(T* p, U v) { T o = *p; *p = (T)(o + (T)v); return o; }
template <class T, class U> static inline T atomicMax(T* p, U v) { T o = *p; if ((T)v > o) *p = (T)v; return o; }
static inline void __syncthreads() {}
// the hardware's double-to-int conversion: saturating, NaN to 0
static inline int emu_cvt_i32_sat(double x)
{
    if (x != x) return 0;
    if (x >= 2147483647.0) return 2147483647;
    if (x <= -2147483648.0) return -2147483647 - 1;
    return (int)x;
}
static inline long long __double_as_longlong(double x) { long long b; __builtin_memcpy(&b, &x, sizeof b); return b; }
static inline double __longlong_as_double(long long b) { double x; __builtin_memcpy(&x, &b, sizeof x); return x; }
template <class T> static inline T min(T a, T b) { return b < a ? b : a; }
template <class T> static inline T max(T a, T b) { return a < b ? b : a; }
static inline long min(long a, int b) { return b < a ? b : a; }
static inline long max(long a, int b) { return a < b ? b : a; }
