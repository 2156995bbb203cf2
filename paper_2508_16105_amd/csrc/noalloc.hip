// noalloc.hip -- the fixed scratch memory of chem_integrate_noalloc and the
// small kernel that writes its field table.
//
// The scratch is a file-scope device array in the library's own code object,
// so each GPU the library runs on holds one copy (about 36 MB) from the set-up
// of its first mechanism there until the process ends.  Host code never uses
// the array's name as an address: noalloc_scratch() asks the runtime for the
// device address of this device's copy (hipGetSymbolAddress, with the device
// current) once per device and keeps it.
#include <hip/hip_runtime.h>

#include <mutex>

#include "runtime.hpp"

namespace chemmi {

static __device__ __align__(256) unsigned char scratch[kNoallocBytes];

namespace {
std::mutex g_mu;
void* g_addr[kNoallocMaxDevices] = {};
}  // namespace

int noalloc_scratch(int device, void** out)
{
    *out = nullptr;
    if (device < 0 || device >= kNoallocMaxDevices)
        return set_error(CHEM_E_UNSUPPORTED, "device index beyond the allocation-free scratch table");
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_addr[device]) {
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e == hipSuccess && cur != device) e = hipErrorInvalidDevice;   // the caller makes it current
        void* p = nullptr;
        if (e == hipSuccess) e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_error(e, "hipGetSymbolAddress(scratch)");
        g_addr[device] = p;
    }
    *out = g_addr[device];
    return 0;
}

// The field table of one field (header, then its FieldDesc), written on the
// stream by a kernel so the call needs no host-to-device copy.
__global__ void __launch_bounds__(64) chem_noalloc_write_block(PersistHeader h, FieldDesc f, char* dst)
{
    if (threadIdx.x == 0) {
        *reinterpret_cast<PersistHeader*>(dst) = h;
        *reinterpret_cast<FieldDesc*>(dst + sizeof(PersistHeader)) = f;
    }
}

int noalloc_write_block(char* dst, const PersistHeader& h, const FieldDesc& f, hipStream_t stream)
{
    hipLaunchKernelGGL(chem_noalloc_write_block, dim3(1), dim3(64), 0, stream, h, f, dst);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_error(e, "chem_noalloc_write_block");
    return 0;
}

}  // namespace chemmi
