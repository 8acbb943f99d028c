// Static device scratch of the entry points that allocate nothing: a
// file-scope device array (one copy per GPU, held until the process ends)
// whose device address is looked up once per device at context set-up and
// kept per device. Host code never hands the array's own name to a kernel
// or a copy (in host code that name is a host-side stand-in, not a device
// address); it uses the looked-up address only.
#include <hip/hip_runtime.h>

#include <mutex>

#include "noalloc.hpp"

namespace fepa {

static __device__ __align__(256) double scratch[kStaticScratchDoubles];

namespace {
std::mutex g_mu;
double *g_ptr[kStaticScratchDevices] = {};
}  // namespace

int static_scratch_init(int device)
{
    if (device < 0 || device >= kStaticScratchDevices) return -1;
    std::lock_guard<std::mutex> lock(g_mu);
    if (g_ptr[device]) return 0;
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess || cur != device) return -1;
    void *p = nullptr;
    const hipError_t rc = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (rc != hipSuccess || !p) {
        (void)hipGetLastError();
        return -1;
    }
    g_ptr[device] = static_cast<double *>(p);
    return 0;
}

double *static_scratch(int device)
{
    if (device < 0 || device >= kStaticScratchDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_mu);
    return g_ptr[device];
}

}  // namespace fepa
