// Static device workspace of the allocation-free product (procmv_apply_noalloc).
//
// The partial slots of a product live in a file-scope device array that the
// code object carries, so a caller that cannot allocate device memory (code
// under stream capture, tight serving loops) still gets a product.  Each
// device holds its own copy of the array for the life of the process; its
// address is looked up once per device with hipGetSymbolAddress and that
// pointer, never the array's name, is what host code hands to kernels.
#include <mutex>

#include "kernels.h"

namespace procmv {

constexpr size_t kStaticWorkspaceBytes = size_t(64) << 20;   // 64 MiB per device
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kStaticWorkspaceBytes];

static std::mutex g_mu;
static void* g_ptr[kMaxDevices] = {};

size_t static_workspace_bytes() { return kStaticWorkspaceBytes; }

hipError_t static_workspace(void** ptr, size_t* bytes)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_mu);
    if (g_ptr[dev] == nullptr) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_ptr[dev] = p;
    }
    *ptr = g_ptr[dev];
    *bytes = kStaticWorkspaceBytes;
    return hipSuccess;
}

}  // namespace procmv
