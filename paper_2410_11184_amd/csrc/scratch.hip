// Fixed device scratch of the allocation-free entry point
// (hs_mult_relin_noalloc): one array per device, held from the first load of
// this code object on that device until the process ends.  Host code never
// passes the array's name to a kernel: in host code it names a host-side
// stand-in.  Its device address is looked up once per device, with that
// device current, and that address is what the library hands to kernels.
#include <hip/hip_runtime.h>

#include <mutex>

#include "dev.h"

namespace hs {

static __device__ __align__(256) u64 scratch[kScratchBytes / sizeof(u64)];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_addr[kMaxDevices] = {};
int g_state[kMaxDevices] = {};   // 0 not looked up, 1 found, -1 lookup failed
}  // namespace

// Called by context creation with `device` current.
int scratch_init(int device) {
    if (device < 0 || device >= kMaxDevices) return -1;
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_state[device] != 0) return g_state[device];
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
        (void)hipGetLastError();
        g_state[device] = -1;
        return -1;
    }
    g_addr[device] = p;
    g_state[device] = 1;
    return 1;
}

void* scratch_device_ptr(int device) {
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_mu);
    return g_state[device] == 1 ? g_addr[device] : nullptr;
}

}  // namespace hs
