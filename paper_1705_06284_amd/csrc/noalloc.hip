// noalloc.hip -- the library's static device scratch, for callers that cannot
// allocate device memory (code under HIP graph capture, tight serving loops,
// harnesses that forbid hipMalloc).
//
// `scratch` is a file-scope device array; every GPU the library runs on holds
// its own copy, at its own address, until the process ends.  Host code never
// uses the array's name as memory: scratch_address() looks the device address
// up once per device (with that device current) and hands it out from then on.
#include <hip/hip_runtime.h>

#include <mutex>

#include "noalloc.hpp"

static __device__ __align__(256) unsigned char scratch[bispec::kScratchBytes];

namespace bispec {

namespace {
std::mutex g_mu;
void *g_addr[kScratchMaxDevices] = {};
unsigned long long g_owner[kScratchMaxDevices] = {};
}  // namespace

hipError_t scratch_address(int device, void **addr) {
    if (device < 0 || device >= kScratchMaxDevices || !addr) return hipErrorInvalidValue;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_addr[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_addr[device] = p;
    }
    *addr = g_addr[device];
    return hipSuccess;
}

bool scratch_claim(int device, unsigned long long owner) {
    std::lock_guard<std::mutex> lk(g_mu);
    const bool same = g_owner[device] == owner;
    g_owner[device] = owner;
    return same;
}

void scratch_release(int device) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_owner[device] = 0;
}

}  // namespace bispec
