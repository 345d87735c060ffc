// Fixed device scratch for ffa_syrk_modp_noalloc, the entry point for callers
// that cannot allocate device memory (code under graph capture, serving loops,
// harnesses that forbid hipMalloc).
//
// The scratch is a file-scope device array of FFA_SCRATCH_BYTES: every GPU the
// library runs on holds its own copy from the moment the code object is loaded
// until the process ends.  In host code the name `scratch` only stands for the
// symbol; its device address on a GPU comes from hipGetSymbolAddress, looked up
// once per device (with that device current) when a context is created on it
// and kept here.  Every use on the host goes through that address.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/ffa.h"
#include "ffa_internal.h"

namespace ffa {

static __device__ __align__(256) char scratch[FFA_SCRATCH_BYTES];

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
char* g_base[MAX_DEVICES] = {};  // device address of `scratch` per device (null until looked up)

}  // namespace

int scratch_setup(int device)
{
    if (device < 0 || device >= MAX_DEVICES) return (int)hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_base[device]) return 0;
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return (int)e;
    if (cur != device) return (int)hipErrorInvalidDevice;  // the caller makes the device current
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return (int)e;
    if (!p) return (int)hipErrorInvalidSymbol;
    g_base[device] = (char*)p;
    return 0;
}

char* scratch_base(int device)
{
    if (device < 0 || device >= MAX_DEVICES) return nullptr;
    std::lock_guard<std::mutex> lk(g_mu);
    return g_base[device];
}

}  // namespace ffa
