// Allocation-free energy readout: the variant of wdg_energy for callers that cannot allocate device
// memory (HIP graph capture, tight serving loops).  Its per-block partial sums live in a file-scope
// device array instead of the context's scratch buffer; the energy kernels are the same.
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>
#include <string>

#include "context.hpp"

namespace wdg {
namespace {

// Per-block partial energies of one call.  Each GPU the library runs on holds its own copy until the
// process ends; every call on that GPU shares it.
constexpr size_t kScratchBytes = static_cast<size_t>(WDG_NOALLOC_MAX_BLOCKS) * sizeof(double);
__device__ __align__(256) double scratch[WDG_NOALLOC_MAX_BLOCKS];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};  // device address of `scratch` on each device (null: not looked up yet)

}  // namespace

// Looks up the device address of the scratch array on `device` (current) once; 0 on success.
int noalloc_setup(int device) {
    if (device < 0 || device >= kMaxDevices) return static_cast<int>(hipErrorInvalidDevice);
    std::lock_guard<std::mutex> lock(g_mu);
    if (g_ptr[device]) return 0;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return static_cast<int>(e);
    g_ptr[device] = p;
    return 0;
}

}  // namespace wdg

extern "C" int32_t wdg_energy_noalloc(wdg_ctx* c, double* out_device, void* hip_stream) {
    using namespace wdg;
    if (!c || !out_device) return WDG_EINVAL;
    if (int e = check_state(c)) return e;
    if (c->S.nblk > WDG_NOALLOC_MAX_BLOCKS)
        return fail(c, WDG_EINVAL, "mesh too large for the allocation-free energy: " + std::to_string(c->S.nblk) +
                                       " element blocks, at most " + std::to_string(WDG_NOALLOC_MAX_BLOCKS));
    void* ptr = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_mu);
        if (c->device >= 0 && c->device < kMaxDevices) ptr = g_ptr[c->device];
    }
    if (!ptr) return fail(c, WDG_ESTATE, "scratch address of this device not set up (context created without a device)");
    static_assert(kScratchBytes == sizeof(scratch), "scratch size");
    EnergyParams p{};
    p.q = c->q[c->cur];
    p.J = static_cast<const double*>(c->Jk.p);
    p.M = static_cast<const double*>(c->Mref.p);
    p.partial = static_cast<double*>(ptr);  // every partial is written before the sum reads it
    p.nblk = c->S.nblk;
    const int e = launch_energy(c->precision, c->S.ref.N, p, out_device, static_cast<hipStream_t>(hip_stream));
    if (e != 0) return fail(c, WDG_EHIP, std::string("energy launch: ") + hipGetErrorString(static_cast<hipError_t>(e)));
    return WDG_OK;
}
