// Energy evaluation for callers that cannot allocate device memory (code under
// HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
// the same program and kernels as sv_qaoa_energy, with the reduction partials
// and the phase tables in one fixed device array instead of the state's work
// buffers, and the three results written to a device array of the caller.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>

#include "sv_internal.h"

namespace {
// Reduction partials: 3 slots (norm, energy, p_gs) per tile of the largest
// tile group, 2^20 tiles at n = 33 complex128 and n = 34 complex64 (24 MiB),
// and the first stage of the slot reduction (256 x 8 doubles).
constexpr size_t kPartDoubles = (size_t(3) << 20) + 2048;
// Phase tables, double2 entries (8 MiB): per layer 32 register phases plus the
// 2L + 1 entries of an integer-energy table.
constexpr size_t kTabEntries = size_t(1) << 19;
constexpr int kMaxDevices = 64;
}  // namespace

// One copy per device, kept until the process ends.  Host code never passes
// this name to a kernel: it takes the device address from hipGetSymbolAddress.
static __device__ __align__(256) double scratch[kPartDoubles + 2 * kTabEntries];

static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices];  // device address of `scratch`, per device

// Device address of the array on device dev (looked up once per device, with
// dev current).
static int scratch_ptr(int dev, void** out) {
    if (dev < 0 || dev >= kMaxDevices)
        return sv_internal_set_error(SV_ERR_UNSUPPORTED, "sv_qaoa_energy_noalloc: device index out of range");
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || ptr == nullptr)
            return sv_internal_set_error(SV_ERR_HIP, "sv_qaoa_energy_noalloc: hipGetSymbolAddress(scratch) failed");
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return SV_OK;
}

extern "C" int sv_qaoa_energy_noalloc(sv_state s, sv_ising H, int p, const double* gamma, const double* beta,
                                      int from_plus, double* d_out) {
    if (d_out == nullptr || (reinterpret_cast<uintptr_t>(d_out) & 7u) != 0)
        return sv_internal_set_error(SV_ERR_ARG, "sv_qaoa_energy_noalloc: d_out is NULL or not 8-byte aligned");
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess)
        return sv_internal_set_error(SV_ERR_HIP, "sv_qaoa_energy_noalloc: hipGetDevice failed");
    void* base = nullptr;
    const int rc = scratch_ptr(dev, &base);
    if (rc) return rc;
    svk::FixedScratch fx;
    fx.part = static_cast<double*>(base);
    fx.part_doubles = kPartDoubles;
    fx.tab = reinterpret_cast<double2*>(static_cast<double*>(base) + kPartDoubles);
    fx.tab_entries = kTabEntries;
    fx.out = d_out;
    return sv_internal_qaoa_energy_fixed(s, H, p, gamma, beta, from_plus, dev, fx);
}
