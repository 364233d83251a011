// pfc_energy_static: the discrete energy and mass of pfc_energy without a
// handle and without allocating.  The per-block partial sums that pfc_energy
// keeps in a buffer of its handle live here in a file-scope device array,
// `scratch`, that every call on a device shares.
//
// The array's name is only a host-side stand-in for the device symbol: host
// code never passes it to a kernel.  The first call on a device, with that
// device current, asks the runtime for the array's device address
// (hipGetSymbolAddress) and keeps it per device; kernels receive that
// address.
#include "pfc.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>
#include <string>

#include "pfc_internal.h"
#include "runtime_internal.h"

namespace {

// k_energy_part leaves 6 sums per workgroup and launches at most
// kMaxReduceBlocks workgroups, whatever n is.
constexpr size_t kScratchDoubles = (size_t)pfc::kMaxReduceBlocks * 6;
constexpr int kMaxDevices = 64;

__device__ __align__(256) double scratch[kScratchDoubles];

std::mutex g_mutex;
double *g_scratch[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up once per
// device); nullptr and a message on failure.
double *scratch_on_current_device(std::string &why) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        why = std::string("hipGetDevice: ") + hipGetErrorString(e);
        return nullptr;
    }
    if (dev < 0 || dev >= kMaxDevices) {
        why = "device ordinal " + std::to_string(dev) + " out of range";
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(g_mutex);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            why = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
            return nullptr;
        }
        g_scratch[dev] = static_cast<double *>(p);
    }
    return g_scratch[dev];
}

}  // namespace

extern "C" pfc_status pfc_energy_static(int32_t n, double L, double eps, const double *phi,
                                        const double *phi_prev, double *out3, void *stream) {
    using namespace pfc;
    if (n < 4 || n > PFC_ENERGY_STATIC_MAX_N)
        return fail(nullptr, PFC_ERR_INVALID_ARG,
                    "pfc_energy_static: n must be in [4, " +
                        std::to_string(PFC_ENERGY_STATIC_MAX_N) + "], got " + std::to_string(n));
    if (!(L > 0) || !std::isfinite(L) || !std::isfinite(eps))
        return fail(nullptr, PFC_ERR_INVALID_ARG, "pfc_energy_static: L must be > 0, eps finite");
    if (!phi || !out3) return fail(nullptr, PFC_ERR_INVALID_ARG, "pfc_energy_static: NULL pointer");
    if ((size_t)energy_blocks(n) * 6 > kScratchDoubles)
        return fail(nullptr, PFC_ERR_INVALID_ARG, "pfc_energy_static: scratch too small");
    std::string why;
    double *part = scratch_on_current_device(why);
    if (!part) return fail(nullptr, PFC_ERR_HIP, "pfc_energy_static: " + why);
    const double h = L / n;
    // Every partial that k_energy_final reads is written first by
    // k_energy_part in the same call: nothing needs clearing.
    launch_energy(static_cast<hipStream_t>(stream), make_lay(n, false), h, eps, phi, phi_prev, part,
                  out3);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return fail(nullptr, PFC_ERR_HIP, std::string("pfc_energy_static: ") + hipGetErrorString(e));
    return PFC_OK;
}
