// Entry point for callers that cannot allocate device memory (code under
// HIP graph capture, serving loops, harnesses that forbid hipMalloc): the
// dipole of me_dipole, d = h^3 sum_i (h*ix_i - L/2) rho_i, of a caller's
// density, with the per-workgroup partial sums in a fixed device array of
// this file instead of a system's workspace.  Same kernels, same fixed
// summation order as me_dipole.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <string>

#include "../../include/modehr.h"
#include "adjoint.hpp"

// Partial sums of me_dipole_noalloc.  Each GPU the library runs on holds its
// own copy until the process ends.  Host code reaches it only through the
// address hipGetSymbolAddress returns with that device current (the name is
// a host-side stand-in, not a device address).
static __device__ __align__(256) double scratch[ME_NOALLOC_MAX_PARTS];

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
double* g_scratch[MAX_DEVICES] = {};    // per device: address of `scratch`, null until taken

// address of `scratch` on the current device (taken once per device)
me_status scratch_address(double** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        me::set_thread_error(std::string("hipGetDevice: ") + hipGetErrorString(e));
        return ME_EDEVICE;
    }
    if (dev < 0 || dev >= MAX_DEVICES) {
        me::set_thread_error("device ordinal beyond the library's table of scratch addresses");
        return ME_EDEVICE;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch[dev] == nullptr) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || p == nullptr) {
            me::set_thread_error(std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
            return ME_EDEVICE;
        }
        g_scratch[dev] = static_cast<double*>(p);
    }
    *out = g_scratch[dev];
    return ME_OK;
}

}  // namespace

extern "C" me_status me_dipole_noalloc(const double* rho_dev, const int32_t n[3], double h, double* d_dev,
                                       void* stream) {
    if (!rho_dev || !n || !d_dev) {
        me::set_thread_error("rho_dev, n and d_dev must not be NULL");
        return ME_EINVAL;
    }
    if (n[0] < 1 || n[1] < 1 || n[2] < 1 || !(h > 0.0)) {
        me::set_thread_error("grid sizes must be >= 1 and h > 0");
        return ME_EINVAL;
    }
    const int64_t N = (int64_t)n[0] * n[1] * n[2];
    const int64_t parts = (N + 255) / 256;
    if (parts > ME_NOALLOC_MAX_PARTS) {
        me::set_thread_error("grid too large for the fixed scratch: at most 256 * ME_NOALLOC_MAX_PARTS points");
        return ME_EINVAL;
    }
    double* part = nullptr;
    const me_status st = scratch_address(&part);
    if (st != ME_OK) return st;
    const double h3 = h * h * h;
    // every partial slot [0, parts) is written before it is read: nothing to clear
    const hipError_t e = me::launch_field_dot(rho_dev, n[0], N, h, n[0] * h, part, d_dev, h3,
                                              static_cast<hipStream_t>(stream));
    if (e != hipSuccess) {
        me::set_thread_error(std::string("launch: ") + hipGetErrorString(e));
        return ME_EDEVICE;
    }
    return ME_OK;
}
