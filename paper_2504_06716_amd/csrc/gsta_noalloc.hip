// gsta_l1_loss_noalloc: the L1 loss of gsta_l1_loss for callers that cannot
// allocate device memory (code under HIP graph capture, tight serving loops,
// harnesses that forbid allocation).  It needs no context: the first pass's
// per-workgroup partial sums live in a file-scope device array instead of a
// context's scratch.  Same kernels, same fixed summation order, so its
// results equal gsta_l1_loss's bit for bit.
#include "../../include/gsta.h"
#include "gsta_internal.h"

#include <cstdio>
#include <mutex>

namespace {

// One double2 partial (sum |d|, sum of squared clamped errors) per workgroup
// of the first pass; the launch never uses more than kL1Blocks workgroups.
// Each GPU the library runs on holds its own copy until the process ends.
__device__ __align__(256) double2 scratch[gsta::kL1Blocks];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
double2* g_scratch[kMaxDevices] = {};   // device address of `scratch`, per device

// The device address of `scratch` on the current device, looked up once per
// device (with that device current).  Host code passes only this address to
// kernels: the array's name is a host-side stand-in, not a device address.
gsta_status scratch_on_current_device(double2** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        gsta::set_noctx_error("hipGetDevice: %s", hipGetErrorString(e));
        return GSTA_ERR_HIP;
    }
    if (dev < 0 || dev >= kMaxDevices) {
        gsta::set_noctx_error("device %d beyond the %d devices gsta_l1_loss_noalloc supports", dev, kMaxDevices);
        return GSTA_ERR_INVALID;
    }
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            gsta::set_noctx_error("hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
            return GSTA_ERR_HIP;
        }
        g_scratch[dev] = static_cast<double2*>(p);
    }
    *out = g_scratch[dev];
    return GSTA_OK;
}

}  // namespace

extern "C" gsta_status gsta_l1_loss_noalloc(const float* image, const float* target, int64_t count,
                                            float* dL_dimage, double* sums, hipStream_t stream) {
    if (count < 1 || count > GSTA_L1_NOALLOC_MAX_COUNT) {
        gsta::set_noctx_error("gsta_l1_loss_noalloc: count = %lld outside [1, %lld]", (long long)count,
                              (long long)GSTA_L1_NOALLOC_MAX_COUNT);
        return GSTA_ERR_INVALID;
    }
    if (!image || !target || !dL_dimage || !sums) {
        gsta::set_noctx_error("gsta_l1_loss_noalloc: NULL pointer argument");
        return GSTA_ERR_INVALID;
    }
    double2* part = nullptr;
    const gsta_status st = scratch_on_current_device(&part);
    if (st != GSTA_OK) return st;
    // every partial the second pass reads is written by this call's first
    // pass, so nothing in the scratch needs clearing
    gsta::launch_l1(image, target, count, dL_dimage, sums, part, stream);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        gsta::set_noctx_error("gsta_l1_loss_noalloc launch: %s", hipGetErrorString(e));
        return GSTA_ERR_HIP;
    }
    return GSTA_OK;
}
