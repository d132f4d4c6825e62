// dgfs_collide_static: the collide of dgfs_collide with a workspace the library owns, for
// callers that cannot allocate device memory (code under HIP graph capture, serving loops
// that must not call hipMalloc, harnesses that forbid it).
//
// The workspace is a file-scope device array of fixed size.  Each GPU the library runs
// on holds its own copy until the process ends; in host code the array's name is only a
// stand-in, so its device address is looked up once per device (hipGetSymbolAddress, with
// that device current) and only that address is ever handed to kernels.  Every call on a
// device shares the array: the collide kernels write every workspace value they read, so
// nothing needs clearing between calls, but two calls that overlap on one device (other
// streams, other threads) race on it.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "dgfs.h"
#include "plan.hpp"

namespace {

constexpr size_t kScratchBytes = size_t(256) << 20;   // 256 MiB per device
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on device `dev` (the current device), looked up on the
// first call for that device.
dgfs_status scratch_address(int dev, void** out) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || ptr == nullptr)
            return dgfs::set_error(DGFS_EDEVICE, std::string("hipGetSymbolAddress of the static workspace failed: ") +
                                                     hipGetErrorString(e));
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return DGFS_OK;
}

}  // namespace

extern "C" {

size_t dgfs_static_workspace_bytes(void) { return kScratchBytes; }

dgfs_status dgfs_collide_static(const dgfs_plan* plan, const void* f, void* Q, int64_t batch, void* stream) {
    if (!plan) return dgfs::set_error(DGFS_EINVAL, "plan is NULL");
    if (batch < 0) return dgfs::set_error(DGFS_EINVAL, "batch must be >= 0");
    if (batch == 0) return DGFS_OK;
    if (!f || !Q) return dgfs::set_error(DGFS_EINVAL, "f and Q are required");
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return dgfs::set_error(DGFS_EDEVICE, "no HIP device");
    if (dev != plan->device)
        return dgfs::set_error(DGFS_EINVAL, "the plan's device must be the current device");
    if (dev < 0 || dev >= kMaxDevices) return dgfs::set_error(DGFS_EUNSUPPORTED, "device index beyond 63");
    const size_t one = plan->ws_per_node(false) + plan->ws_slack();
    if (one > kScratchBytes)
        return dgfs::set_error(DGFS_ENOMEM, "one node of this plan needs " + std::to_string(one) +
                                                " bytes of workspace, more than the static workspace of " +
                                                std::to_string(kScratchBytes) + " bytes");
    void* ptr = nullptr;
    const dgfs_status st = scratch_address(dev, &ptr);
    if (st != DGFS_OK) return st;
    return dgfs::collide_with_workspace(plan, f, Q, batch, ptr, kScratchBytes, stream);
}

}  // extern "C"
