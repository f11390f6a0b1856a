// noalloc.hip -- afs_eval_noalloc: the evaluation of afs_eval with a static
// device scratch array in place of the caller's workspace, for callers that
// cannot allocate device memory (code under graph capture, tight serving loops).
//
// The array lives in this file; each device that loads the library holds its own
// copy until the process ends.  Host code never passes the array's name to a
// kernel (on the host it names a stand-in, not device memory): the address on
// each device is looked up once, with that device current, and that pointer is
// what the kernels receive.

#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "afsat.h"
#include "instance.hpp"

namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;     // AFS_NOALLOC_SCRATCH_BYTES
static_assert(kScratchBytes == AFS_NOALLOC_SCRATCH_BYTES, "header and library disagree");
constexpr int kMaxDevices = 64;

}  // namespace

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

std::mutex g_mu;
void *g_scratch[kMaxDevices];          // the array's device address per device (null: not looked up)

// Device address of `scratch` on `device`, looked up on first use with that
// device current (the caller's current device is restored).
afs_status scratch_on(int device, void **out)
{
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_scratch[device]) {
        int prev = -1;
        hipError_t e = hipGetDevice(&prev);
        if (e == hipSuccess && prev != device) e = hipSetDevice(device);
        void *p = nullptr;
        if (e == hipSuccess) e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (prev >= 0 && prev != device) (void)hipSetDevice(prev);
        if (e != hipSuccess || !p)
            return afs::set_last_error(AFS_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") +
                                                        hipGetErrorString(e));
        g_scratch[device] = p;
    }
    *out = g_scratch[device];
    return AFS_OK;
}

}  // namespace

extern "C" afs_status afs_eval_noalloc(afs_instance *inst, int32_t B, const float *x, float *obj, float *grad,
                                       float *fe, float *adj, void *stream)
{
    if (!inst) return afs::set_last_error(AFS_EINVAL, "instance is NULL");
    if (inst->device < 0) return afs::set_last_error(AFS_ESTATE, "instance was created host-only (device -1)");
    if (inst->device >= kMaxDevices) return afs::set_last_error(AFS_EINVAL, "device ordinal above 63");
    if (B < 0) return afs::set_last_error(AFS_EINVAL, "B must be >= 0");
    const size_t need = afs::eval_scratch_bytes(inst, B);
    if (need > kScratchBytes)
        return afs::set_last_error(AFS_EINVAL, "afs_eval_noalloc: this instance needs " + std::to_string(need) +
                                                   " bytes of scratch at B = " + std::to_string(B) +
                                                   "; the static scratch holds " + std::to_string(kScratchBytes) +
                                                   " (use afs_eval with a workspace)");
    void *p = nullptr;
    const afs_status st = scratch_on(inst->device, &p);
    if (st != AFS_OK) return st;
    return afs::eval_in_scratch(inst, B, x, p, kScratchBytes, obj, grad, fe, adj, stream);
}
