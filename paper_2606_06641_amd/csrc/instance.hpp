// instance.hpp -- the opaque afs_instance (shared by the C ABI translation units).
#pragma once

#include <cstdint>
#include <mutex>
#include <string>
#include <vector>

#include <hip/hip_runtime_api.h>

#include "afsat.h"
#include "host.hpp"
#include "kernels.hpp"

// Device copy of the variable-constraint graph used by the message-passing
// network (built on first use, owned by the instance).
struct GnnGraph {
    bool built = false;
    const float *fcon = nullptr;     // [C][16] constraint features
    const float *fvar = nullptr;     // [n][16] variable features
    const int32_t *var_off = nullptr; // [n+1] incidences of each variable
    const int32_t *var_con = nullptr; // [L] constraint of each incidence
    const float *var_sgn = nullptr;   // [L] literal sign (+1 / -1)
    const float *inv_k = nullptr;     // [C] 1 / constraint length
    const float *inv_deg = nullptr;   // [n] 1 / max(1, occurrences)
};

namespace afs {
// Set the thread-local message returned by afs_last_error; returns s.
afs_status set_last_error(afs_status s, const std::string &msg);
}  // namespace afs

struct afs_instance;

namespace afs {
// Bytes of scratch afs_eval uses at B restarts (the adjoint rows and the
// objective partials of its workspace).
size_t eval_scratch_bytes(const afs_instance *I, int32_t B);
// afs_eval with `scratch` (256-byte aligned, scratch_bytes long) in place of
// the caller's workspace; AFS_EINVAL when it is too small.
afs_status eval_in_scratch(afs_instance *I, int32_t B, const float *x, void *scratch, size_t scratch_bytes,
                           float *obj, float *grad, float *fe, float *adj, void *stream);
}  // namespace afs

struct afs_instance {
    afs::HostInstance H;
    afs::DevInstance D;
    int device = -1;
    std::vector<void *> allocs;      // every device allocation, freed at destroy
    GnnGraph gnn;
    // Second stream for the short-constraint buckets (memory-bound), which then
    // run beside the long ones (ALU-bound) on the caller's stream; fork and join
    // events order it against the caller's stream.  The mutex keeps one call's
    // record / wait pairs together when several host threads use the instance.
    hipStream_t side = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
    // Long buckets are few constraints each, so one of them rarely fills the
    // device; they are split between the caller's stream and the `side_long`
    // streams (each joined back through its `join_long` event) so that
    // 1 + kLongSides run at a time.  Three at a time measured within 1 % of two
    // on the bench workloads (better on the small ones, worse on the long-CARD
    // one), and the driver's verification stream makes a fifth on a device with
    // four hardware queues, so two it is.
    static constexpr int kLongSides = 1;
    hipStream_t side_long[kLongSides] = {};
    hipEvent_t join_long[kLongSides] = {};
    std::mutex side_mu;
    // Private stream of the Algorithm 1 driver (afs_pgd), which captures its
    // iterations in a graph there; events order it against the caller's stream.
    hipStream_t drive = nullptr;
    hipEvent_t drive_in = nullptr, drive_out = nullptr;
    std::mutex drive_mu;
    // The driver verifies iteration t on its own stream while iteration t+1's FE
    // kernels run (they touch neither the bits nor the counts); `stepped` orders
    // the verification after the step, `verified` the next step after it.
    hipStream_t verify = nullptr;
    hipEvent_t stepped = nullptr, verified = nullptr;
    // Pinned host copy of the driver's counter (four int32), read between blocks.
    int32_t *counter_host = nullptr;
};
