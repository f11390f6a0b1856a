// kernels.hpp -- device kernels of the Accelerated Fourier SAT hot path (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace afs {

// Device copies of the packed instance (all owned by the instance).
struct DevInstance {
    int32_t n = 0, C = 0;
    int64_t L = 0;
    // bucket-ordered constraints
    const int32_t *bc_slot0 = nullptr, *bc_k = nullptr, *bc_tab = nullptr, *bc_orig = nullptr;
    const float *bc_w = nullptr;
    // literal slots
    const int32_t *slot_lit = nullptr, *slot_to_lit = nullptr;
    // coefficient tables
    const float4 *tab = nullptr;
    // variable -> slot transpose
    const int32_t *voff = nullptr, *vslot = nullptr;
    // original-order constraints (verification)
    const int32_t *con_off = nullptr, *lits = nullptr, *types = nullptr, *params = nullptr;
    // block-diagonal batches: sub-instance of each constraint / variable
    int32_t n_inst = 1;
    const int32_t *con_inst = nullptr, *var_inst = nullptr;
    // constraints of the counted types (CARD >= K, CARD < K, EK), input order
    int32_t n_counted = 0;
    const int32_t *counted = nullptr;
};

// The device copy of the literal array carries kLitPad trailing zeros, so that
// verification reads whole batches of literals without a bounds check.
constexpr int kLitPad = 32;

struct BucketLaunch {
    int J, S;
    int32_t c0, nc, tile, ntiles, tile0;
};

// FE (and with grad, per-literal adjoints) of one length bucket.
//   adj  [L][Bp] (slot order, written when grad), part [tiles][Bp] objective partials
//   (may be null), fe [C][B] (may be null), dobj [B] per-restart seed of the adjoint
//   (may be null: 1).
hipError_t launch_fe_grad(const DevInstance &I, const BucketLaunch &bk, int B, int Bp,
                          const float *x, float *adj, float *part, float *fe, const float *dobj,
                          bool grad, hipStream_t s);

// grad[v][b] = sum of adj over the slots of v, ascending.
hipError_t launch_scatter(const DevInstance &I, int B, int Bp, const float *adj, float *grad,
                          hipStream_t s);

// Per-(sub-instance, restart) arrays (unsat, done, first_sat) are [n_inst][B].
// Fused: gradient sum, projected step, rounding into bits [n][W] and unsat = 0.
hipError_t launch_scatter_step(const DevInstance &I, int B, int Bp, const float *adj, float *x,
                               float lr, const uint8_t *fixed, const uint8_t *done,
                               uint32_t *bits, int32_t *unsat, hipStream_t s);

// obj[b] = sum over tiles of part[t][b] (two fixed-order passes through part2).
hipError_t launch_obj_reduce(int tiles, int B, int Bp, const float *part, float *part2,
                             float *obj, hipStream_t s);

hipError_t launch_step(const DevInstance &I, int B, float *x, const float *grad, float lr,
                       const uint8_t *fixed, const uint8_t *done, hipStream_t s);

// bits from x and unsat = 0.
hipError_t launch_round(const DevInstance &I, int B, const float *x, uint32_t *bits, int32_t *unsat,
                        hipStream_t s);

// unsat[b] += number of violated constraints (unsat must be zeroed before);
// viol [W][C rounded up to 4] is scratch for the per-constraint violation masks.
hipError_t launch_verify(const DevInstance &I, int B, const uint32_t *bits, uint32_t *viol,
                         int32_t *unsat, hipStream_t s);

enum FinalizeMode { FIN_INIT = 0, FIN_STEP = 1, FIN_VERIFY = 2 };
// over all n_inst * B (sub-instance, restart) pairs
hipError_t launch_finalize(int count, const int32_t *unsat, uint8_t *done, int32_t *first_sat,
                           int32_t *counter, int mode, hipStream_t s);

// adj_out[slot_to_lit[s]][b] = adj[s][b]
hipError_t launch_permute_adj(const DevInstance &I, int B, int Bp, const float *adj,
                              float *adj_out, hipStream_t s);

}  // namespace afs
