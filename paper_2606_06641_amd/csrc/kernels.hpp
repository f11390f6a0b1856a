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
    int64_t tab_rows = 0;
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
    int32_t rpl;          // J == 1: restarts per lane asked for (0: 4 for S <= 8, else 1)
};

// FE (and with grad, per-literal adjoints) of one length bucket.
//   adj  [L][Bp] (slot order, written when grad), part [tiles][Bp] objective partials
//   (may be null), fe [C][B] (may be null), dobj [B] per-restart seed of the adjoint
//   (may be null: 1).  skip [B] (may be null): a wave whose restarts all have
//   skip != 0 returns at once and writes nothing, so their outputs keep old values.
hipError_t launch_fe_grad(const DevInstance &I, const BucketLaunch &bk, int B, int Bp,
                          const float *x, float *adj, float *part, float *fe, const float *dobj,
                          bool grad, hipStream_t s, const uint8_t *skip = nullptr);

// grad[v][b] = sum of adj over the slots of v, ascending.
hipError_t launch_scatter(const DevInstance &I, int B, int Bp, const float *adj, float *grad,
                          hipStream_t s);

// Per-(sub-instance, restart) arrays (unsat, done, first_sat) are [n_inst][B].
// Fused: gradient sum, projected step, rounding into bits [n][W] and unsat = 0.
// fixed [n_partial][n]: restart b uses row b * n_partial / B (nullptr: none fixed).
// vel [n][B] (nullptr: plain step): heavy-ball velocity, v = mu v + g, and the
// step follows v.
hipError_t launch_scatter_step(const DevInstance &I, int B, int Bp, const float *adj, float *x,
                               float lr, const uint8_t *fixed, int n_partial, const uint8_t *done,
                               uint32_t *bits, int32_t *unsat, hipStream_t s, uint8_t *moved = nullptr,
                               float eps = 0.0f, float *vel = nullptr, float mu = 0.0f);

// obj[b] = sum over tiles of part[t][b] (two fixed-order passes through part2).
hipError_t launch_obj_reduce(int tiles, int B, int Bp, const float *part, float *part2,
                             float *obj, hipStream_t s);

hipError_t launch_step(const DevInstance &I, int B, float *x, const float *grad, float lr,
                       const uint8_t *fixed, int n_partial, const uint8_t *done, hipStream_t s);

// bits from x and unsat = 0.
hipError_t launch_round(const DevInstance &I, int B, const float *x, uint32_t *bits, int32_t *unsat,
                        hipStream_t s);

// unsat[b] += number of violated constraints (unsat must be zeroed before);
// viol [W][C rounded up to 4] is scratch for the per-constraint violation masks.
hipError_t launch_verify(const DevInstance &I, int B, const uint32_t *bits, uint32_t *viol,
                         int32_t *unsat, hipStream_t s);

enum FinalizeMode { FIN_INIT = 0, FIN_STEP = 1, FIN_VERIFY = 2 };
// over all count = n_inst * B (sub-instance, restart) pairs.  done: 1 verified,
// 2 converged (FIN_STEP: step length eta[b] (or eta_const when eta is null) below
// delta > 0, or with eps > 0 no flag in moved [count] set by the step); moved,
// when given, is cleared at FIN_INIT and after every FIN_STEP.  counter = {t,
// verified pairs, frozen pairs, 0}.
hipError_t launch_finalize(int count, int B, const int32_t *unsat, uint8_t *done, int32_t *first_sat,
                           int32_t *counter, int mode, hipStream_t s, const float *eta = nullptr,
                           float eta_const = 0.0f, float delta = 0.0f, uint8_t *moved = nullptr,
                           float eps = 0.0f);

// ---- line search (search_kernels.hip) ----
// Trial point of the backtracking search for the restarts still searching
// (acc[b] == 0): xt = x for fixed variables, else clip(x - eta[b] * g); other
// restarts copy x.  dot_part [ceil(n / kTrialVars)][Bp] receives the per-tile
// partial sums of g * (xt - x) (zero for b >= B).  g, x, xt: [n][B].
constexpr int kTrialVars = 32;
hipError_t launch_trial(const DevInstance &I, int B, int Bp, const float *x, const float *g, const float *eta,
                        const uint8_t *acc, const uint8_t *fixed, int n_partial, float *xt, float *dot_part,
                        hipStream_t s);
// eta[b] = s, acc[b] = done[b] != 0 (done may be null)
hipError_t launch_search_init(int B, float step, const uint8_t *done, float *eta, uint8_t *acc, hipStream_t s);
// Armijo test of one trial for the restarts still searching: accept when
// ft <= f0 + c * dot, else eta *= beta (after the last trial: eta = 0, no step).
hipError_t launch_accept(int B, const float *f0, const float *ft, const float *dot, float c, float beta,
                         bool last, float *eta, uint8_t *acc, hipStream_t s);
// x <- clip(x - eta[b] * g) (not for fixed variables or done restarts), rounding
// into bits and unsat = 0, as the fused step of the constant-step path.
hipError_t launch_search_step(const DevInstance &I, int B, float *x, const float *g, const float *eta,
                              const uint8_t *fixed, int n_partial, const uint8_t *done, uint32_t *bits,
                              int32_t *unsat, hipStream_t s, uint8_t *moved = nullptr, float eps = 0.0f);
// Starting points (Sec. 3.4): x[v][b] uniform in [-1, 1) from Philox4x32-10 keyed
// by seed with counter (b, v, 0, 0), except where values[p][v] != 0 (row p =
// b * n_partial / B): -1 for +1 (True), +1 for -1 (False).
hipError_t launch_init_points(int n, int B, uint64_t seed, const int8_t *values, int n_partial, float *x,
                              hipStream_t s);

// Precision study: fe[b] = Re sum_m d_m prod_i (alpha_m + beta_m y[i][b]) in FP32
// (fp64 false; tables and y rounded to FP32 first) or FP64; tab [k+1][6] =
// alpha, beta, d as (re, im) pairs.
hipError_t launch_fe_generic(int k, const double *tab, bool fp64, int B, const double *y, double *fe,
                             hipStream_t s);

// adj_out[slot_to_lit[s]][b] = adj[s][b]
hipError_t launch_permute_adj(const DevInstance &I, int B, int Bp, const float *adj,
                              float *adj_out, hipStream_t s);

}  // namespace afs
