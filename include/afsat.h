/*
 * afsat.h -- C ABI of the MI355X Accelerated Fourier SAT hot path.
 *
 * The library evaluates, for a batch of B real points x in [-1,1]^n ("restarts"),
 * the Walsh-Fourier expansion FE of every symmetric constraint of an instance
 * (Sec. 2.1, Eq. 1), the objective F = sum_c w_c FE_c (Sec. 2.1.1, Eq. 2) and its
 * gradient, takes the projected gradient step of Algorithm 1, rounds the points to
 * Boolean assignments and counts unsatisfied constraints exactly (Algorithm 1's
 * unsat_count).  FE is computed the way Sec. 2.1.2 describes: a product, per root
 * of unity of order k+1, of one factor per literal, contracted against a per
 * constraint coefficient vector (an inverse DFT of the constraint's truth table).
 *
 * Conventions shared by every call:
 *   - Truth values: True -> -1, False -> +1 (Sec. 2.1).  A constraint's FE is -1
 *     when it is satisfied and +1 when it is violated at a Boolean corner.
 *   - Points: x is a device float32 array of shape [n][B] (restart index
 *     contiguous, row stride B).  grad has the same shape.  Literal i of a
 *     constraint has value y_i = x[v] for a positive DIMACS literal v+1 and
 *     y_i = -x[v] for a negative one.
 *   - Rounding: variable v of restart b is True iff x[v][b] < 0 (so +0.0, -0.0
 *     and NaN are False).  A literal is true iff its variable's truth differs from
 *     the literal's negation.
 *   - Ownership: an instance owns its device tables (allocated at create, freed
 *     at destroy).  Every per-call buffer and the workspace are owned by the
 *     caller and passed as raw device pointers.  Nothing a call receives is
 *     retained after it returns.
 *   - Execution: device calls enqueue work on `stream` (a hipStream_t; NULL is
 *     the default stream) and return without synchronising.  afs_eval, afs_fe_grad,
 *     afs_scatter, afs_step, afs_round_verify and afs_pgd_step allocate nothing
 *     and copy nothing between host and device.
 *   - Errors: invalid arguments return AFS_EINVAL before anything is launched; a
 *     launch failure returns AFS_EDEVICE.  afs_last_error() gives a message for
 *     the last non-OK status of the calling thread.
 *   - Thread safety: an instance is immutable after creation; concurrent calls
 *     on different streams with distinct workspaces and outputs are safe.
 *   - A restart is satisfied iff its unsat count is 0.  Finding no satisfied
 *     restart means "unknown", never "unsatisfiable" (the method is incomplete).
 */
#ifndef AFSAT_H
#define AFSAT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    AFS_OK = 0,
    AFS_EINVAL = -1,   /* invalid argument or instance */
    AFS_EUNSAT = -2,   /* input proven unsatisfiable while parsing (afs_parse_*) */
    AFS_ENOMEM = -3,   /* host or device allocation failed */
    AFS_EDEVICE = -4,  /* HIP runtime or kernel launch error */
    AFS_ESTATE = -5    /* call not valid for this instance (e.g. host-only) */
} afs_status;

/* Longest constraint the evaluation kernels take. */
#define AFS_MAX_LEN 1024

/* Symmetric constraint types (Table 1; Table 2 and the CARD normalisation of
 * Appendix A).  t = number of true literals out of k. */
typedef enum {
    AFS_OR = 0,       /* t >= 1                                    */
    AFS_XOR = 1,      /* t = param (mod 2); param 1 = odd parity   */
    AFS_NAE = 2,      /* 0 < t < k                                 */
    AFS_CARD_GE = 3,  /* t >= param                                */
    AFS_CARD_LT = 4,  /* t <  param                                */
    AFS_AMO = 5,      /* t <= 1                                    */
    AFS_EO = 6,       /* t == 1                                    */
    AFS_EK = 7        /* t == param                                */
} afs_ctype;

typedef struct afs_instance afs_instance;

typedef struct {
    int32_t n_vars;
    int32_t n_cons;
    int64_t n_lits;      /* L = total literal occurrences */
    int32_t n_buckets;   /* length buckets (one kernel launch each) */
    int32_t n_tables;    /* distinct (type, k, param) coefficient tables */
    int32_t max_k;
    int32_t device;      /* HIP device ordinal, or -1 for a host-only instance */
    int32_t n_inst;      /* sub-instances: 1, or the number of parts of a batch */
} afs_info;

/* One length bucket: constraints of lengths [k_lo, k_hi] evaluated by one kernel
 * variant.  lanes_per_restart = 1 means one lane per restart holding the whole
 * constraint; otherwise that many lanes split the literals of one restart into
 * segments of lits_per_lane. */
typedef struct {
    int32_t k_lo, k_hi;
    int32_t n_cons;
    int64_t n_lits;
    int32_t lanes_per_restart;
    int32_t lits_per_lane;
    int64_t slot0;       /* first literal slot of the bucket */
    int32_t tile;        /* constraints per work tile */
    int32_t rpl;         /* one-lane buckets: restarts per lane asked for (0: default) */
} afs_bucket_info;

/* ---- instance -------------------------------------------------------------- */

/* Build an instance from a constraint list in CSR form (Sec. 2.1.1: a formula is a
 * list of symmetric constraints C_1..C_m over n variables).
 *   n_vars   : number of variables, >= 1
 *   n_cons   : number of constraints, >= 0
 *   con_off  : host int64 [n_cons+1], con_off[0] = 0, non-decreasing; constraint
 *              c owns lits[con_off[c] .. con_off[c+1]) and has length
 *              1 <= k <= AFS_MAX_LEN (longer OR, XOR, NAE, AMO and EO constraints
 *              can be split first by afs_decompose)
 *   lits     : host int32 [L] DIMACS literals, +-(1..n_vars)
 *   types    : host int32 [n_cons] afs_ctype
 *   params   : host int32 [n_cons] XOR parity (0/1), or K for CARD_GE/CARD_LT/EK
 *              (any integer; K outside 0..k+1 makes the constraint constant);
 *              ignored for other types.  May be NULL if no type needs it.
 *   weights  : host float [n_cons] constraint weights w_c, or NULL for all 1
 *   device   : HIP device ordinal, or -1 to build host tables only (for
 *              inspection; device calls on it return AFS_ESTATE)
 *   out      : receives the instance
 * Computes the truth table g_c(t) of every constraint, its coefficient vector
 * (an FP64 DFT with exactly mirrored roots, Sec. 3.5.1), length buckets and the
 * variable -> literal-slot transpose, then uploads them.  Host arrays are copied;
 * the caller keeps ownership. */
afs_status afs_instance_create(int32_t n_vars, int32_t n_cons, const int64_t *con_off,
                               const int32_t *lits, const int32_t *types,
                               const int32_t *params, const float *weights,
                               int32_t device, afs_instance **out);

/* Optional packing choices (every field 0 / NULL: the built-in defaults).
 *   n_shapes, shape_k_hi, shape_lanes, shape_seg: kernel shape per length range for
 *       constraints longer than 16: a constraint of length k uses the first entry
 *       with k <= shape_k_hi[e] (ascending), evaluated by shape_lanes[e] lanes per
 *       restart (2, 4, 8, 16, 32 or 64) holding shape_seg[e] literals each (even,
 *       4 to 32), with lanes * seg >= shape_k_hi[e].  Lengths past the last entry
 *       use the default shape model.  (These are what the autotuner picks.)
 *   tile_short / tile_long: constraints per work tile (one wave's share of a
 *       bucket, 0 to 4096, 0: default) for lengths <= 16 / > 16.
 *   shape_tile: int32 [n_shapes] or NULL: constraints per work tile of each shape
 *       entry (0: tile_long or the default).
 *   short_tile, short_rpl: int32 [16] or NULL, index k-1 for length k <= 16:
 *       constraints per work tile (0: tile_short or the default) and restarts
 *       held per lane by the one-lane kernel (0: the default, 4 for k <= 8 and 1
 *       above; else 1, 2, or 4 for k <= 8).  A launch whose B or x (or adjoint
 *       seed) alignment does not allow the asked count uses 1.
 * Restarts per lane change only the time; tiles also change how the objective
 * is split into partial sums, and a segment shape the order of the FP32
 * products, so those results differ by rounding (within the same error
 * bounds). */
typedef struct {
    int32_t n_shapes;
    const int32_t *shape_k_hi;
    const int32_t *shape_lanes;
    const int32_t *shape_seg;
    int32_t tile_short;
    int32_t tile_long;
    const int32_t *shape_tile;
    const int32_t *short_tile;
    const int32_t *short_rpl;
} afs_options;

/* afs_instance_create with packing options (opts may be NULL). */
afs_status afs_instance_create_ex(int32_t n_vars, int32_t n_cons, const int64_t *con_off,
                                  const int32_t *lits, const int32_t *types,
                                  const int32_t *params, const float *weights,
                                  const afs_options *opts, int32_t device, afs_instance **out);

/* Block-diagonal batch of independent instances, evaluated together: the
 * variables and constraints of parts[0..n_parts) are concatenated (variables of
 * part p follow those of parts 0..p-1), so every kernel launch covers all parts
 * and one restart column b of the batch holds restart b of every part.  FE,
 * gradient and step are exactly those of the parts; unsat / done / first_sat
 * become per (part, restart): arrays [n_parts][B] (see afs_pgd_state).  The
 * parts are read (their host copies), not retained; they may be host-only.
 * Many uneven instances run in one set of launches this way, with one shape
 * choice per length range across all of them. */
afs_status afs_batch_create(const afs_instance *const *parts, int32_t n_parts, const afs_options *opts,
                            int32_t device, afs_instance **out);

/* First variable of each part of a batch: var0 int32 [n_inst+1] (host). */
afs_status afs_batch_var_offsets(const afs_instance *inst, int32_t *var0);

/* Free the instance and its device tables.  NULL is accepted.  Waits for all
 * work on the instance's device to finish first (a device-wide synchronisation),
 * so work still queued on any stream never reads freed tables; the caller's own
 * buffers stay the caller's. */
void afs_instance_destroy(afs_instance *inst);

afs_status afs_instance_info(const afs_instance *inst, afs_info *out);

/* Describe bucket `b` (0 <= b < n_buckets). */
afs_status afs_bucket_info_get(const afs_instance *inst, int32_t b, afs_bucket_info *out);

/* Host copy of the literal slot order: slot_to_lit[s] = index into the input
 * `lits` array of the literal occurrence stored in slot s (int64 [L]). */
afs_status afs_instance_slot_map(const afs_instance *inst, int64_t *slot_to_lit);

/* Host copy of the variable -> slot transpose: voff int64 [n_vars+1] and
 * vslot int64 [L]; the slots of variable v are vslot[voff[v] .. voff[v+1]),
 * ascending. */
afs_status afs_instance_transpose(const afs_instance *inst, int64_t *voff, int64_t *vslot);

/* FP64 coefficient vector of one constraint (Sec. 2.1.2): with N = k+1 and
 * omega = exp(2*pi*i/N), d_m = (1/N) * sum_{t=0..k} g(t) * omega^(-m*t) for
 * m = 0..k, where g(t) = -1 if t true literals satisfy the constraint, else +1.
 * re, im: host double [k+1].  Needs no instance. */
afs_status afs_coefficients(int32_t type, int32_t k, int32_t param, double *re, double *im);

/* Bytes of device workspace that afs_eval / afs_fe_grad / afs_pgd_step need for
 * B restarts.  The workspace is caller-owned, at least 256-byte aligned, and may
 * be reused across calls on the same stream. */
afs_status afs_workspace_bytes(const afs_instance *inst, int32_t B, size_t *bytes);

/* ---- evaluation (Sec. 2.1.2; Sec. 2.1.1 Eq. 2) ------------------------------- */

/* FE, objective and gradient at B points.
 *   x    : device f32 [n][B], values in [-1,1]
 *   ws   : device workspace of afs_workspace_bytes(inst, B) bytes
 *   obj  : device f32 [B]      sum_c w_c FE_c                   (NULL: skip)
 *   grad : device f32 [n][B]   dF/dx                            (NULL: skip)
 *   fe   : device f32 [C][B]   FE_c per constraint, input order (NULL: skip)
 *   adj  : device f32 [L][B]   w_c * dFE_c/dx_v per literal occurrence, in the
 *                              input literal order              (NULL: skip) */
afs_status afs_eval(afs_instance *inst, int32_t B, const float *x, void *ws, size_t ws_bytes,
                    float *obj, float *grad, float *fe, float *adj, void *stream);

/* Lower-level pieces of afs_eval, in the order they must run on one stream:
 * afs_fe_grad evaluates buckets [bucket_lo, bucket_hi) into the workspace (per
 * literal adjoints, and per-tile objective partials when want_obj != 0; fe as in
 * afs_eval, for the constraints of those buckets); afs_scatter sums the adjoints
 * of each variable in ascending slot order into grad and reduces the objective
 * partials into obj (either may be NULL; obj needs every bucket evaluated with
 * want_obj != 0). */
afs_status afs_fe_grad(afs_instance *inst, int32_t B, const float *x, void *ws, size_t ws_bytes,
                       int32_t bucket_lo, int32_t bucket_hi, int32_t want_obj, float *fe,
                       void *stream);
afs_status afs_scatter(afs_instance *inst, int32_t B, void *ws, size_t ws_bytes,
                       float *obj, float *grad, void *stream);

/* afs_fe_grad over an explicit set of buckets: buckets host int32 [n_buckets],
 * distinct indices in any order (AFS_EINVAL otherwise).  As for a range, short
 * buckets run on a second stream beside the long ones, and the long ones are
 * split between the caller's stream and a third, so one call over many buckets
 * keeps more of the device busy than a call per bucket. */
afs_status afs_fe_grad_buckets(afs_instance *inst, int32_t B, const float *x, void *ws, size_t ws_bytes,
                               const int32_t *buckets, int32_t n_buckets, int32_t want_obj, float *fe,
                               void *stream);

/* ---- differentiation (the objective as a differentiable function of x) ---------- */

/* Forward: obj[b] = sum_c w_c FE_c(x_b) and optionally fe [C][B], with no adjoint
 * work (each root's product chain runs once, nothing is stored for a backward
 * pass).  obj: device f32 [B] (required); fe may be NULL. */
afs_status afs_eval_fwd(afs_instance *inst, int32_t B, const float *x, void *ws, size_t ws_bytes,
                        float *obj, float *fe, void *stream);

/* Backward (adjoint): grad[v][b] = dobj[b] * dF_b/dx[v][b], the vector-Jacobian
 * product of afs_eval_fwd.  The products are recomputed from x (nothing is kept
 * from the forward).  dobj: device f32 [B], or NULL for all ones; grad: device
 * f32 [n][B] (overwritten); adj: device f32 [L][B] or NULL, receives
 * dobj[b] * w_c * dFE_c/dx_v per literal occurrence in the input literal order
 * (the terms grad sums). */
afs_status afs_eval_adjoint(afs_instance *inst, int32_t B, const float *x, const float *dobj,
                            void *ws, size_t ws_bytes, float *grad, float *adj, void *stream);

/* ---- Algorithm 1 --------------------------------------------------------------- */

/* Partial assignments (Sec. 3.4).  Wherever a call takes `fixed, n_partial`,
 * fixed is NULL (nothing fixed) or device u8 [n_partial][n] (n_partial 0 reads as
 * 1): the B restarts are divided evenly among the rows, restart b using row
 * b * n_partial / B, and variable v is held where that row's entry is nonzero.
 * n_partial > B is rejected.  The values the variables are held at are those in
 * x (afs_init_points writes them). */

/* Projected gradient step with constant step length (Algorithm 1,
 * projectToBounds onto [-1,1]^n):  x <- min(1, max(-1, x - lr * grad)) in FP32,
 * skipped for fixed variables (Sec. 3.4) and restarts with done != 0 (finished
 * candidates do no-ops, Sec. 3.3).
 *   x: device f32 [n][B] updated in place; grad: device f32 [n][B];
 *   fixed, n_partial: as above; done: device u8 [P][B] or NULL (P as in
 *   afs_pgd_state; variable v of part p is frozen where done[p][b] != 0). */
afs_status afs_step(afs_instance *inst, int32_t B, float *x, const float *grad, float lr,
                    const uint8_t *fixed, int32_t n_partial, const uint8_t *done, void *stream);

/* Round and count unsatisfied constraints exactly (Algorithm 1's unsat_count).
 *   x    : device f32 [n][B]
 *   bits : device u32 [n][ceil(B/32)]: bit (b % 32) of word b/32 = (x[v][b] < 0)
 *          (NULL: not returned; a workspace copy is used)
 *   ws   : workspace as for afs_eval (required: it holds the per-constraint
 *          violation masks of the count)
 *   unsat: device i32 [P][B] (required; P = 1, or the parts of a batch)
 *   done : device u8 [P][B] or NULL; set to 1 where unsat == 0 (never cleared) */
afs_status afs_round_verify(afs_instance *inst, int32_t B, const float *x, uint32_t *bits,
                            void *ws, size_t ws_bytes, int32_t *unsat, uint8_t *done,
                            void *stream);

/* Device state of a batched run of Algorithm 1 (all caller-owned device arrays).
 * For a batch of P parts the per-restart arrays are [P][B] (part-major); a plain
 * instance has P = 1. */
typedef struct {
    int32_t *unsat;      /* [P][B] unsat count at the current point                 */
    uint8_t *done;       /* [P][B] 0 searching, 1 verified, 2 converged (its step
                            length fell below delta, Algorithm 1, or its point moved
                            less than epsilon, Sec. 3.3); either freezes it          */
    int32_t *first_sat;  /* [P][B] iteration at which it verified, -1 if not yet    */
    int32_t *counter;    /* [4] {iteration t, pairs verified, pairs frozen (verified
                            or converged), 0}; t counts completed iterations        */
} afs_pgd_state;

/* Reset the state and check the initial point X_(0): unsat, done and first_sat = 0
 * where X_(0) already verifies, t = 0. */
afs_status afs_pgd_init(afs_instance *inst, int32_t B, const float *x, void *ws, size_t ws_bytes,
                        const afs_pgd_state *st, void *stream);

/* One iteration of Algorithm 1 with constant step length lr: the gradient at
 * X_(t-1), the projected step to X_(t) (frozen for done restarts and fixed
 * variables), rounding and the exact unsat count of X_(t); restarts that verify
 * become done with first_sat = t.  Same launches every call (the iteration
 * number lives in st->counter), so a sequence of calls may be captured in a
 * HIP graph and replayed. */
afs_status afs_pgd_step(afs_instance *inst, int32_t B, float *x, float lr, const uint8_t *fixed,
                        int32_t n_partial, void *ws, size_t ws_bytes, const afs_pgd_state *st,
                        void *stream);

/* The part of afs_pgd_step that follows the FE kernels: with the per-literal
 * adjoints of X_(t-1) already in the workspace (afs_fe_grad over every bucket),
 * sum them per variable, take the projected step, round, count unsatisfied
 * constraints and update the state.  afs_fe_grad(all buckets) followed by
 * afs_pgd_update is exactly afs_pgd_step. */
afs_status afs_pgd_update(afs_instance *inst, int32_t B, float *x, float lr, const uint8_t *fixed,
                          int32_t n_partial, void *ws, size_t ws_bytes, const afs_pgd_state *st,
                          void *stream);

/* One iteration of another search algorithm in PGD's place (Sec. 3.2 allows
 * other algorithms with compatible implementations; this one is projected
 * gradient descent with heavy-ball momentum): with g the gradient at X_(t-1),
 * v <- mu v + g and X_(t) = clip(X_(t-1) - lr v, -1, 1), then rounding, the exact
 * unsat count and the state update as afs_pgd_step.  Done restarts and fixed
 * variables keep both x and v.
 *   vel: device f32 [n][B], the velocity, caller-owned and updated in place
 *     (zero it before the first step); mu in [0, 1) (mu = 0 gives afs_pgd_step).
 * Same launches every call, so it may be captured in a graph like
 * afs_pgd_step.  AFS_EINVAL for a NULL vel (B > 0) or mu outside [0, 1). */
afs_status afs_pgd_step_momentum(afs_instance *inst, int32_t B, float *x, float *vel, float lr, float mu,
                                 const uint8_t *fixed, int32_t n_partial, void *ws, size_t ws_bytes,
                                 const afs_pgd_state *st, void *stream);

/* Backtracking line search (Algorithm 1's lineSearch with maximum step s;
 * Sec. 3.3: each restart picks its own step length).  Per restart: f0 = F(x) and
 * g = grad F(x); trial j = 0..trials-1 takes eta = max_step * shrink^j and
 * xt = clip(x - eta g, -1, 1) (fixed variables held) and accepts the first trial
 * with F(xt) <= f0 + armijo * <g, xt - x> (sufficient decrease along the
 * projection arc); when none is accepted eta = 0 and the restart does not move.
 * F(xt) is the same FE kernels' forward pass; the sums are fixed-order. */
typedef struct {
    float max_step;         /* s > 0: the first trial step length                */
    float shrink;           /* in (0,1): factor between consecutive trials        */
    float armijo;           /* in [0,1): sufficient-decrease constant             */
    int32_t trials;         /* trial step lengths per iteration, 1..64            */
} afs_line_search;

/* Bytes of the second workspace a line search needs for B restarts (gradient
 * and trial point [n][B] and per-restart vectors); caller-owned, 256-byte
 * aligned. */
afs_status afs_search_workspace_bytes(const afs_instance *inst, int32_t B, size_t *bytes);

/* One iteration of Algorithm 1 with the line search above: search, step to
 * X_(t) with the chosen eta, rounding, exact unsat count and state update as in
 * afs_pgd_step; then a restart that did not verify and whose eta < delta
 * (delta > 0) converges (done = 2).  eta: device f32 [B] receiving the chosen
 * step lengths, or NULL.  Plain instances only (a batch returns AFS_EINVAL).
 * Launch-only, so a sequence of calls may be captured in a HIP graph. */
afs_status afs_pgd_search_step(afs_instance *inst, int32_t B, float *x, const afs_line_search *ls,
                               const uint8_t *fixed, int32_t n_partial, float delta, void *ws,
                               size_t ws_bytes, void *search_ws, size_t search_ws_bytes,
                               const afs_pgd_state *st, float *eta, void *stream);

/* Starting points (Sec. 3.4: fixed variables across all restarts, the rest
 * random).  x[v][b] = -1 where values[p][v] > 0 (True), +1 where it is < 0
 * (False), with p = b * n_partial / B; elsewhere uniform on [-1, 1): the top 24
 * bits u of the first word of Philox4x32-10 (Salmon et al., SC 2011) with key
 * (seed low word, seed high word) and counter (b, v, 0, 0), x = u * 2^-23 - 1.
 * values: device i8 [n_partial][n] or NULL (all random); a values array may
 * serve as the fixed mask of the other calls (nonzero = fixed).  x: device
 * f32 [n][B]. */
afs_status afs_init_points(afs_instance *inst, int32_t B, uint64_t seed, const int8_t *values,
                           int32_t n_partial, float *x, void *stream);

/* Parameters of afs_pgd. */
typedef struct {
    float lr;               /* constant step length (Algorithm 1 with lineSearch fixed)   */
    int32_t max_iters;      /* iteration budget d (>= 0)                                  */
    int32_t poll;           /* iterations between reads of the done counter (>= 1)        */
    int32_t stop_on_sat;    /* != 0: stop at the first read that finds a verified restart */
    int32_t use_graph;      /* != 0: capture min(poll, 64) iterations once in a HIP graph
                               and replay it (the iterations are identical either way)    */
    const uint8_t *fixed;   /* device u8 [n_partial][n] or NULL: variables held at their
                               value (partial assignments, Sec. 3.4)                       */
    int32_t n_partial;      /* rows of fixed (0 reads as 1)                                 */
    float delta;            /* > 0: a restart whose step length falls below delta
                               converges and stops (Algorithm 1); 0: off                   */
    const afs_line_search *search;  /* NULL: constant step lr; else the line search
                               (plain instances only)                                       */
    void *search_ws;        /* line-search workspace (afs_search_workspace_bytes)          */
    size_t search_ws_bytes;
    float epsilon;          /* > 0: a restart whose new point lies within epsilon of the
                               previous one in every variable (max |x_t - x_(t-1)| <
                               epsilon, Sec. 3.3) converges and stops; 0: off.  A
                               restart that verifies in the same iteration counts as
                               verified.  Uses the flags at the end of the workspace,
                               which afs_pgd_init clears                                    */
    float momentum;         /* > 0 (below 1): heavy-ball momentum in PGD's place, each
                               iteration as afs_pgd_step_momentum; 0: plain steps. Not
                               with the line search                                        */
    float *velocity;        /* device f32 [n][B], the velocity (required with momentum;
                               caller-owned, updated in place, zero it first)              */
} afs_pgd_params;

/* Algorithm 1 on the B columns of x (device f32 [n][B], updated in place to the
 * final point): afs_pgd_init, then up to max_iters iterations of afs_pgd_step
 * (constant step), afs_pgd_search_step (line search) or afs_pgd_step_momentum
 * (momentum > 0), reading the device counter every `poll` iterations (when
 * stop_on_sat is set or delta or epsilon > 0) and
 * stopping when stop_on_sat is set and some (part, restart) has verified, or
 * when every (part, restart) has verified or converged.
 * On return st holds unsat / done / first_sat / counter as after those calls,
 * obj (device f32 [B] or NULL) the objective F at the final point (Eq. 2), and
 * *iters (host, or NULL) the number of iterations run.  The work runs on a
 * stream private to the instance, ordered after the caller's stream on entry
 * and before it on return; the call synchronises with that private stream when
 * it reads the counter, and with use_graph it builds a graph and, once its last
 * replay has finished (another synchronisation), frees it, so it is not itself
 * capturable (capture afs_pgd_step instead).  Concurrent calls on one instance
 * are serialised. */
afs_status afs_pgd(afs_instance *inst, int32_t B, float *x, const afs_pgd_params *params, void *ws,
                   size_t ws_bytes, const afs_pgd_state *st, float *obj, int32_t *iters, void *stream);

/* Autotuner for the FE kernel configuration of each length range.  Sec. 4.2 finds
 * throughput governed by the maximum constraint length and tunes the batch size
 * for it; here the kernel that evaluates each length is tuned on the device
 * instead (the results are what afs_options' shape, tile and short arrays take).
 * Ranges: each length 1..16 alone (the one-lane kernel), then the ranges between
 * consecutive candidate capacities J*S (J in {2, ..., 64}, S even in 4..32).  For
 * every range that holds constraints of inst (a plain instance or a batch, device
 * or host-only), the constraints in that range -- an evenly spaced sample of at
 * most max_cons (<= 0: all; one-lane lengths: at least 65,536) -- are packed alone
 * once per candidate and their FE+gradient pass at B restarts is timed on
 * `device` (median of reps launches after one warm-up, HIP events on a private
 * stream).  The fastest shape with J*S >= the range's upper length at the default
 * tile wins.  With tiles != 0 a second stage follows: for one-lane lengths the
 * restarts per lane in {4 (k <= 8), 2, 1} dividing B are timed, then tiles of 1,
 * 2, 4, 8 and 16 constraints for the configuration, and one other than the
 * default must be 2% faster to replace it.  With tiles == 0 (the recommended
 * setting for iterations of mixed lengths, where the short buckets run beside the
 * long ones and configurations chosen by their time alone made iterations
 * slower) one-lane lengths are not timed and get the defaults, and every range
 * reports tile 0 and rpl 0 (the defaults).
 *   cache_in, cache_out: text files (either may be NULL) with one line per
 *     result, "<arch> <revision> <B> <k_lo> <k_hi> <class> <lanes> <seg> <tile>
 *     <rpl> <ms> <timed>", where class = floor(log2(constraints of the instance
 *     in the range)) (a range of a few constraints and one of thousands are
 *     tuned apart) and tile 0 marks a shape-only result; results found in either
 *     are reused (cache_in's where both hold one for the same key; with tiles !=
 *     0 only results with a tile), and cache_out is rewritten with them plus the
 *     new ones, keeping only the current kernel revision.
 *   k_lo, k_hi, lanes, seg: host int32 [max_ranges] (lanes 1 and seg k for a
 *     one-lane length); tile, rpl: host int32 [max_ranges] or NULL (0: the
 *     default; rpl 0 for segment shapes); ms: host float [max_ranges] or NULL (the
 *     winner's median, -1 when it came from a cache, 0 for a one-lane length left
 *     at its defaults); *n_ranges: the number of ranges the instance has (entries
 *     past max_ranges are not written).
 * Allocates device memory, synchronises `device`, and restores the caller's
 * current device. */
afs_status afs_autotune(const afs_instance *inst, int32_t device, int32_t B, int32_t reps, int32_t max_cons,
                        int32_t tiles, const char *cache_in, const char *cache_out, int32_t max_ranges, int32_t *k_lo,
                        int32_t *k_hi, int32_t *lanes, int32_t *seg, int32_t *tile, int32_t *rpl, float *ms,
                        int32_t *n_ranges);

/* ---- learned initialisation: message-passing network ---------------------------- */

/* A network over the variable-constraint graph of an instance (3 rounds by
 * default, hidden width 64) that maps uniform random starting points x0 [n][B]
 * to starting points xhat in (-1,1) for Algorithm 1; trained by its own forward,
 * backward (BCE on a target assignment) and Adam kernels.  Dense layers run on
 * BF16 MFMA with FP32 accumulation.  Parameters live on the device in one flat
 * FP32 array (gradients and Adam moments alongside).  A network is used from one
 * stream at a time. */
typedef struct afs_gnn afs_gnn;

/* Create with seeded He-normal weights; rounds 1..8. */
afs_status afs_gnn_create(int32_t rounds, uint64_t seed, int32_t device, afs_gnn **out);
/* Free the network; waits for all work on its device to finish first. */
void afs_gnn_destroy(afs_gnn *net);
afs_status afs_gnn_num_params(const afs_gnn *net, int64_t *count);
/* Synchronous host copies of the flat arrays: which = 0 parameters, 1 gradients,
 * 2 and 3 the Adam moments; host holds afs_gnn_num_params floats. */
afs_status afs_gnn_get(const afs_gnn *net, int32_t which, float *host);
afs_status afs_gnn_set(afs_gnn *net, int32_t which, const float *host);

/* Host copy of the input features and signed incidence lists of an instance:
 * fcon [C][16], fvar [n][16], var_off int32 [n+1], var_con int32 [L] (constraint
 * of each occurrence, grouped by variable), var_sgn [L] (+1 / -1).  The last three
 * may be NULL. */
afs_status afs_gnn_features(afs_instance *inst, float *fcon, float *fvar, int32_t *var_off,
                            int32_t *var_con, float *var_sgn);

/* Workspace bytes for an instance and B restarts (caller-owned, 256-byte aligned). */
afs_status afs_gnn_workspace_bytes(const afs_gnn *net, const afs_instance *inst, int32_t B,
                                   size_t *bytes);

/* xhat [n][B] (device) from x0 [n][B] (device). */
afs_status afs_gnn_forward(afs_gnn *net, afs_instance *inst, int32_t B, const float *x0, void *ws,
                           size_t ws_bytes, float *xhat, void *stream);

/* Forward, then the mean binary cross-entropy against target [n] (device u8, 1 =
 * variable True) over all (v, b), written to loss [1] (device), and its gradient
 * accumulated into the network's gradient array. */
afs_status afs_gnn_backward(afs_gnn *net, afs_instance *inst, int32_t B, const float *x0,
                            const uint8_t *target, void *ws, size_t ws_bytes, float *loss,
                            void *stream);

afs_status afs_gnn_zero_grad(afs_gnn *net, void *stream);

/* One Adam step (bias-corrected, step number t >= 1). */
afs_status afs_gnn_adam(afs_gnn *net, float lr, float beta1, float beta2, float eps, int32_t t,
                        void *stream);

/* The network's dense-layer kernel on its own: C[M][N] = A B with A(m,k) =
 * A[m*sam + k*sak] and B(k,n) = B[k*sbk + n*sbn] (device f32, element strides),
 * both rounded to BF16, FP32 accumulation, C row stride ldc. */
afs_status afs_gnn_gemm_bf16(int32_t M, int32_t N, int32_t K, const float *A, int64_t sam, int64_t sak,
                             const float *B, int64_t sbk, int64_t sbn, float *C, int64_t ldc,
                             void *stream);

/* ---- Precision study: the two DFT forms (Sec. 2.1.2; Sec. 3.5) ----
 * Form A is the paper's evaluation: FE(y) = Re sum_m c_m prod_i (omega^m + y_i)
 * with c_m = (1/N) sum_j fhat_(k-j) omega^(-m j), N = k + 1, fhat_t the
 * Walsh-Fourier coefficient of a size-t literal set; its products span about 2^k
 * to eps^k near a corner, which limits it to k near 50 in FP64.  Form B is the
 * count basis of the library's FE kernels: FE(y) = Re sum_m d_m prod_i
 * (alpha_m + beta_m y_i) with alpha_m = (1 + omega^m)/2, beta_m = (1 - omega^m)/2
 * and d as afs_coefficients. */
typedef enum { AFS_FORM_A = 0, AFS_FORM_B = 1 } afs_form;

/* Tables of one constraint in either form: alpha, beta, d host double
 * [2(k+1)] as (re, im) pairs.  fhat_t is summed exactly in 128-bit integers and
 * divided by 2^k last (Sec. 3.5.1), so form A takes k <= 120. */
afs_status afs_form_tables(int32_t type, int32_t k, int32_t param, int32_t form, double *alpha,
                           double *beta, double *d);

/* FE(y) = Re sum_m d_m prod_i (alpha_m + beta_m y[i][b]) for b < B, one lane per
 * point with no rescaling, in FP32 (fp64 == 0: tables and y rounded to FP32
 * first) or FP64.  y: device f64 [k][B]; fe: device f64 [B].  An experiment
 * entry, not a hot-path one: it uploads the tables, allocates, and returns after
 * the stream has finished. */
afs_status afs_fe_generic(int32_t k, const double *alpha, const double *beta, const double *d, int32_t fp64,
                          int32_t B, const double *y, double *fe, int32_t device, void *stream);

/* ---- Input files (App. A) ----
 * DIMACS CNF and the hybrid symmetric-constraint format: an optional 'h' marker,
 * an optional type identifier (x/xor, n/nae, a/amo, e/eo, k/ek K, d/card T with
 * T = K (K > 0: at least K; K < 0: fewer than |K|) or >=K, >K, <K, <=K) and
 * literals, ended by 0; comment lines start with 'c' or '*'; text after a
 * constraint's 0 is a comment; "p cnf <vars> <constraints>" is optional.  CARD
 * thresholds are normalised to AFS_CARD_GE / AFS_CARD_LT and XOR to odd parity.
 * The simplifications of App. A are applied: one-literal OR and EO constraints
 * and CARD >= k / EK k over k literals fix their literals True, EK 0 fixes its
 * literals False, one-literal AMO and CARD >= 0 are dropped, CARD >= 1 becomes
 * OR and EK 1 becomes EO; fixing a variable both ways returns AFS_EUNSAT, as
 * does a threshold no assignment meets (CARD >= K or EK K with K above the
 * length, CARD < K with K <= 0).  CARD < K with K above the length is dropped,
 * and a plain threshold 0 reads as ">= 0".  The operator may stand apart from
 * its number ("d >= 2").  The fixed variables are returned as units (a partial
 * assignment, Sec. 3.4) and not propagated further. */
typedef struct afs_parsed afs_parsed;

typedef struct {
    int32_t n_vars;          /* from the problem line, else the largest variable */
    int32_t n_cons;          /* constraints kept                                  */
    int64_t n_lits;
    int32_t n_units;         /* variables fixed by the simplifications            */
    int32_t n_dropped;       /* constraints removed by the simplifications        */
    int32_t declared_cons;   /* constraint count of the problem line, -1 if none  */
} afs_parsed_info;

/* Parse len bytes of text, or the file at path.  On error *out is NULL and the
 * message (with the line number) is in afs_last_error(). */
afs_status afs_parse_text(const char *text, size_t len, afs_parsed **out);
afs_status afs_parse_file(const char *path, afs_parsed **out);
afs_status afs_parsed_get_info(const afs_parsed *p, afs_parsed_info *out);

/* Copy the kept constraints into host arrays sized from afs_parsed_get_info:
 * con_off int64 [n_cons+1], lits int32 [n_lits], types int32 [n_cons], params
 * int32 [n_cons] (the afs_instance_create arrays), and units int8 [n_vars]
 * (+1 fixed True, -1 fixed False, 0 free).  Any pointer may be NULL. */
afs_status afs_parsed_arrays(const afs_parsed *p, int64_t *con_off, int32_t *lits, int32_t *types,
                             int32_t *params, int8_t *units);
void afs_parsed_destroy(afs_parsed *p);

/* Unit folding (Sec. 3.4): write the parsed units into each of n_partial partial
 * assignments values (host i8 [n_partial][n_vars]: +1 True, -1 False, 0 free,
 * updated in place).  A unit that contradicts a partial assignment returns
 * AFS_EUNSAT naming the row and the variable (values is then unspecified).  With
 * no partial assignments of its own a caller passes one zero row and receives the
 * units as a partial assignment for every restart. */
afs_status afs_parsed_fold_units(const afs_parsed *p, int32_t n_partial, int8_t *values);

/* ---- Long-constraint decomposition (Sec. 5, constraint length ceiling) ----
 * The paper proposes replacing a long constraint by O(k / 50) shorter
 * constraints of the same type, for every type but EK and CARD.  Here a
 * constraint of type OR, XOR, NAE, AMO or EO longer than max_len becomes a chain
 * of p = ceil((k - 2) / (max_len - 2)) pieces of that type joined by p - 1 new
 * auxiliary variables a_1 .. a_(p-1):
 *   piece 1      : G_1 and a_1
 *   piece i      : -a_(i-1), G_i and a_i        (1 < i < p)
 *   piece p      : -a_(p-1) and G_p
 * where G_1 .. G_p split the literals in their order, the piece lengths differing
 * by at most one (every piece <= max_len, every G_i non-empty).  XOR pieces keep
 * the literal a_i in both neighbours instead (a_i is the parity so far), with
 * parity 0 for every piece but the last, which keeps the constraint's parity.
 * For every assignment of the original variables, the original constraint holds
 * exactly when some values of the auxiliary variables satisfy every piece.  EK,
 * CARD >= and CARD < constraints, and constraints of length <= max_len, are
 * copied unchanged.  Each piece keeps its constraint's weight.  Auxiliary
 * variables are numbered n+1, n+2, ... in the order of the constraints.
 * afs_decompose_size gives the sizes of the result (host arrays as for
 * afs_instance_create: con_off int64 [C+1], types int32 [C]; max_len in
 * [3, AFS_MAX_LEN]); afs_decompose writes it into caller arrays of those sizes:
 * con_off_out int64 [C_out+1], lits_out int32 [L_out], types_out and params_out
 * int32 [C_out], origin_out int32 [C_out] (the input constraint of each output
 * constraint), weights_out float [C_out] (written when weights is non-NULL;
 * may be NULL when weights is NULL).  Host-only, no device use; invalid input
 * (a type out of range, an empty constraint, a literal 0 or above n, sizes that
 * overflow int32) returns AFS_EINVAL and writes nothing. */
afs_status afs_decompose_size(int32_t n, int32_t C, const int64_t *con_off, const int32_t *types, int32_t max_len,
                              int32_t *n_out, int32_t *C_out, int64_t *L_out);
afs_status afs_decompose(int32_t n, int32_t C, const int64_t *con_off, const int32_t *lits, const int32_t *types,
                         const int32_t *params, const float *weights, int32_t max_len, int64_t *con_off_out,
                         int32_t *lits_out, int32_t *types_out, int32_t *params_out, float *weights_out,
                         int32_t *origin_out);

/* ---- evaluation without allocation -------------------------------------------------- */

/* For callers that cannot allocate device memory or pass a workspace (code under
 * HIP graph capture that must not call hipMalloc, tight serving loops, harnesses
 * that forbid allocation): afs_eval with a static scratch array of the library
 * in place of the workspace.  Outputs, their layout and the arithmetic are those
 * of afs_eval (same kernels, same order).
 *   The scratch is a device array of AFS_NOALLOC_SCRATCH_BYTES (64 MiB) per
 *   device, held from the library's first use on that device until the process
 *   ends.  The call allocates nothing and calls no allocating routine; it
 *   returns AFS_EINVAL (nothing launched) when the instance needs more scratch
 *   at B than that: afs_workspace_bytes-style sizing, the adjoint rows L x
 *   round_up(B, 64) floats plus the objective partials.  Every call on one
 *   device shares that device's array, which keeps the last call's contents:
 *   calls that overlap on one device (different streams or host threads) race
 *   and give wrong results; order them on one stream. */
#define AFS_NOALLOC_SCRATCH_BYTES (64ull << 20)
afs_status afs_eval_noalloc(afs_instance *inst, int32_t B, const float *x, float *obj, float *grad, float *fe,
                            float *adj, void *stream);

/* ---- peak probes (roofline denominators) ------------------------------------------ */

/* Small kernels that measure the device's attainable peaks for this build's
 * code, reported beside the published figures (HBM 8 TB/s, FP32 vector
 * 157.3 TFLOP/s, dense BF16 MFMA 2.5 PFLOP/s).  Each enqueues one launch of
 * `blocks` workgroups of 256 work-items on `stream` and returns at once; the
 * caller times it (HIP events on the same stream).  No allocation, no
 * synchronisation.  Invalid sizes or NULL pointers return AFS_EINVAL; a launch
 * failure AFS_EDEVICE.
 *
 * afs_probe_fma: every work-item runs 16 independent chains of `iters` plain
 *   FP32 operations (the library's kernels are built without packed FP32
 *   instructions, so these bound the issue rate of their arithmetic):
 *   variant 0 fused multiply-adds acc = acc * a + b with uniform a, b;
 *   variant 1 acc += x * y with per-lane x, y; variant 2 multiplies acc *= x;
 *   variant 3 the FE kernels' product step (r, i) <- (r - i z, i + r z) on 8
 *   complex chains; variant 4 acc = acc * x + y with per-lane x, y (the
 *   three-address form); variant 5 multiplies acc *= a with a uniform; variant 6
 *   acc += a * x with a uniform, x per lane.  out: device float [blocks * 256],
 *   one value per work-item.  *flops (host, may be NULL) = 2 (variants 2 and
 *   5: 1) * 16 * iters * blocks * 256.
 * afs_probe_mfma_bf16: every wave runs `iters` rounds of 8 independent
 *   16x16x32 BF16 matrix products with FP32 accumulation.  out as above;
 *   *flops = 2 * 16 * 16 * 32 * 8 * iters * blocks * 4.
 * afs_probe_copy: dst = src over `bytes` (a multiple of 16; both 16-byte
 *   aligned device pointers), 16-byte non-temporal loads and stores, grid-stride
 *   over `blocks` workgroups; reads and writes `bytes` each. */
afs_status afs_probe_fma(int32_t variant, int32_t blocks, int32_t iters, float *out, double *flops,
                         void *stream);
afs_status afs_probe_mfma_bf16(int32_t blocks, int32_t iters, float *out, double *flops, void *stream);
afs_status afs_probe_copy(const void *src, void *dst, int64_t bytes, int32_t blocks, void *stream);

/* Starting points for Algorithm 1 from the network's output (Sec. 3.3 takes
 * uniform random points; this is the learned alternative).  xhat, x0, out:
 * device f32 [n][B] (x0 the noise the network was given, xhat its output
 * tanh(z)); out may alias neither input.  The output is softened to tanh(z / T)
 * (T = temperature > 0); with sample != 0 every point keeps magnitude |x0| and
 * takes the sign of a draw from the softened marginal P(True) = (1 - tanh(z/T))/2
 * (True -> negative), u uniform on [0, 1) from Philox4x32-10 keyed by seed with
 * counter (b, v, 1, 0), u < P(True) meaning True; otherwise the point is
 * (1 - mix) tanh(z / T) + mix x0 (0 <= mix <= 1).  A non-finite network output
 * falls back to the uniform point x0.  Clamped to [-1, 1].  Enqueued on stream;
 * no allocation. */
afs_status afs_gnn_starts(int32_t n, int32_t B, const float *xhat, const float *x0, uint64_t seed, float temperature,
                          float mix, int32_t sample, float *out, void *stream);

/* Thread-local message for the last non-OK status of an afs_gnn_* call. */
const char *afs_gnn_last_error(void);

/* Thread-local message describing the last non-OK status. */
const char *afs_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* AFSAT_H */
