/*
 * oracle.c -- plain FP64 CPU oracle for the Accelerated Fourier SAT hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct
 * reference that the GPU library is checked against.  Only the test suite,
 * the smoke check and the benchmark's CPU-baseline leg may load it.  It shares
 * no code, headers, tables or helpers with the GPU library.
 *
 * What it computes (all in IEEE binary64):
 *   - orc_sat        : the truth predicate of each symmetric constraint type
 *                      (Table 1 and Table 2: OR, XOR, NAE, AMO, EO, EK, CARD,
 *                      with CARD normalised to ">=" or "<" as Appendix A
 *                      prescribes).
 *   - orc_eval       : the Walsh-Fourier expansion FE of every constraint at
 *                      real points y in [-1,1]^k (Sec. 2.1, Eq. 1), its
 *                      gradient, and the objective sum_c w_c FE_c (Sec. 2.1.1,
 *                      Eq. 2).  True is -1, False is +1 (Sec. 2.1).
 *   - orc_step       : the projected gradient step of Algorithm 1.
 *   - orc_verify     : rounding and the exact unsatisfied-constraint count of
 *                      Algorithm 1's outputs.
 *   - orc_pgd        : Algorithm 1 with a constant step length, FP64 end to end.
 *
 * How FE is computed.  For a symmetric constraint the expansion is the unique
 * multilinear polynomial that agrees with the truth value (+1 violated,
 * -1 satisfied) on every corner of the cube.  Evaluated at an interior point y
 * it equals the expectation of that truth value when literal i is true
 * independently with probability p_i = (1 - y_i)/2.  Because the truth value
 * depends only on the count T of true literals (Sec. 2.1), FE is
 *     FE = sum_t g(t) * Pr[T = t],
 * and Pr[T = t] is the elementary-symmetric-polynomial sequence that Sec. 2.1.2
 * builds by linear convolution of per-literal length-2 sequences; here each
 * literal contributes the sequence [1 - p_i, p_i] (the probability of being
 * false / true), and the convolution is carried out directly, literal by
 * literal -- no DFT.  All terms are non-negative, so the recursion is stable
 * at any length.
 *
 * The gradient is the exact reverse-mode adjoint of that recursion.
 *
 * Value convention: x in [-1,1], -1 = True.  A literal with a negative
 * DIMACS index has value y = -x.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { ORC_OR = 0, ORC_XOR = 1, ORC_NAE = 2, ORC_CARD_GE = 3, ORC_CARD_LT = 4,
       ORC_AMO = 5, ORC_EO = 6, ORC_EK = 7 };

/* Truth predicate of one constraint given t true literals out of k
 * (Table 1; Table 2; CARD normalisation in Appendix A).
 * Returns 1 if satisfied, 0 if violated, -1 for an unknown type. */
int orc_sat(int type, int k, int param, int t)
{
    switch (type) {
    case ORC_OR:      return t >= 1;
    case ORC_XOR:     return (t & 1) == (param & 1);   /* param 1: odd parity */
    case ORC_NAE:     return t > 0 && t < k;
    case ORC_CARD_GE: return t >= param;
    case ORC_CARD_LT: return t < param;
    case ORC_AMO:     return t <= 1;
    case ORC_EO:      return t == 1;
    case ORC_EK:      return t == param;
    default:          return -1;
    }
}

/* g(t): +1 if the constraint is violated with t true literals, -1 if
 * satisfied (True -> -1, Sec. 2.1). */
static double truth_value(int type, int k, int param, int t)
{
    return orc_sat(type, k, param, t) == 1 ? -1.0 : 1.0;
}

typedef struct {
    int n, C, B;
    const int64_t *con_off;
    const int32_t *lits, *types, *params;
    const double *weights;
    const double *x;          /* [n][B] */
    double *obj, *fe, *adj, *grad;
    int kmax;
    int b_begin, b_end;
    int status;
} eval_job;

/* FE and gradient of one constraint at one restart.
 * q holds the triangular table of Pr[T_i = t] for every prefix i (row i has
 * i+1 entries), lam is a work row of length k+1, dy receives dFE/dy_i. */
static double eval_one(int k, int type, int param, const double *y,
                       double *q, double *lam, double *dy)
{
    /* forward: q^(0) = [1]; q^(i)_t = (1-p_i) q^(i-1)_t + p_i q^(i-1)_{t-1} */
    q[0] = 1.0;
    size_t row = 0;                 /* start of row i-1 */
    for (int i = 1; i <= k; ++i) {
        const double p = 0.5 * (1.0 - y[i - 1]);
        const double *prev = q + row;
        double *cur = q + row + (size_t)i;   /* row i-1 has i entries */
        for (int t = 0; t <= i; ++t) {
            const double stay = (t < i) ? prev[t] : 0.0;
            const double move = (t > 0) ? prev[t - 1] : 0.0;
            cur[t] = (1.0 - p) * stay + p * move;
        }
        row += (size_t)i;
    }
    const double *qk = q + row;     /* row k, k+1 entries */
    double fe = 0.0;
    for (int t = 0; t <= k; ++t) {
        lam[t] = truth_value(type, k, param, t);
        fe += lam[t] * qk[t];
    }
    /* reverse: lam^(k) = g; for i = k..1:
     *   dFE/dp_i = sum_t q^(i-1)_t (lam^(i)_{t+1} - lam^(i)_t)
     *   lam^(i-1)_t = (1-p_i) lam^(i)_t + p_i lam^(i)_{t+1}
     * and dp_i/dy_i = -1/2. */
    for (int i = k; i >= 1; --i) {
        row -= (size_t)i;           /* start of row i-1 */
        const double *prev = q + row;
        const double p = 0.5 * (1.0 - y[i - 1]);
        double dp = 0.0;
        for (int t = 0; t < i; ++t)
            dp += prev[t] * (lam[t + 1] - lam[t]);
        dy[i - 1] = -0.5 * dp;
        for (int t = 0; t < i; ++t)
            lam[t] = (1.0 - p) * lam[t] + p * lam[t + 1];
    }
    return fe;
}

static void *eval_worker(void *arg)
{
    eval_job *J = (eval_job *)arg;
    const int k1 = J->kmax + 1;
    double *q = (double *)malloc(sizeof(double) * (size_t)k1 * (size_t)(k1 + 1) / 2 + sizeof(double));
    double *lam = (double *)malloc(sizeof(double) * (size_t)(k1 + 1));
    double *y = (double *)malloc(sizeof(double) * (size_t)k1);
    double *dy = (double *)malloc(sizeof(double) * (size_t)k1);
    if (!q || !lam || !y || !dy) {
        J->status = -3;
        free(q); free(lam); free(y); free(dy);
        return NULL;
    }
    const int B = J->B;
    for (int b = J->b_begin; b < J->b_end; ++b) {
        double obj = 0.0;
        for (int c = 0; c < J->C; ++c) {
            const int64_t o0 = J->con_off[c], o1 = J->con_off[c + 1];
            const int k = (int)(o1 - o0);
            for (int i = 0; i < k; ++i) {
                const int32_t l = J->lits[o0 + i];
                const int v = (l > 0 ? l : -l) - 1;
                const double xv = J->x[(size_t)v * B + b];
                y[i] = l > 0 ? xv : -xv;
            }
            const double w = J->weights ? J->weights[c] : 1.0;
            const double f = eval_one(k, J->types[c], J->params[c], y, q, lam, dy);
            obj += w * f;
            if (J->fe) J->fe[(size_t)c * B + b] = f;
            for (int i = 0; i < k; ++i) {
                const int32_t l = J->lits[o0 + i];
                const double a = w * (l > 0 ? dy[i] : -dy[i]);   /* dFE/dx_v */
                if (J->adj) J->adj[(size_t)(o0 + i) * B + b] = a;
                if (J->grad) {
                    const int v = (l > 0 ? l : -l) - 1;
                    J->grad[(size_t)v * B + b] += a;
                }
            }
        }
        if (J->obj) J->obj[b] = obj;
    }
    free(q); free(lam); free(y); free(dy);
    return NULL;
}

static int check_instance(int n, int C, const int64_t *con_off, const int32_t *lits,
                          const int32_t *types, int *kmax)
{
    if (n < 0 || C < 0 || !con_off || (C > 0 && (!lits || !types))) return -1;
    if (con_off[0] != 0) return -1;
    int km = 0;
    for (int c = 0; c < C; ++c) {
        const int64_t k = con_off[c + 1] - con_off[c];
        if (k < 1 || k > 1000000) return -1;
        if (types[c] < 0 || types[c] > 7) return -1;
        if (k > km) km = (int)k;
        for (int64_t i = con_off[c]; i < con_off[c + 1]; ++i) {
            const int32_t l = lits[i];
            if (l == 0 || l > n || l < -n) return -1;
        }
    }
    *kmax = km;
    return 0;
}

/*
 * FE, objective and gradient at B points (Sec. 2.1 Eq. 1; Sec. 2.1.1 Eq. 2).
 *   x      : [n][B] FP64 values in [-1,1], restart index contiguous
 *   obj    : [B]      sum_c w_c FE_c                      (may be NULL)
 *   fe     : [C][B]   FE_c                                (may be NULL)
 *   adj    : [L][B]   w_c * dFE_c/dx_v for each literal occurrence, in the
 *                      input literal order                 (may be NULL)
 *   grad   : [n][B]   dF/dx (zeroed here)                  (may be NULL)
 * Returns 0, -1 on an invalid instance, -3 on allocation failure.
 */
int orc_eval(int n, int C, const int64_t *con_off, const int32_t *lits,
             const int32_t *types, const int32_t *params, const double *weights,
             int B, const double *x, double *obj, double *fe, double *adj,
             double *grad, int nthreads)
{
    int kmax = 0;
    if (B < 0 || check_instance(n, C, con_off, lits, types, &kmax)) return -1;
    if (grad) memset(grad, 0, sizeof(double) * (size_t)n * (size_t)B);
    if (B == 0) return 0;
    if (nthreads < 1) nthreads = 1;
    if (nthreads > B) nthreads = B;
    eval_job *jobs = (eval_job *)calloc((size_t)nthreads, sizeof(eval_job));
    pthread_t *th = (pthread_t *)calloc((size_t)nthreads, sizeof(pthread_t));
    if (!jobs || !th) { free(jobs); free(th); return -3; }
    for (int j = 0; j < nthreads; ++j) {
        eval_job *J = &jobs[j];
        J->n = n; J->C = C; J->B = B; J->con_off = con_off; J->lits = lits;
        J->types = types; J->params = params; J->weights = weights; J->x = x;
        J->obj = obj; J->fe = fe; J->adj = adj; J->grad = grad; J->kmax = kmax;
        J->b_begin = (int)((int64_t)B * j / nthreads);
        J->b_end = (int)((int64_t)B * (j + 1) / nthreads);
    }
    char *started = (char *)calloc((size_t)nthreads, 1);
    if (!started) { free(jobs); free(th); return -3; }
    for (int j = 1; j < nthreads; ++j)
        started[j] = pthread_create(&th[j], NULL, eval_worker, &jobs[j]) == 0;
    eval_worker(&jobs[0]);
    int status = jobs[0].status;
    for (int j = 1; j < nthreads; ++j) {
        if (started[j]) pthread_join(th[j], NULL);
        else eval_worker(&jobs[j]);           /* thread did not start: run inline */
        if (jobs[j].status) status = jobs[j].status;
    }
    free(started);
    free(jobs); free(th);
    return status;
}

/* Projected gradient step of Algorithm 1 with a constant step length:
 *   x' = projectToBounds(x - lr * grad) = min(1, max(-1, x - lr * grad)),
 * leaving fixed variables (partial assignment, Sec. 3.4: zero gradient) and
 * finished restarts (Sec. 3.3: converged candidates do no-ops) unchanged. */
void orc_step(int n, int B, const double *x, const double *grad, double lr,
              const uint8_t *fixed, const uint8_t *done, double *xout)
{
    for (int v = 0; v < n; ++v)
        for (int b = 0; b < B; ++b) {
            const size_t i = (size_t)v * B + b;
            double xv = x[i];
            if (!(fixed && fixed[v]) && !(done && done[b])) {
                xv = xv - lr * grad[i];
                if (xv > 1.0) xv = 1.0;
                if (xv < -1.0) xv = -1.0;
            }
            xout[i] = xv;
        }
}

/* Rounding and unsat_count of Algorithm 1, on FP32 points.
 * A variable rounds to True iff x < 0 (so +0 and -0 are both False); a
 * literal is true iff its variable's truth differs from the literal's
 * negation flag; each constraint is judged by its exact integer predicate.
 *   bits  : [n][ceil(B/32)] bit (b mod 32) of word b/32 = (x[v][b] < 0)  (may be NULL)
 *   unsat : [B] number of violated constraints */
int orc_verify(int n, int C, const int64_t *con_off, const int32_t *lits,
               const int32_t *types, const int32_t *params, int B, const float *x,
               int32_t *unsat, uint32_t *bits)
{
    int kmax;
    if (B < 0 || check_instance(n, C, con_off, lits, types, &kmax)) return -1;
    const int W = (B + 31) / 32;
    if (bits) {
        memset(bits, 0, sizeof(uint32_t) * (size_t)n * (size_t)W);
        for (int v = 0; v < n; ++v)
            for (int b = 0; b < B; ++b)
                if (x[(size_t)v * B + b] < 0.0f)
                    bits[(size_t)v * W + b / 32] |= 1u << (b % 32);
    }
    for (int b = 0; b < B; ++b) {
        int32_t u = 0;
        for (int c = 0; c < C; ++c) {
            const int64_t o0 = con_off[c], o1 = con_off[c + 1];
            int t = 0;
            for (int64_t i = o0; i < o1; ++i) {
                const int32_t l = lits[i];
                const int v = (l > 0 ? l : -l) - 1;
                const int var_true = x[(size_t)v * B + b] < 0.0f;
                const int neg = l < 0;
                t += var_true ^ neg;
            }
            if (orc_sat(types[c], (int)(o1 - o0), params[c], t) != 1) ++u;
        }
        unsat[b] = u;
    }
    return 0;
}

/* Same rounding and count on FP64 points (for the oracle's own PGD). */
static int32_t unsat_count_f64(int C, const int64_t *con_off, const int32_t *lits,
                               const int32_t *types, const int32_t *params,
                               int B, const double *x, int b)
{
    int32_t u = 0;
    for (int c = 0; c < C; ++c) {
        int t = 0;
        for (int64_t i = con_off[c]; i < con_off[c + 1]; ++i) {
            const int32_t l = lits[i];
            const int v = (l > 0 ? l : -l) - 1;
            t += (x[(size_t)v * B + b] < 0.0) ^ (l < 0);
        }
        if (orc_sat(types[c], (int)(con_off[c + 1] - con_off[c]), params[c], t) != 1) ++u;
    }
    return u;
}

/*
 * Algorithm 1 (projected gradient descent) with eta = lr constant, in FP64.
 * The initial point is checked first; then for t = 1..steps a step is taken
 * from the gradient at X_(t-1), projected, and X_(t) is checked.  A restart
 * that verifies is frozen (its later steps are no-ops).
 *   x        : [n][B] in: X_(0); out: final point
 *   unsat    : [B] unsatisfied count at the final point
 *   first_sat: [B] first t at which the restart verified, or -1
 *   obj      : [B] objective at the final point (may be NULL)
 */
int orc_pgd(int n, int C, const int64_t *con_off, const int32_t *lits,
            const int32_t *types, const int32_t *params, const double *weights,
            int B, double *x, double lr, int steps, const uint8_t *fixed,
            int32_t *unsat, int32_t *first_sat, double *obj, int nthreads)
{
    int kmax;
    if (B < 0 || steps < 0 || check_instance(n, C, con_off, lits, types, &kmax)) return -1;
    const size_t nb = (size_t)n * (size_t)B;
    double *grad = (double *)malloc(sizeof(double) * (nb ? nb : 1));
    double *xn = (double *)malloc(sizeof(double) * (nb ? nb : 1));
    uint8_t *done = (uint8_t *)calloc((size_t)(B ? B : 1), 1);
    if (!grad || !xn || !done) { free(grad); free(xn); free(done); return -3; }
    for (int b = 0; b < B; ++b) {
        first_sat[b] = -1;
        if (unsat_count_f64(C, con_off, lits, types, params, B, x, b) == 0) {
            done[b] = 1; first_sat[b] = 0;
        }
    }
    int rc = 0;
    for (int t = 1; t <= steps; ++t) {
        int all = 1;
        for (int b = 0; b < B; ++b) all &= done[b];
        if (all) break;
        rc = orc_eval(n, C, con_off, lits, types, params, weights, B, x, NULL, NULL,
                      NULL, grad, nthreads);
        if (rc) break;
        orc_step(n, B, x, grad, lr, fixed, done, xn);
        memcpy(x, xn, sizeof(double) * nb);
        for (int b = 0; b < B; ++b)
            if (!done[b] && unsat_count_f64(C, con_off, lits, types, params, B, x, b) == 0) {
                done[b] = 1; first_sat[b] = t;
            }
    }
    if (!rc) {
        for (int b = 0; b < B; ++b)
            unsat[b] = unsat_count_f64(C, con_off, lits, types, params, B, x, b);
        if (obj)
            rc = orc_eval(n, C, con_off, lits, types, params, weights, B, x, obj, NULL,
                          NULL, NULL, nthreads);
    }
    free(grad); free(xn); free(done);
    return rc;
}
