// search_kernels.hip -- backtracking line search (Algorithm 1's lineSearch with
// a maximum step s) and seeded starting points (Sec. 3.4) for gfx950 (wave64).
//
// One iteration of the search, per restart b (all restarts in lockstep, the ones
// that have decided doing no-ops):
//   f0 = F(x), g = grad F(x);  eta = s
//   trial j = 0..T-1:  xt = clip(x - eta g)   (fixed variables held)
//                      accept when F(xt) <= f0 + c <g, xt - x>   (Armijo along
//                      the projection arc), else eta *= beta
//   no trial accepted: eta = 0 (no step)
//   x = clip(x - eta g)
// The objective sums are fixed-order reductions (the same two-pass reduction as
// the objective), so every decision is deterministic.  The trials' FE passes skip
// every wave whose restarts have all decided; the objective partials of those
// restarts then hold stale values, which the test never reads.
//
// Layouts: x, g, xt [n][B] f32; per-restart vectors [B] (padded to Bp).

#include "kernels.hpp"

#include "device_common.hpp"
#include "philox.hpp"

namespace afs {

namespace {

using namespace dev;

__device__ __forceinline__ float clip_step(float xv, float g, float eta)
{
    float t = xv - eta * g;
    t = t > 1.0f ? 1.0f : t;
    t = t < -1.0f ? -1.0f : t;
    return t;
}

struct TrialArgs {
    const float *x, *g, *eta;
    const uint8_t *acc, *fixed;
    float *xt, *dot_part;
    int n, n_partial, B, Bp, nchunks;
    int64_t items, item0;
};

// one wave per (tile of kTrialVars variables, 64 restarts), one restart per lane
__global__ __launch_bounds__(kBlock) void trial_kernel(TrialArgs A)
{
    const int64_t item = A.item0 + (int64_t)blockIdx.x * kWavesPerBlock + wave_id();
    if (item >= A.items) return;
    const int tile = (int)(item / A.nchunks), chunk = (int)(item % A.nchunks);
    const int b = chunk * kWave + (threadIdx.x & 63);
    float dot = 0.0f;
    if (b < A.B && !A.acc[b]) {
        const float eb = A.eta[b];
        const int v0 = tile * kTrialVars;
        const int v1 = v0 + kTrialVars < A.n ? v0 + kTrialVars : A.n;
        for (int v = v0; v < v1; ++v) {
            const int64_t at = (int64_t)v * A.B + b;
            const float xv = A.x[at];
            float t = xv;
            if (!is_fixed(A.fixed, A.n_partial, A.n, A.B, v, b)) {
                const float gv = A.g[at];
                t = clip_step(xv, gv, eb);
                dot += gv * (t - xv);
            }
            A.xt[at] = t;
        }
    }
    A.dot_part[(int64_t)tile * A.Bp + b] = dot;
}

__global__ __launch_bounds__(kBlock) void search_init_kernel(int B, float step, const uint8_t *done, float *eta,
                                                             uint8_t *acc)
{
    const int b = blockIdx.x * kBlock + threadIdx.x;
    if (b >= B) return;
    eta[b] = step;
    acc[b] = (done && done[b]) ? 1 : 0;
}

__global__ __launch_bounds__(kBlock) void accept_kernel(int B, const float *f0, const float *ft, const float *dot,
                                                        float c, float beta, int last, float *eta, uint8_t *acc)
{
    const int b = blockIdx.x * kBlock + threadIdx.x;
    if (b >= B || acc[b]) return;
    if (ft[b] <= f0[b] + c * dot[b]) {
        acc[b] = 1;
    } else if (last) {
        eta[b] = 0.0f;
        acc[b] = 1;
    } else {
        eta[b] *= beta;
    }
}

struct StepArgs {
    float *x;
    const float *g, *eta;
    const uint8_t *fixed, *done;
    const int32_t *var_inst;
    uint32_t *bits;
    int32_t *unsat;
    uint8_t *moved;              // [n_inst][B]: set where some variable moves by >= eps (NULL: not tracked)
    float eps;
    int n, n_partial, n_inst, B, W, nchunks;
    int64_t items, item0;
};

constexpr int kStepRestarts = 4;
constexpr int kStepChunk = kWave * kStepRestarts;

template <int CTRL>
__device__ __forceinline__ uint32_t dpp_u(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, CTRL, 0xF, 0xF, false);
}

// one wave per (variable, 256 restarts), four consecutive restarts per lane; the
// rounded bits of eight lanes form one 32-bit word (row shifts inside a row)
__global__ __launch_bounds__(kBlock) void search_step_kernel(StepArgs A)
{
    const int64_t item = A.item0 + (int64_t)blockIdx.x * kWavesPerBlock + wave_id();
    if (item >= A.items) return;
    const int v = (int)(item / A.nchunks), chunk = (int)(item % A.nchunks);
    const int lane = threadIdx.x & 63;
    const int b0 = chunk * kStepChunk + lane * kStepRestarts;
    const uint8_t *done = A.done ? A.done + (int64_t)A.var_inst[v] * A.B : nullptr;
    uint32_t nib = 0;
#pragma unroll
    for (int e = 0; e < kStepRestarts; ++e) {
        const int b = b0 + e;
        if (b < A.B) {
            const int64_t at = (int64_t)v * A.B + b;
            float xv = A.x[at];
            if (!is_fixed(A.fixed, A.n_partial, A.n, A.B, v, b) && !(done && done[b])) {
                const float x0 = xv;
                xv = clip_step(xv, A.g[at], A.eta[b]);
                A.x[at] = xv;
                // several variables may store 1 into one flag: every store writes the same value
                if (A.moved && fabsf(xv - x0) >= A.eps) A.moved[(int64_t)A.var_inst[v] * A.B + b] = 1;
            }
            if (v < A.n_inst) A.unsat[(int64_t)v * A.B + b] = 0;
            nib |= (xv < 0.0f ? 1u : 0u) << e;
        }
    }
    uint32_t t = nib | (dpp_u<0x101>(nib) << 4);   // row_shl:1
    t |= dpp_u<0x102>(t) << 8;                     // row_shl:2
    t |= dpp_u<0x104>(t) << 16;                    // row_shl:4
    const int w = chunk * (kStepChunk / 32) + (lane >> 3);
    if ((lane & 7) == 0 && w < A.W) A.bits[(int64_t)v * A.W + w] = t;
}

__global__ __launch_bounds__(kBlock) void init_points_kernel(int n, int B, uint32_t k0, uint32_t k1,
                                                             const int8_t *values, int n_partial, float *x,
                                                             int nchunks, int64_t items, int64_t item0)
{
    const int64_t item = item0 + (int64_t)blockIdx.x * kWavesPerBlock + wave_id();
    if (item >= items) return;
    const int v = (int)(item / nchunks), chunk = (int)(item % nchunks);
    const int b = chunk * kWave + (threadIdx.x & 63);
    if (b >= B) return;
    int val = 0;
    if (values) {
        const int p = n_partial > 1 ? (int)(((int64_t)b * n_partial) / B) : 0;
        val = values[(int64_t)p * n + v];
    }
    float out;
    if (val > 0) {
        out = -1.0f;
    } else if (val < 0) {
        out = 1.0f;
    } else {
        const U4 r = philox4x32_10(U4{(uint32_t)b, (uint32_t)v, 0u, 0u}, k0, k1);
        out = philox_pm1(r.x);          // top 24 bits: a multiple of 2^-23 in [-1, 1)
    }
    x[(int64_t)v * B + b] = out;
}

}  // namespace

hipError_t launch_trial(const DevInstance &I, int B, int Bp, const float *x, const float *g, const float *eta,
                        const uint8_t *acc, const uint8_t *fixed, int n_partial, float *xt, float *dot_part,
                        hipStream_t s)
{
    if (B == 0 || I.n == 0) return hipSuccess;
    TrialArgs a{};
    a.x = x; a.g = g; a.eta = eta; a.acc = acc; a.fixed = fixed; a.xt = xt; a.dot_part = dot_part;
    a.n = I.n; a.n_partial = n_partial; a.B = B; a.Bp = Bp;
    a.nchunks = Bp / kWave;
    const int tiles = (I.n + kTrialVars - 1) / kTrialVars;
    a.items = (int64_t)tiles * a.nchunks;
    return for_launch_chunks(a.items, [&](int64_t first, int64_t count) {
        a.item0 = first;
        hipLaunchKernelGGL(trial_kernel, grid_for_waves(count), dim3(kBlock), 0, s, a);
    });
}

hipError_t launch_search_init(int B, float step, const uint8_t *done, float *eta, uint8_t *acc, hipStream_t s)
{
    if (B == 0) return hipSuccess;
    hipLaunchKernelGGL(search_init_kernel, dim3((B + kBlock - 1) / kBlock), dim3(kBlock), 0, s, B, step, done,
                       eta, acc);
    return hipGetLastError();
}

hipError_t launch_accept(int B, const float *f0, const float *ft, const float *dot, float c, float beta,
                         bool last, float *eta, uint8_t *acc, hipStream_t s)
{
    if (B == 0) return hipSuccess;
    hipLaunchKernelGGL(accept_kernel, dim3((B + kBlock - 1) / kBlock), dim3(kBlock), 0, s, B, f0, ft, dot, c, beta,
                       last ? 1 : 0, eta, acc);
    return hipGetLastError();
}

hipError_t launch_search_step(const DevInstance &I, int B, float *x, const float *g, const float *eta,
                              const uint8_t *fixed, int n_partial, const uint8_t *done, uint32_t *bits,
                              int32_t *unsat, hipStream_t s, uint8_t *moved, float eps)
{
    if (B == 0) return hipSuccess;
    StepArgs a{};
    a.x = x; a.g = g; a.eta = eta; a.fixed = fixed; a.done = done; a.var_inst = I.var_inst;
    a.bits = bits; a.unsat = unsat; a.moved = moved; a.eps = eps;
    a.n = I.n; a.n_partial = n_partial; a.n_inst = I.n_inst; a.B = B; a.W = (B + 31) / 32;
    a.nchunks = (B + kStepChunk - 1) / kStepChunk;
    a.items = (int64_t)I.n * a.nchunks;
    return for_launch_chunks(a.items, [&](int64_t first, int64_t count) {
        a.item0 = first;
        hipLaunchKernelGGL(search_step_kernel, grid_for_waves(count), dim3(kBlock), 0, s, a);
    });
}

hipError_t launch_init_points(int n, int B, uint64_t seed, const int8_t *values, int n_partial, float *x,
                              hipStream_t s)
{
    if (B == 0 || n == 0) return hipSuccess;
    const int nchunks = (B + kWave - 1) / kWave;
    const int64_t items = (int64_t)n * nchunks;
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    return for_launch_chunks(items, [&](int64_t first, int64_t count) {
        hipLaunchKernelGGL(init_points_kernel, grid_for_waves(count), dim3(kBlock), 0, s, n, B, k0, k1, values,
                           n_partial, x, nchunks, items, first);
    });
}

}  // namespace afs
