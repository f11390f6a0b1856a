// gnn.hip -- learned initialisation: a message-passing network over the
// variable-constraint graph of an instance, with hand-written forward,
// backward, loss and optimiser kernels for gfx950.
//
// Network (hidden width H = 64, input features F = 16, R rounds):
//   hv = relu(fv Wv0 + bv0)                 fv [n][F]   variable features
//   hc = relu(fc Wc0 + bc0)                 fc [C][F]   constraint features
//   round r = 1..R:
//     ac = agg_c(hv)     ac_c = (1/k_c)   sum_{literals e of c} s_e hv_{v(e)}
//     hc = relu([hc, ac] U_r + bu_r)        U_r [2H][H]
//     av = agg_v(hc)     av_v = (1/deg_v) sum_{occurrences e of v} s_e hc_{c(e)}
//     hv = relu([hv, av] V_r + bv_r)        V_r [2H][H]
//   head, per restart b:  u = relu(hv Wh + bh + x0_{v,b} wx),  z = u . wo + bo,
//                         xhat_{v,b} = tanh(z)
// (s_e = +1 for a positive literal, -1 for a negated one.)  Dense layers run on
// BF16 MFMA with FP32 accumulation: both operands are rounded to BF16 (nearest
// even) as they are loaded.  The head has one scalar input per restart, so it is
// an elementwise kernel (restart-independent part hv Wh + bh computed once).
//
// Training target: a Boolean assignment t_v (True = 1) per instance.  With
// P(v True) = (1 - xhat)/2 = sigmoid(-2z) the loss is the mean binary
// cross-entropy over (v, b):  y softplus(2z) + (1-y) softplus(-2z).
// All reductions run in a fixed order (no float atomics).

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "afsat.h"
#include "instance.hpp"
#include "philox.hpp"

namespace afs {
namespace gnn {

constexpr int H = 64;
constexpr int F = 16;
constexpr int kBlock = 256;

typedef short short4v __attribute__((ext_vector_type(4)));
typedef float float4v __attribute__((ext_vector_type(4)));

// FP32 -> BF16 bits, round to nearest even (NaN kept quiet).
__device__ __forceinline__ short to_bf16(float f)
{
    unsigned u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u) return (short)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
    u += 0x7fffu + ((u >> 16) & 1u);
    return (short)(u >> 16);
}

// ---------------------------------------------------------------------------
// C(m,n) = sum_k A(m,k) B(k,n) on v_mfma_f32_16x16x16_bf16 tiles.
//   A(m,k) = k < ksplit ? a1[m*sam + k*sak] : a2[m*sam + (k-ksplit)*sak]
//   B(k,n) = b[k*sbk + n*sbn]
//   out    = C(m,n) (+ out if accumulate) (+ bias[n]) (relu if set), written to
//            c[split * split_stride + m*ldc + n]; split = blockIdx.y covers
//            k in [split*kchunk, (split+1)*kchunk).
// Each wave owns one 16x16 output tile.  Lane l feeds row/column l%16 and the
// four k values 4*(l/16)..+3 of each 16-wide k step, and receives rows
// 4*(l/16)..+3 of column l%16 of the result.
// ---------------------------------------------------------------------------
struct GemmArgs {
    const float *a1, *a2;
    int64_t sam, sak;
    int ksplit;
    const float *b;
    int64_t sbk, sbn;
    float *c;
    int64_t ldc, split_stride;
    const float *bias;
    int relu, accumulate;
    int M, N, K, kchunk;
    int rtw;                     // layer-shape path: row tiles per wave
};

__global__ __launch_bounds__(kBlock) void gemm_bf16_kernel(GemmArgs g)
{
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int tiles_n = (g.N + 15) / 16;
    const int64_t tiles = (int64_t)((g.M + 15) / 16) * tiles_n;
    const int64_t tile = (int64_t)blockIdx.x * (kBlock / 64) + wave;
    if (tile >= tiles) return;
    const int tm = (int)(tile / tiles_n), tn = (int)(tile % tiles_n);
    const int arow = tm * 16 + (lane & 15);
    const int bcol = tn * 16 + (lane & 15);
    const int kq = (lane >> 4) * 4;
    const int k0 = blockIdx.y * g.kchunk;
    const int k1 = min(g.K, k0 + g.kchunk);
    float4v acc = {0.f, 0.f, 0.f, 0.f};
    for (int kb = k0; kb < k1; kb += 16) {
        short4v av, bv;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int k = kb + kq + i;
            float a = 0.f, bb = 0.f;
            if (arow < g.M && k < k1)
                a = k < g.ksplit ? g.a1[arow * g.sam + k * g.sak] : g.a2[arow * g.sam + (k - g.ksplit) * g.sak];
            if (bcol < g.N && k < k1) bb = g.b[k * g.sbk + bcol * g.sbn];
            av[i] = to_bf16(a);
            bv[i] = to_bf16(bb);
        }
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, acc, 0, 0, 0);
    }
    const int ocol = tn * 16 + (lane & 15);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int orow = tm * 16 + (lane >> 4) * 4 + i;
        if (orow < g.M && ocol < g.N) {
            float *dst = g.c + (int64_t)blockIdx.y * g.split_stride + (int64_t)orow * g.ldc + ocol;
            float v = acc[i];
            if (g.accumulate) v += *dst;
            if (g.bias) v += g.bias[ocol];
            if (g.relu) v = fmaxf(v, 0.f);
            *dst = v;
        }
    }
}

// ---------------------------------------------------------------------------
// The same product for the network's layer shapes (N = 64 output columns,
// K = 16 * KSTEPS <= 128, A rows contiguous in k, one k chunk): B is rounded to
// BF16 once per block and kept in LDS (transposed, so that a lane's four k
// values are one 8-byte read), and each wave produces whole 16 x 64 slabs --
// four MFMA tiles sharing one A fragment -- for rtw consecutive row tiles,
// so A is read once with 16-byte loads, the next row tile's loads in flight
// while the current one is multiplied and stored.  Every output tile sees the same MFMA
// sequence as in gemm_bf16_kernel (k steps in ascending order), so the results
// are identical.
// ---------------------------------------------------------------------------
constexpr int kMaxRowTiles = 16;
constexpr int kBtPad = 8;            // shorts of padding per LDS row (bank spread)

template <int KSTEPS>
__device__ __forceinline__ void load_row_tile(const GemmArgs &g, int64_t tm, int lane, bool vec, float (&av)[KSTEPS][4])
{
    const int arow = (int)(tm * 16) + (lane & 15);
    const int kq = (lane >> 4) * 4;
#pragma unroll
    for (int s = 0; s < KSTEPS; ++s) {
        const int k = s * 16 + kq;
        const float *src = k < g.ksplit ? g.a1 + (int64_t)arow * g.sam + k
                                        : g.a2 + (int64_t)arow * g.sam + (k - g.ksplit);
        if (tm * 16 >= g.M || arow >= g.M) {
            av[s][0] = av[s][1] = av[s][2] = av[s][3] = 0.f;
        } else if (vec) {                            // read once: do not keep it in the caches
            const float4v v = __builtin_nontemporal_load(reinterpret_cast<const float4v *>(src));
            av[s][0] = v[0]; av[s][1] = v[1]; av[s][2] = v[2]; av[s][3] = v[3];
        } else {
#pragma unroll
            for (int i = 0; i < 4; ++i) av[s][i] = src[i];
        }
    }
}

template <int KSTEPS>
__global__ __launch_bounds__(kBlock) void gemm_rows64_kernel(GemmArgs g)
{
    constexpr int K = 16 * KSTEPS;
    constexpr int LD = K + kBtPad;
    __shared__ short bt[H * LD];                      // bt[n][k] = bf16(B(k, n))
    __shared__ float cs[kBlock / 64][16][H + 4];      // one 16 x 64 result slab per wave
    for (int t = threadIdx.x; t < K * H; t += kBlock) {
        const int k = t / H, n = t % H;
        bt[n * LD + k] = to_bf16(g.b[k * g.sbk + n * g.sbn]);
    }
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int kq = (lane >> 4) * 4;
    const bool vec = (g.sam % 4 == 0) && ((reinterpret_cast<uintptr_t>(g.a1) | reinterpret_cast<uintptr_t>(g.a2)) % 16 == 0);
    const bool vec_out = g.ldc % 4 == 0 && reinterpret_cast<uintptr_t>(g.c) % 16 == 0;
    const int c4 = (lane & 15) * 4;
    float4 bias4 = make_float4(0.f, 0.f, 0.f, 0.f);
    if (g.bias) bias4 = make_float4(g.bias[c4], g.bias[c4 + 1], g.bias[c4 + 2], g.bias[c4 + 3]);
    const int64_t tm0 = ((int64_t)blockIdx.x * (kBlock / 64) + wave) * g.rtw;
    float av[KSTEPS][4], an[KSTEPS][4];
    load_row_tile<KSTEPS>(g, tm0, lane, vec, av);
    for (int rt = 0; rt < g.rtw; ++rt) {
        const int64_t tm = tm0 + rt;
        if (tm * 16 >= g.M) break;                    // wave-uniform
        // the next row tile's loads are in flight while this one is multiplied and stored
        if (rt + 1 < g.rtw) load_row_tile<KSTEPS>(g, tm + 1, lane, vec, an);
        float4v acc[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) acc[t] = float4v{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int s = 0; s < KSTEPS; ++s) {
            short4v a;
#pragma unroll
            for (int i = 0; i < 4; ++i) a[i] = to_bf16(av[s][i]);
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const short4v b = *reinterpret_cast<const short4v *>(&bt[(t * 16 + (lane & 15)) * LD + s * 16 + kq]);
                acc[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc[t], 0, 0, 0);
            }
        }
        // through LDS, so that lane l writes columns 4(l%16)..+3 of rows 4q + l/16:
        // each store instruction then covers four whole 256-byte rows
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int i = 0; i < 4; ++i) cs[wave][(lane >> 4) * 4 + i][t * 16 + (lane & 15)] = acc[t][i];
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int r = q * 4 + (lane >> 4);
            const int64_t orow = tm * 16 + r;
            if (orow < g.M) {
                float *dst = g.c + orow * g.ldc + c4;
                // the general kernel's epilogue: accumulate, bias, relu, in that order
                float w[4];
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    w[e] = cs[wave][r][c4 + e];
                    if (g.accumulate) w[e] += dst[e];
                }
                if (g.bias) { w[0] += bias4.x; w[1] += bias4.y; w[2] += bias4.z; w[3] += bias4.w; }
                if (g.relu)
#pragma unroll
                    for (int e = 0; e < 4; ++e) w[e] = fmaxf(w[e], 0.f);
                if (vec_out) {                                  // written once, read by a later kernel
                    __builtin_nontemporal_store(float4v{w[0], w[1], w[2], w[3]}, reinterpret_cast<float4v *>(dst));
                } else {
#pragma unroll
                    for (int e = 0; e < 4; ++e) dst[e] = w[e];
                }
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");   // the slab is rewritten next
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
        for (int s = 0; s < KSTEPS; ++s)
#pragma unroll
            for (int i = 0; i < 4; ++i) av[s][i] = an[s][i];
    }
}

// out[i][j] (ld_out) (+)= sum_s part[s][i][j] (fixed order), for i < rows, j < cols
__global__ __launch_bounds__(kBlock) void sum_splits_kernel(const float *part, int splits, int64_t split_stride,
                                                             int rows, int cols, float *out, int64_t ld_out,
                                                             int accumulate)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)rows * cols) return;
    const int i = (int)(t / cols), j = (int)(t % cols);
    float s = 0.f;
    for (int q = 0; q < splits; ++q) s += part[q * split_stride + (int64_t)i * cols + j];
    float *d = out + (int64_t)i * ld_out + j;
    *d = accumulate ? *d + s : s;
}

// ---------------------------------------------------------------------------
// Graph aggregations (one wave per destination row, lane = feature, H = 64).
// agg_c : dst_c (+)= sum_{e in c} s_e w_e src_{v(e)},  w_e = inv_k[c] or inv_deg[v(e)]
// agg_v : dst_v (+)= sum_{e of v} s_e w_e src_{c(e)},  w_e = inv_deg[v] or inv_k[c(e)]
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void agg_c_kernel(const int32_t *con_off, const int32_t *lits,
                                                       const float *inv_k, const float *inv_deg, int by_dst,
                                                       const float *src, int64_t ld_src, float *dst,
                                                       int64_t ld_dst, int C, int accumulate)
{
    const int c = blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
    if (c >= C) return;
    const int j = threadIdx.x & 63;
    float s = 0.f;
    for (int e = con_off[c]; e < con_off[c + 1]; ++e) {
        const int l = lits[e];
        const int v = (l > 0 ? l : -l) - 1;
        const float w = by_dst ? 1.0f : inv_deg[v];
        const float x = src[(int64_t)v * ld_src + j] * w;
        s += l > 0 ? x : -x;
    }
    if (by_dst) s *= inv_k[c];
    float *d = dst + (int64_t)c * ld_dst + j;
    *d = accumulate ? *d + s : s;
}

__global__ __launch_bounds__(kBlock) void agg_v_kernel(const int32_t *var_off, const int32_t *var_con,
                                                       const float *var_sgn, const float *inv_k,
                                                       const float *inv_deg, int by_dst, const float *src,
                                                       int64_t ld_src, float *dst, int64_t ld_dst, int n,
                                                       int accumulate)
{
    const int v = blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
    if (v >= n) return;
    const int j = threadIdx.x & 63;
    float s = 0.f;
    for (int e = var_off[v]; e < var_off[v + 1]; ++e) {
        const int c = var_con[e];
        const float w = by_dst ? 1.0f : inv_k[c];
        s += var_sgn[e] * (src[(int64_t)c * ld_src + j] * w);
    }
    if (by_dst) s *= inv_deg[v];
    float *d = dst + (int64_t)v * ld_dst + j;
    *d = accumulate ? *d + s : s;
}

// dpre[i][j] = h[i][j] > 0 ? dh[i][j] : 0   (rows x H)
__global__ __launch_bounds__(kBlock) void relu_grad_kernel(const float *dh, int64_t ld_dh, const float *h,
                                                           int64_t ld_h, float *dpre, int rows)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)rows * H) return;
    const int i = (int)(t / H), j = (int)(t % H);
    dpre[t] = h[(int64_t)i * ld_h + j] > 0.f ? dh[(int64_t)i * ld_dh + j] : 0.f;
}

// column sums of a rows x H matrix: pass 1 per chunk of 256 rows, pass 2 fixed order
__global__ __launch_bounds__(H) void colsum1_kernel(const float *m, int rows, float *part)
{
    const int j = threadIdx.x, chunk = blockIdx.x;
    const int r0 = chunk * 256, r1 = min(rows, r0 + 256);
    float s = 0.f;
    for (int r = r0; r < r1; ++r) s += m[(int64_t)r * H + j];
    part[(int64_t)chunk * H + j] = s;
}

__global__ __launch_bounds__(H) void colsum2_kernel(const float *part, int chunks, float *out)
{
    const int j = threadIdx.x;
    float s = 0.f;
    for (int q = 0; q < chunks; ++q) s += part[(int64_t)q * H + j];
    out[j] += s;
}

__global__ void fill_kernel(float *p, int64_t count, float v)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < count) p[t] = v;
}

// ---------------------------------------------------------------------------
// Head.  One thread per (v, b); a block holds 256 restarts of one variable.
// ---------------------------------------------------------------------------
struct HeadArgs {
    const float *P;           // [n][H]  hv Wh + bh
    const float *wx, *wo, *bo;
    const float *x0;          // [n][B]
    float *xhat;              // [n][B] (forward)
    const uint8_t *target;    // [n] (backward)
    float *dP;                // [n][H] (backward)
    float *part;              // [blocks][2H + 2]: dwx, dwo, dbo, loss (backward)
    int n, B, chunks;         // chunks = ceil(B / 256)
    float inv_count;
};

__device__ __forceinline__ float softplus(float t) { return t > 0.f ? t + log1pf(expf(-t)) : log1pf(expf(t)); }
__device__ __forceinline__ float sigmoid(float t) { return 1.0f / (1.0f + expf(-t)); }

__global__ __launch_bounds__(kBlock) void head_fwd_kernel(HeadArgs A)
{
    const int v = blockIdx.x / A.chunks;
    const int b = (blockIdx.x % A.chunks) * kBlock + threadIdx.x;
    if (b >= A.B) return;
    const float x = A.x0[(int64_t)v * A.B + b];
    float z = A.bo[0];
    for (int j = 0; j < H; ++j) {
        const float u = fmaxf(fmaf(x, A.wx[j], A.P[(int64_t)v * H + j]), 0.f);
        z = fmaf(u, A.wo[j], z);
    }
    A.xhat[(int64_t)v * A.B + b] = tanhf(z);
}

// block reduction of one value over 256 threads into lane 0 of wave 0 (fixed order)
__device__ __forceinline__ float block_sum(float s, float *red)
{
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    float t = 0.f;
    if (threadIdx.x == 0)
        for (int w = 0; w < kBlock / 64; ++w) t += red[w];
    return t;
}

__global__ __launch_bounds__(kBlock) void head_bwd_kernel(HeadArgs A)
{
    __shared__ float red[kBlock / 64];
    const int v = blockIdx.x / A.chunks;
    const int b = (blockIdx.x % A.chunks) * kBlock + threadIdx.x;
    const bool valid = b < A.B;
    const float x = valid ? A.x0[(int64_t)v * A.B + b] : 0.f;
    float z = A.bo[0];
    for (int j = 0; j < H; ++j) {
        const float u = fmaxf(fmaf(x, A.wx[j], A.P[(int64_t)v * H + j]), 0.f);
        z = fmaf(u, A.wo[j], z);
    }
    const float y = A.target[v] ? 1.0f : 0.0f;
    const float loss = valid ? (y * softplus(2.0f * z) + (1.0f - y) * softplus(-2.0f * z)) * A.inv_count : 0.f;
    const float dz = valid ? 2.0f * (sigmoid(2.0f * z) - 1.0f + y) * A.inv_count : 0.f;
    float *part = A.part + (int64_t)blockIdx.x * (2 * H + 2);
    for (int j = 0; j < H; ++j) {
        const float pre = fmaf(x, A.wx[j], A.P[(int64_t)v * H + j]);
        const float u = fmaxf(pre, 0.f);
        const float du = pre > 0.f ? dz * A.wo[j] : 0.f;
        const float s_dp = block_sum(du, red);
        const float s_dwx = block_sum(du * x, red);
        const float s_dwo = block_sum(dz * u, red);
        if (threadIdx.x == 0) {
            part[j] = s_dwx;
            part[H + j] = s_dwo;
            // dP partial of restart chunk q of v at [q][v][j]; chunks are summed in order later
            A.dP[((int64_t)(blockIdx.x % A.chunks) * A.n + v) * H + j] = s_dp;
        }
    }
    const float s_dbo = block_sum(dz, red);
    const float s_loss = block_sum(loss, red);
    if (threadIdx.x == 0) {
        part[2 * H] = s_dbo;
        part[2 * H + 1] = s_loss;
    }
}

// Adam on the flat parameter array (bias-corrected moments; t >= 1).
__global__ __launch_bounds__(kBlock) void adam_kernel(float *p, const float *g, float *m, float *v, int64_t count,
                                                      float lr, float b1, float b2, float eps, float c1, float c2)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= count) return;
    const float gt = g[t];
    const float mt = b1 * m[t] + (1.0f - b1) * gt;
    const float vt = b2 * v[t] + (1.0f - b2) * gt * gt;
    m[t] = mt;
    v[t] = vt;
    p[t] -= lr * (mt / c1) / (sqrtf(vt / c2) + eps);
}

}  // namespace gnn
}  // namespace afs

using namespace afs::gnn;

// ---------------------------------------------------------------------------
// Parameters: one flat FP32 array (and gradients, Adam moments of the same layout).
// ---------------------------------------------------------------------------
struct ParamLayout {
    int R = 3;
    int64_t Wv0, bv0, Wc0, bc0, U, bu, V, bv, Wh, bh, wx, wo, bo, total;
    explicit ParamLayout(int rounds) : R(rounds)
    {
        int64_t o = 0;
        Wv0 = o; o += F * H; bv0 = o; o += H;
        Wc0 = o; o += F * H; bc0 = o; o += H;
        U = o; o += (int64_t)R * 2 * H * H; bu = o; o += (int64_t)R * H;
        V = o; o += (int64_t)R * 2 * H * H; bv = o; o += (int64_t)R * H;
        Wh = o; o += H * H; bh = o; o += H;
        wx = o; o += H; wo = o; o += H; bo = o; o += 1;
        total = o;
    }
};

struct afs_gnn {
    int device = -1;
    ParamLayout L{3};
    float *p = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;
};

namespace {

thread_local std::string g_gnn_err;

afs_status gfail(afs_status s, const std::string &msg)
{
    g_gnn_err = msg;
    return s;
}

class Dev {
public:
    explicit Dev(int d)
    {
        if (hipGetDevice(&prev_) != hipSuccess) { err_ = hipErrorNoDevice; return; }
        if (prev_ != d) err_ = hipSetDevice(d);
        d_ = d;
    }
    ~Dev() { if (err_ == hipSuccess && prev_ >= 0 && prev_ != d_) (void)hipSetDevice(prev_); }
    hipError_t err() const { return err_; }
private:
    int prev_ = -1, d_ = -1;
    hipError_t err_ = hipSuccess;
};

uint64_t splitmix(uint64_t &s)
{
    uint64_t z = (s += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

double normal01(uint64_t &s)
{
    const double u1 = ((splitmix(s) >> 11) + 1.0) / 9007199254740993.0;
    const double u2 = (splitmix(s) >> 11) / 9007199254740992.0;
    return std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586 * u2);
}

// Host features (16 per row):
//   constraint: one-hot type (8), log2(k+1)/10, parameter (K/(k+1) for the counted
//               types, parity for XOR), weight, 1
//   variable  : log2(1+deg)/10, (pos - neg)/deg, 1
void host_features(const afs::HostInstance &Hh, std::vector<float> &fc, std::vector<float> &fv,
                   std::vector<int32_t> &var_off, std::vector<int32_t> &var_con, std::vector<float> &var_sgn,
                   std::vector<float> &inv_k, std::vector<float> &inv_deg)
{
    const int32_t n = Hh.n, C = Hh.C;
    fc.assign((size_t)C * F, 0.f);
    fv.assign((size_t)n * F, 0.f);
    inv_k.assign(C, 0.f);
    std::vector<int32_t> pos(n, 0), neg(n, 0);
    for (int32_t c = 0; c < C; ++c) {
        const int k = (int)(Hh.con_off[c + 1] - Hh.con_off[c]);
        const int t = Hh.types[c];
        float *f = &fc[(size_t)c * F];
        f[t] = 1.f;
        f[8] = (float)(std::log2((double)k + 1.0) / 10.0);
        if (t == 3 || t == 4 || t == 7) f[9] = (float)Hh.params[c] / (float)(k + 1);
        else if (t == 1) f[9] = (float)(Hh.params[c] & 1);
        f[10] = Hh.weights[c];
        f[11] = 1.f;
        inv_k[c] = 1.0f / (float)k;
        for (int64_t e = Hh.con_off[c]; e < Hh.con_off[c + 1]; ++e) {
            const int32_t l = Hh.lits[e];
            if (l > 0) ++pos[l - 1]; else ++neg[-l - 1];
        }
    }
    var_off.assign(n + 1, 0);
    inv_deg.assign(n, 0.f);
    for (int32_t v = 0; v < n; ++v) {
        const int d = pos[v] + neg[v];
        var_off[v + 1] = var_off[v] + d;
        float *f = &fv[(size_t)v * F];
        f[0] = (float)(std::log2(1.0 + d) / 10.0);
        f[1] = d ? (float)(pos[v] - neg[v]) / (float)d : 0.f;
        f[2] = 1.f;
        inv_deg[v] = 1.0f / (float)std::max(d, 1);
    }
    var_con.assign(var_off[n], 0);
    var_sgn.assign(var_off[n], 0.f);
    std::vector<int32_t> fill(var_off.begin(), var_off.end() - 1);
    for (int32_t c = 0; c < C; ++c)
        for (int64_t e = Hh.con_off[c]; e < Hh.con_off[c + 1]; ++e) {
            const int32_t l = Hh.lits[e];
            const int v = (l > 0 ? l : -l) - 1;
            var_con[fill[v]] = c;
            var_sgn[fill[v]] = l > 0 ? 1.f : -1.f;
            ++fill[v];
        }
}

template <class T>
hipError_t upload_vec(afs_instance *I, const std::vector<T> &v, const T **out)
{
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, std::max<size_t>(v.size() * sizeof(T), 16));
    if (e != hipSuccess) return e;
    I->allocs.push_back(p);
    if (!v.empty()) e = hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice);
    *out = static_cast<const T *>(p);
    return e;
}

afs_status ensure_graph(afs_instance *I)
{
    if (I->gnn.built) return AFS_OK;
    std::vector<float> fc, fv, sg, ik, id;
    std::vector<int32_t> vo, vc;
    host_features(I->H, fc, fv, vo, vc, sg, ik, id);
    hipError_t e = hipSuccess;
    GnnGraph &G = I->gnn;
    if (e == hipSuccess) e = upload_vec(I, fc, &G.fcon);
    if (e == hipSuccess) e = upload_vec(I, fv, &G.fvar);
    if (e == hipSuccess) e = upload_vec(I, vo, &G.var_off);
    if (e == hipSuccess) e = upload_vec(I, vc, &G.var_con);
    if (e == hipSuccess) e = upload_vec(I, sg, &G.var_sgn);
    if (e == hipSuccess) e = upload_vec(I, ik, &G.inv_k);
    if (e == hipSuccess) e = upload_vec(I, id, &G.inv_deg);
    if (e != hipSuccess) return gfail(AFS_EDEVICE, std::string("graph upload: ") + hipGetErrorString(e));
    G.built = true;
    return AFS_OK;
}

// Workspace layout (floats).
struct GnnWs {
    int64_t Xv, Xc, Hv, Hc, P, dXv, dXc, dHv, dHc, dP, dpre, part, wpart, hpart, total;
    int R, n, C, B, chunks, cmax, rows_max, wsplits;
};

constexpr int kWChunk = 2048;   // rows per split of a weight-gradient GEMM (multiple of 16)

GnnWs ws_layout(int R, int n, int C, int B)
{
    GnnWs w{};
    w.R = R; w.n = n; w.C = C; w.B = B;
    w.chunks = (B + kBlock - 1) / kBlock;
    w.rows_max = std::max(n, C);
    w.wsplits = (w.rows_max + kWChunk - 1) / kWChunk;
    int64_t o = 0;
    auto take = [&](int64_t count) { int64_t at = o; o += (count + 63) / 64 * 64; return at; };
    w.Xv = take((int64_t)R * n * 2 * H);
    w.Xc = take((int64_t)R * C * 2 * H);
    w.Hv = take((int64_t)n * H);
    w.Hc = take((int64_t)C * H);
    w.P = take((int64_t)n * H);
    w.dXv = take((int64_t)R * n * 2 * H);
    w.dXc = take((int64_t)R * C * 2 * H);
    w.dHv = take((int64_t)n * H);
    w.dHc = take((int64_t)C * H);
    w.dP = take((int64_t)n * w.chunks * H);
    w.dpre = take((int64_t)w.rows_max * H);
    w.part = take((int64_t)((w.rows_max + 255) / 256) * H);
    w.wpart = take((int64_t)w.wsplits * 2 * H * H);
    w.hpart = take((int64_t)n * w.chunks * (2 * H + 2));
    w.total = o;
    return w;
}

inline unsigned nblocks(int64_t threads) { return (unsigned)((threads + kBlock - 1) / kBlock); }

hipError_t gemm(const float *a1, const float *a2, int ksplit, int64_t sam, int64_t sak, const float *b, int64_t sbk,
                int64_t sbn, float *c, int64_t ldc, const float *bias, bool relu, bool acc, int M, int N, int K,
                hipStream_t s)
{
    if (M == 0 || N == 0) return hipSuccess;
    GemmArgs g{};
    g.a1 = a1; g.a2 = a2 ? a2 : a1; g.ksplit = a2 ? ksplit : K; g.sam = sam; g.sak = sak;
    g.b = b; g.sbk = sbk; g.sbn = sbn; g.c = c; g.ldc = ldc; g.split_stride = 0;
    g.bias = bias; g.relu = relu; g.accumulate = acc; g.M = M; g.N = N; g.K = K;
    g.kchunk = (K + 15) / 16 * 16;
    // the layer shapes: 64 output columns, K a multiple of 16 up to 128, A rows
    // contiguous in k, the two A halves split on a 16 boundary
    if (N == H && K > 0 && K % 16 == 0 && K <= 128 && sak == 1 && g.ksplit % 16 == 0) {
        // a few row tiles per wave on large inputs (B staged once per more rows,
        // loads overlapped), one on small ones (enough waves to fill the device)
        const int64_t row_tiles = (M + 15) / 16;
        g.rtw = (int)std::min<int64_t>(kMaxRowTiles, std::max<int64_t>(1, row_tiles / (4 * 2048)));
        const int64_t per_block = (int64_t)(kBlock / 64) * g.rtw;
        const unsigned blocks = (unsigned)((row_tiles + per_block - 1) / per_block);
        switch (K / 16) {
        case 1: hipLaunchKernelGGL(gemm_rows64_kernel<1>, dim3(blocks), dim3(kBlock), 0, s, g); break;
        case 2: hipLaunchKernelGGL(gemm_rows64_kernel<2>, dim3(blocks), dim3(kBlock), 0, s, g); break;
        case 3: hipLaunchKernelGGL(gemm_rows64_kernel<3>, dim3(blocks), dim3(kBlock), 0, s, g); break;
        case 4: hipLaunchKernelGGL(gemm_rows64_kernel<4>, dim3(blocks), dim3(kBlock), 0, s, g); break;
        case 5: hipLaunchKernelGGL(gemm_rows64_kernel<5>, dim3(blocks), dim3(kBlock), 0, s, g); break;
        case 6: hipLaunchKernelGGL(gemm_rows64_kernel<6>, dim3(blocks), dim3(kBlock), 0, s, g); break;
        case 7: hipLaunchKernelGGL(gemm_rows64_kernel<7>, dim3(blocks), dim3(kBlock), 0, s, g); break;
        default: hipLaunchKernelGGL(gemm_rows64_kernel<8>, dim3(blocks), dim3(kBlock), 0, s, g); break;
        }
        return hipGetLastError();
    }
    const int64_t tiles = (int64_t)((M + 15) / 16) * ((N + 15) / 16);
    hipLaunchKernelGGL(gemm_bf16_kernel, dim3((unsigned)((tiles + 3) / 4), 1), dim3(kBlock), 0, s, g);
    return hipGetLastError();
}

// dW[Kdim][N] += X^T dY : X rows x Kdim (two halves of H columns each when x2 given), dY rows x N
hipError_t wgrad(const float *x1, const float *x2, int64_t ldx, int Kdim, const float *dy, int rows, float *dW,
                 float *wpart, hipStream_t s)
{
    if (rows == 0) return hipSuccess;
    const int splits = (rows + kWChunk - 1) / kWChunk;
    // A(m, k) = X[k][m]  (m < Kdim, k < rows), B(k, n) = dY[k][n]; the two column
    // halves of X (when x2 is given) are two launches writing rows [0, H) and [H, 2H) of dW
    const int halves = x2 ? 2 : 1;
    const int mh = x2 ? Kdim / 2 : Kdim;
    for (int h = 0; h < halves; ++h) {
        GemmArgs q{};
        q.a1 = h == 0 ? x1 : x2; q.a2 = q.a1; q.ksplit = rows; q.sam = 1; q.sak = ldx;
        q.b = dy; q.sbk = H; q.sbn = 1;
        q.c = wpart; q.ldc = H; q.split_stride = (int64_t)mh * H;
        q.bias = nullptr; q.relu = 0; q.accumulate = 0;
        q.M = mh; q.N = H; q.K = rows; q.kchunk = kWChunk;
        const int64_t tiles = (int64_t)((mh + 15) / 16) * ((H + 15) / 16);
        hipLaunchKernelGGL(gemm_bf16_kernel, dim3((unsigned)((tiles + 3) / 4), splits), dim3(kBlock), 0, s, q);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(sum_splits_kernel, dim3(nblocks((int64_t)mh * H)), dim3(kBlock), 0, s, wpart, splits,
                           (int64_t)mh * H, mh, H, dW + (int64_t)h * mh * H, (int64_t)H, 1);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t colsum(const float *m, int rows, float *part, float *out, hipStream_t s)
{
    if (rows == 0) return hipSuccess;
    const int chunks = (rows + 255) / 256;
    hipLaunchKernelGGL(colsum1_kernel, dim3(chunks), dim3(H), 0, s, m, rows, part);
    hipLaunchKernelGGL(colsum2_kernel, dim3(1), dim3(H), 0, s, part, chunks, out);
    return hipGetLastError();
}

hipError_t fill(float *p, int64_t count, float v, hipStream_t s)
{
    if (count == 0) return hipSuccess;
    hipLaunchKernelGGL(fill_kernel, dim3(nblocks(count)), dim3(kBlock), 0, s, p, count, v);
    return hipGetLastError();
}

struct Ctx {
    afs_gnn *G;
    afs_instance *I;
    GnnWs w;
    float *ws;
    hipStream_t s;
    float *at(int64_t off) { return ws + off; }
    float *Xv(int r) { return ws + w.Xv + (int64_t)(r - 1) * w.n * 2 * H; }   // r = 1..R
    float *Xc(int r) { return ws + w.Xc + (int64_t)(r - 1) * w.C * 2 * H; }
    float *dXv(int r) { return ws + w.dXv + (int64_t)(r - 1) * w.n * 2 * H; }
    float *dXc(int r) { return ws + w.dXc + (int64_t)(r - 1) * w.C * 2 * H; }
};

#define GNN_TRY(x) do { hipError_t e_ = (x); if (e_ != hipSuccess) return e_; } while (0)

// Forward through the graph rounds and the head's restart-independent part P.
hipError_t forward_graph(Ctx &X)
{
    const ParamLayout &L = X.G->L;
    const float *p = X.G->p;
    const GnnGraph &gg = X.I->gnn;
    const afs::DevInstance &D = X.I->D;
    const int n = X.w.n, C = X.w.C, R = X.w.R;
    // input layers into the first halves of round 1's inputs
    GNN_TRY(gemm(gg.fvar, nullptr, F, F, 1, p + L.Wv0, H, 1, X.Xv(1), 2 * H, p + L.bv0, true, false, n, H, F, X.s));
    GNN_TRY(gemm(gg.fcon, nullptr, F, F, 1, p + L.Wc0, H, 1, X.Xc(1), 2 * H, p + L.bc0, true, false, C, H, F, X.s));
    for (int r = 1; r <= R; ++r) {
        float *xv = X.Xv(r), *xc = X.Xc(r);
        // ac = agg_c(hv)  (second half of xc)
        hipLaunchKernelGGL(agg_c_kernel, dim3((C + 3) / 4), dim3(kBlock), 0, X.s, D.con_off, D.lits, gg.inv_k,
                           gg.inv_deg, 1, xv, (int64_t)2 * H, xc + H, (int64_t)2 * H, C, 0);
        GNN_TRY(hipGetLastError());
        float *hc_out = r < R ? X.Xc(r + 1) : X.at(X.w.Hc);
        const int64_t ldhc = r < R ? 2 * H : H;
        GNN_TRY(gemm(xc, nullptr, 2 * H, 2 * H, 1, p + L.U + (int64_t)(r - 1) * 2 * H * H, H, 1, hc_out, ldhc,
                     p + L.bu + (int64_t)(r - 1) * H, true, false, C, H, 2 * H, X.s));
        // av = agg_v(hc)
        hipLaunchKernelGGL(agg_v_kernel, dim3((n + 3) / 4), dim3(kBlock), 0, X.s, gg.var_off, gg.var_con,
                           gg.var_sgn, gg.inv_k, gg.inv_deg, 1, hc_out, ldhc, xv + H, (int64_t)2 * H, n, 0);
        GNN_TRY(hipGetLastError());
        float *hv_out = r < R ? X.Xv(r + 1) : X.at(X.w.Hv);
        const int64_t ldhv = r < R ? 2 * H : H;
        GNN_TRY(gemm(xv, nullptr, 2 * H, 2 * H, 1, p + L.V + (int64_t)(r - 1) * 2 * H * H, H, 1, hv_out, ldhv,
                     p + L.bv + (int64_t)(r - 1) * H, true, false, n, H, 2 * H, X.s));
    }
    // P = hv Wh + bh (no activation)
    GNN_TRY(gemm(X.at(X.w.Hv), nullptr, H, H, 1, p + L.Wh, H, 1, X.at(X.w.P), H, p + L.bh, false, false, n, H, H,
                 X.s));
    return hipSuccess;
}

HeadArgs head_args(Ctx &X, const float *x0)
{
    const ParamLayout &L = X.G->L;
    HeadArgs a{};
    a.P = X.at(X.w.P);
    a.wx = X.G->p + L.wx; a.wo = X.G->p + L.wo; a.bo = X.G->p + L.bo;
    a.x0 = x0; a.n = X.w.n; a.B = X.w.B; a.chunks = X.w.chunks;
    a.inv_count = 1.0f / ((float)X.w.n * (float)X.w.B);
    return a;
}

// Backward of everything below the head, from dP (in X.at(w.dP), chunked) into the gradients.
hipError_t backward_graph(Ctx &X)
{
    const ParamLayout &L = X.G->L;
    const float *p = X.G->p;
    float *gp = X.G->g;
    const GnnGraph &gg = X.I->gnn;
    const afs::DevInstance &D = X.I->D;
    const int n = X.w.n, C = X.w.C, R = X.w.R;
    float *dpre = X.at(X.w.dpre), *part = X.at(X.w.part), *wpart = X.at(X.w.wpart);
    // dP (chunks summed in order) -> dWh, dbh, dHv
    float *dP = X.at(X.w.dpre);   // reuse: n x H
    hipLaunchKernelGGL(sum_splits_kernel, dim3(nblocks((int64_t)n * H)), dim3(kBlock), 0, X.s, X.at(X.w.dP), X.w.chunks,
                       (int64_t)n * H, n, H, dP, (int64_t)H, 0);
    GNN_TRY(hipGetLastError());
    GNN_TRY(wgrad(X.at(X.w.Hv), nullptr, H, H, dP, n, gp + L.Wh, wpart, X.s));
    GNN_TRY(colsum(dP, n, part, gp + L.bh, X.s));
    GNN_TRY(fill(X.at(X.w.dXv), (int64_t)R * n * 2 * H, 0.f, X.s));
    GNN_TRY(fill(X.at(X.w.dXc), (int64_t)R * C * 2 * H, 0.f, X.s));
    GNN_TRY(fill(X.at(X.w.dHc), (int64_t)C * H, 0.f, X.s));
    // dHv = dP Wh^T
    GNN_TRY(gemm(dP, nullptr, H, H, 1, p + L.Wh, 1, H, X.at(X.w.dHv), H, nullptr, false, false, n, H, H, X.s));
    for (int r = R; r >= 1; --r) {
        float *xv = X.Xv(r), *xc = X.Xc(r), *dxv = X.dXv(r), *dxc = X.dXc(r);
        const float *hv_out = r < R ? X.Xv(r + 1) : X.at(X.w.Hv);
        const int64_t ldhv = r < R ? 2 * H : H;
        const float *dhv = r < R ? X.dXv(r + 1) : X.at(X.w.dHv);
        const float *hc_out = r < R ? X.Xc(r + 1) : X.at(X.w.Hc);
        const int64_t ldhc = r < R ? 2 * H : H;
        float *dhc = r < R ? X.dXc(r + 1) : X.at(X.w.dHc);
        // variable layer of round r
        hipLaunchKernelGGL(relu_grad_kernel, dim3(nblocks((int64_t)n * H)), dim3(kBlock), 0, X.s, dhv, ldhv, hv_out,
                           ldhv, dpre, n);
        GNN_TRY(hipGetLastError());
        GNN_TRY(wgrad(xv, xv + H, 2 * H, 2 * H, dpre, n, gp + L.V + (int64_t)(r - 1) * 2 * H * H, wpart, X.s));
        GNN_TRY(colsum(dpre, n, part, gp + L.bv + (int64_t)(r - 1) * H, X.s));
        // d[hv_prev, av] = dpre V^T   (V is [2H][H]: B(k, n') = V[n'][k])
        GNN_TRY(gemm(dpre, nullptr, H, H, 1, p + L.V + (int64_t)(r - 1) * 2 * H * H, 1, H, dxv, 2 * H, nullptr, false,
                     true, n, 2 * H, H, X.s));
        // dhc += agg_v^T(dav): per constraint, sum over its literals of s_e dav_v / deg_v
        hipLaunchKernelGGL(agg_c_kernel, dim3((C + 3) / 4), dim3(kBlock), 0, X.s, D.con_off, D.lits, gg.inv_k,
                           gg.inv_deg, 0, dxv + H, (int64_t)2 * H, dhc, r < R ? (int64_t)2 * H : (int64_t)H, C, 1);
        GNN_TRY(hipGetLastError());
        // constraint layer of round r
        hipLaunchKernelGGL(relu_grad_kernel, dim3(nblocks((int64_t)C * H)), dim3(kBlock), 0, X.s, dhc, ldhc, hc_out,
                           ldhc, dpre, C);
        GNN_TRY(hipGetLastError());
        GNN_TRY(wgrad(xc, xc + H, 2 * H, 2 * H, dpre, C, gp + L.U + (int64_t)(r - 1) * 2 * H * H, wpart, X.s));
        GNN_TRY(colsum(dpre, C, part, gp + L.bu + (int64_t)(r - 1) * H, X.s));
        GNN_TRY(gemm(dpre, nullptr, H, H, 1, p + L.U + (int64_t)(r - 1) * 2 * H * H, 1, H, dxc, 2 * H, nullptr, false,
                     true, C, 2 * H, H, X.s));
        // dhv_prev += agg_c^T(dac): per variable, sum over occurrences of s_e dac_c / k_c
        hipLaunchKernelGGL(agg_v_kernel, dim3((n + 3) / 4), dim3(kBlock), 0, X.s, gg.var_off, gg.var_con, gg.var_sgn,
                           gg.inv_k, gg.inv_deg, 0, dxc + H, (int64_t)2 * H, dxv, (int64_t)2 * H, n, 1);
        GNN_TRY(hipGetLastError());
    }
    // input layers: dhv0 = first half of dXv(1), dhc0 = first half of dXc(1)
    hipLaunchKernelGGL(relu_grad_kernel, dim3(nblocks((int64_t)n * H)), dim3(kBlock), 0, X.s, X.dXv(1), (int64_t)2 * H,
                       X.Xv(1), (int64_t)2 * H, dpre, n);
    GNN_TRY(hipGetLastError());
    GNN_TRY(wgrad(gg.fvar, nullptr, F, F, dpre, n, gp + L.Wv0, wpart, X.s));
    GNN_TRY(colsum(dpre, n, part, gp + L.bv0, X.s));
    hipLaunchKernelGGL(relu_grad_kernel, dim3(nblocks((int64_t)C * H)), dim3(kBlock), 0, X.s, X.dXc(1), (int64_t)2 * H,
                       X.Xc(1), (int64_t)2 * H, dpre, C);
    GNN_TRY(hipGetLastError());
    GNN_TRY(wgrad(gg.fcon, nullptr, F, F, dpre, C, gp + L.Wc0, wpart, X.s));
    GNN_TRY(colsum(dpre, C, part, gp + L.bc0, X.s));
    return hipSuccess;
}

// Starting points from the network's output xhat = tanh(z) and the noise x0 it
// was given (one thread per (v, b)).  The output is softened to tanh(z / T);
// with `sample` each point takes magnitude |x0| and the sign of a draw from the
// softened marginal P(True) = (1 - tanh(z / T)) / 2 (True -> negative), the draw
// u uniform on [0, 1) from Philox4x32-10 with counter (b, v, 1, 0); otherwise
// the point is (1 - mix) tanh(z / T) + mix x0.  A non-finite network output
// falls back to the uniform point x0.  Result clamped to [-1, 1].
__global__ __launch_bounds__(kBlock) void starts_kernel(int64_t count, int B, const float *xhat, const float *x0,
                                                        uint32_t k0, uint32_t k1, float inv_t, float mix,
                                                        int sample, float *out)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= count) return;
    const float xh = xhat[i], x = x0[i];
    float r;
    if (!isfinite(xh)) {
        r = x;
    } else {
        float soft = xh;
        if (inv_t != 1.0f) {
            const float c = fminf(fmaxf(xh, -0.999999f), 0.999999f);
            soft = tanhf(atanhf(c) * inv_t);
        }
        if (sample) {
            const int v = (int)(i / B), b = (int)(i - (int64_t)v * B);
            const afs::dev::U4 w = afs::dev::philox4x32_10(afs::dev::U4{(uint32_t)b, (uint32_t)v, 1u, 0u}, k0, k1);
            const float u = (float)(w.x >> 8) * 0x1p-24f;          // [0, 1)
            r = u < 0.5f * (1.0f - soft) ? -fabsf(x) : fabsf(x);
        } else {
            r = (1.0f - mix) * soft + mix * x;
        }
    }
    out[i] = fminf(1.0f, fmaxf(-1.0f, r));
}

afs_status check(afs_gnn *G, afs_instance *I, int32_t B, void *ws, size_t ws_bytes, GnnWs &w)
{
    if (!G || !I) return gfail(AFS_EINVAL, "NULL network or instance");
    if (I->device != G->device) return gfail(AFS_EINVAL, "network and instance are on different devices");
    if (B < 1) return gfail(AFS_EINVAL, "B must be >= 1");
    w = ws_layout(G->L.R, I->H.n, I->H.C, B);
    if (!ws || ws_bytes < (size_t)w.total * sizeof(float)) return gfail(AFS_EINVAL, "GNN workspace too small");
    if (reinterpret_cast<uintptr_t>(ws) % 256) return gfail(AFS_EINVAL, "workspace is not 256-byte aligned");
    return AFS_OK;
}

}  // namespace

extern "C" {

const char *afs_gnn_last_error(void) { return g_gnn_err.c_str(); }

afs_status afs_gnn_create(int32_t rounds, uint64_t seed, int32_t device, afs_gnn **out)
{
    if (!out) return gfail(AFS_EINVAL, "out is NULL");
    *out = nullptr;
    if (rounds < 1 || rounds > 8) return gfail(AFS_EINVAL, "rounds must be 1..8");
    Dev dg(device);
    if (dg.err() != hipSuccess) return gfail(AFS_EDEVICE, "hipSetDevice failed");
    afs_gnn *G = new (std::nothrow) afs_gnn();
    if (!G) return gfail(AFS_ENOMEM, "host allocation failed");
    G->device = device;
    G->L = ParamLayout(rounds);
    const int64_t P = G->L.total;
    // He-normal weights (fan-in), zero biases; the output layer starts small.
    std::vector<float> init(P, 0.f);
    uint64_t s = seed;
    auto fill_w = [&](int64_t off, int64_t count, int fan_in, double gain) {
        const double sd = gain * std::sqrt(2.0 / fan_in);
        for (int64_t i = 0; i < count; ++i) init[off + i] = (float)(sd * normal01(s));
    };
    const ParamLayout &L = G->L;
    fill_w(L.Wv0, F * H, 3, 1.0);
    fill_w(L.Wc0, F * H, 4, 1.0);
    fill_w(L.U, (int64_t)rounds * 2 * H * H, 2 * H, 1.0);
    fill_w(L.V, (int64_t)rounds * 2 * H * H, 2 * H, 1.0);
    fill_w(L.Wh, H * H, H, 1.0);
    fill_w(L.wx, H, 1, 1.0);
    fill_w(L.wo, H, H, 0.1);
    hipError_t e = hipSuccess;
    float **bufs[4] = {&G->p, &G->g, &G->m, &G->v};
    for (float **b : bufs) {
        if (e == hipSuccess) e = hipMalloc((void **)b, (size_t)P * sizeof(float));
        if (e == hipSuccess) e = hipMemset(*b, 0, (size_t)P * sizeof(float));
    }
    if (e == hipSuccess) e = hipMemcpy(G->p, init.data(), (size_t)P * sizeof(float), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        for (float **b : bufs) if (*b) (void)hipFree(*b);
        delete G;
        return gfail(AFS_EDEVICE, std::string("GNN allocation: ") + hipGetErrorString(e));
    }
    *out = G;
    return AFS_OK;
}

void afs_gnn_destroy(afs_gnn *G)
{
    if (!G) return;
    Dev dg(G->device);
    (void)hipDeviceSynchronize();   // queued work may still read the parameters
    for (float *b : {G->p, G->g, G->m, G->v}) if (b) (void)hipFree(b);
    delete G;
}

afs_status afs_gnn_num_params(const afs_gnn *G, int64_t *count)
{
    if (!G || !count) return gfail(AFS_EINVAL, "NULL argument");
    *count = G->L.total;
    return AFS_OK;
}

afs_status afs_gnn_get(const afs_gnn *G, int32_t which, float *host)
{
    if (!G || !host || which < 0 || which > 3) return gfail(AFS_EINVAL, "invalid argument");
    Dev dg(G->device);
    const float *src[4] = {G->p, G->g, G->m, G->v};
    hipError_t e = hipMemcpy(host, src[which], (size_t)G->L.total * sizeof(float), hipMemcpyDeviceToHost);
    return e == hipSuccess ? AFS_OK : gfail(AFS_EDEVICE, hipGetErrorString(e));
}

afs_status afs_gnn_set(afs_gnn *G, int32_t which, const float *host)
{
    if (!G || !host || which < 0 || which > 3) return gfail(AFS_EINVAL, "invalid argument");
    Dev dg(G->device);
    float *dst[4] = {G->p, G->g, G->m, G->v};
    hipError_t e = hipMemcpy(dst[which], host, (size_t)G->L.total * sizeof(float), hipMemcpyHostToDevice);
    return e == hipSuccess ? AFS_OK : gfail(AFS_EDEVICE, hipGetErrorString(e));
}

afs_status afs_gnn_features(afs_instance *I, float *fcon, float *fvar, int32_t *var_off, int32_t *var_con,
                            float *var_sgn)
{
    if (!I || !fcon || !fvar) return gfail(AFS_EINVAL, "NULL argument");
    std::vector<float> fc, fv, sg, ik, id;
    std::vector<int32_t> vo, vc;
    host_features(I->H, fc, fv, vo, vc, sg, ik, id);
    std::memcpy(fcon, fc.data(), fc.size() * sizeof(float));
    std::memcpy(fvar, fv.data(), fv.size() * sizeof(float));
    if (var_off) std::memcpy(var_off, vo.data(), vo.size() * sizeof(int32_t));
    if (var_con) std::memcpy(var_con, vc.data(), vc.size() * sizeof(int32_t));
    if (var_sgn) std::memcpy(var_sgn, sg.data(), sg.size() * sizeof(float));
    return AFS_OK;
}

afs_status afs_gnn_workspace_bytes(const afs_gnn *G, const afs_instance *I, int32_t B, size_t *bytes)
{
    if (!G || !I || !bytes || B < 1) return gfail(AFS_EINVAL, "invalid argument");
    *bytes = (size_t)ws_layout(G->L.R, I->H.n, I->H.C, B).total * sizeof(float);
    return AFS_OK;
}

afs_status afs_gnn_forward(afs_gnn *G, afs_instance *I, int32_t B, const float *x0, void *ws, size_t ws_bytes,
                           float *xhat, void *stream)
{
    GnnWs w;
    afs_status st = check(G, I, B, ws, ws_bytes, w);
    if (st != AFS_OK) return st;
    if (!x0 || !xhat) return gfail(AFS_EINVAL, "x0 or xhat is NULL");
    Dev dg(G->device);
    if ((st = ensure_graph(I)) != AFS_OK) return st;
    Ctx X{G, I, w, static_cast<float *>(ws), (hipStream_t)stream};
    hipError_t e = forward_graph(X);
    if (e == hipSuccess) {
        HeadArgs a = head_args(X, x0);
        a.xhat = xhat;
        hipLaunchKernelGGL(head_fwd_kernel, dim3((unsigned)((int64_t)w.n * w.chunks)), dim3(kBlock), 0, X.s, a);
        e = hipGetLastError();
    }
    return e == hipSuccess ? AFS_OK : gfail(AFS_EDEVICE, std::string("GNN forward: ") + hipGetErrorString(e));
}

afs_status afs_gnn_backward(afs_gnn *G, afs_instance *I, int32_t B, const float *x0, const uint8_t *target,
                            void *ws, size_t ws_bytes, float *loss, void *stream)
{
    GnnWs w;
    afs_status st = check(G, I, B, ws, ws_bytes, w);
    if (st != AFS_OK) return st;
    if (!x0 || !target || !loss) return gfail(AFS_EINVAL, "x0, target or loss is NULL");
    Dev dg(G->device);
    if ((st = ensure_graph(I)) != AFS_OK) return st;
    Ctx X{G, I, w, static_cast<float *>(ws), (hipStream_t)stream};
    hipError_t e = forward_graph(X);
    const ParamLayout &L = G->L;
    const int blocks = w.n * w.chunks;
    if (e == hipSuccess) {
        HeadArgs a = head_args(X, x0);
        a.target = target;
        a.dP = X.at(w.dP);
        a.part = X.at(w.hpart);
        hipLaunchKernelGGL(head_bwd_kernel, dim3((unsigned)blocks), dim3(kBlock), 0, X.s, a);
        e = hipGetLastError();
    }
    // head parameter gradients and the loss: fixed-order sums of the block partials
    if (e == hipSuccess) {
        float *hp = X.at(w.hpart);
        const int stride = 2 * H + 2;
        // dwx (j), dwo (H + j), dbo (2H), loss (2H + 1): rows = blocks, column stride 1
        hipLaunchKernelGGL(sum_splits_kernel, dim3(nblocks(H)), dim3(kBlock), 0, X.s, hp, blocks, (int64_t)stride, 1,
                           H, G->g + L.wx, (int64_t)H, 1);
        hipLaunchKernelGGL(sum_splits_kernel, dim3(nblocks(H)), dim3(kBlock), 0, X.s, hp + H, blocks, (int64_t)stride, 1,
                           H, G->g + L.wo, (int64_t)H, 1);
        hipLaunchKernelGGL(sum_splits_kernel, dim3(1), dim3(kBlock), 0, X.s, hp + 2 * H, blocks, (int64_t)stride, 1, 1,
                           G->g + L.bo, (int64_t)1, 1);
        hipLaunchKernelGGL(sum_splits_kernel, dim3(1), dim3(kBlock), 0, X.s, hp + 2 * H + 1, blocks, (int64_t)stride, 1,
                           1, loss, (int64_t)1, 0);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = backward_graph(X);
    return e == hipSuccess ? AFS_OK : gfail(AFS_EDEVICE, std::string("GNN backward: ") + hipGetErrorString(e));
}

afs_status afs_gnn_zero_grad(afs_gnn *G, void *stream)
{
    if (!G) return gfail(AFS_EINVAL, "NULL network");
    Dev dg(G->device);
    hipError_t e = fill(G->g, G->L.total, 0.f, (hipStream_t)stream);
    return e == hipSuccess ? AFS_OK : gfail(AFS_EDEVICE, hipGetErrorString(e));
}

afs_status afs_gnn_adam(afs_gnn *G, float lr, float beta1, float beta2, float eps, int32_t t, void *stream)
{
    if (!G || t < 1) return gfail(AFS_EINVAL, "invalid argument");
    Dev dg(G->device);
    const float c1 = 1.0f - std::pow(beta1, (float)t), c2 = 1.0f - std::pow(beta2, (float)t);
    hipLaunchKernelGGL(adam_kernel, dim3(nblocks(G->L.total)), dim3(kBlock), 0, (hipStream_t)stream, G->p, G->g, G->m,
                       G->v, G->L.total, lr, beta1, beta2, eps, c1, c2);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? AFS_OK : gfail(AFS_EDEVICE, hipGetErrorString(e));
}

afs_status afs_gnn_starts(int32_t n, int32_t B, const float *xhat, const float *x0, uint64_t seed, float temperature,
                          float mix, int32_t sample, float *out, void *stream)
{
    if (n < 0 || B < 0 || !(temperature > 0.0f) || !(mix >= 0.0f && mix <= 1.0f))
        return gfail(AFS_EINVAL, "need n, B >= 0, temperature > 0, 0 <= mix <= 1");
    const int64_t count = (int64_t)n * B;
    if (count == 0) return AFS_OK;
    if (count >= ((int64_t)1 << 38)) return gfail(AFS_EINVAL, "n * B too large");
    if (!xhat || !x0 || !out) return gfail(AFS_EINVAL, "NULL array");
    hipLaunchKernelGGL(starts_kernel, dim3(nblocks(count)), dim3(kBlock), 0, (hipStream_t)stream, count, B, xhat, x0,
                       (uint32_t)seed, (uint32_t)(seed >> 32), 1.0f / temperature, mix, sample ? 1 : 0, out);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? AFS_OK : gfail(AFS_EDEVICE, hipGetErrorString(e));
}

afs_status afs_gnn_gemm_bf16(int32_t M, int32_t N, int32_t K, const float *A, int64_t sam, int64_t sak, const float *B,
                             int64_t sbk, int64_t sbn, float *C, int64_t ldc, void *stream)
{
    if (M < 0 || N < 0 || K < 0 || !A || !B || !C) return gfail(AFS_EINVAL, "invalid GEMM arguments");
    hipError_t e = gemm(A, nullptr, K, sam, sak, B, sbk, sbn, C, ldc, nullptr, false, false, M, N, K,
                        (hipStream_t)stream);
    return e == hipSuccess ? AFS_OK : gfail(AFS_EDEVICE, hipGetErrorString(e));
}

}  // extern "C"
