// kernels.hip -- HIP kernels for gfx950 (CDNA4, wave64).
//
// Evaluation of a symmetric constraint of length k at a real point (Sec. 2.1.2).
// With p_i = (1 - y_i)/2 the probability that literal i is true, the generating
// function of the number of true literals is prod_i ((1-p_i) + p_i z); its values
// at the N = k+1 roots of unity z = omega^m are G_m = prod_i a_{i,m}, and
// FE = sum_m d_m G_m with d = inverse DFT of the truth table.  Because d and G are
// conjugate symmetric and G_0 = 1,
//     FE = d_0 + 2 sum_{m=1..M} Re(d_m G_m) + [k odd] d_{N/2} prod_i y_i,  M = floor(k/2).
// The gradient is taken by prefix and suffix products (no division):
//     dFE/dy_i = 2 sum_m Re(d_m beta_m prod_{l != i} a_{l,m}) + [k odd] d_{N/2} prod_{l != i} y_l
// with beta_m = (1 - omega^m)/2 = da/dy.  Every true factor has |a| <= 1, so the
// true products cannot overflow at any length; the kernels carry them in the
// rotated form described above mul_unit.
//
// Layouts: x [n][B] f32 (restart contiguous); adj [L][Bp] f32 in slot order with
// Bp = B rounded up to 64; constraint and literal metadata are wave-uniform and
// are read through the scalar cache.

#include "kernels.hpp"

namespace afs {

namespace {

constexpr int kWave = 64;
constexpr int kBlock = 256;
constexpr int kWavesPerBlock = kBlock / kWave;
constexpr int kXcds = 8;

// Workgroups are handed to the 8 XCDs round-robin.  Renumber them so that each
// XCD receives one contiguous range of logical blocks (and with it a contiguous
// range of restart columns, whose x rows then stay in that XCD's L2).
__device__ __forceinline__ int64_t xcd_block()
{
    const int64_t nb = gridDim.x;
    const int64_t i = blockIdx.x;
    const int64_t xcd = i % kXcds, idx = i / kXcds;
    const int64_t base = nb / kXcds, extra = nb % kXcds;
    return xcd * base + (xcd < extra ? xcd : extra) + idx;
}

__device__ __forceinline__ int wave_id()
{
    return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
}

__device__ __forceinline__ void cmul(float &ar, float &ai, float br, float bi)
{
    const float r = ar * br - ai * bi;
    ai = ar * bi + ai * br;
    ar = r;
}

struct FeArgs {
    const float *x;
    float *adj, *part, *fe;
    const float *dobj;          // per-restart seed of the adjoint (NULL: 1)
    const int32_t *bc_slot0, *bc_k, *bc_tab, *bc_orig;
    const float *bc_w;
    const int32_t *slot_lit;
    const float4 *tab;
    int B, Bp;
    int32_t c0, nc, tile, ntiles, tile0;
    int64_t items;
};

// ---------------------------------------------------------------------------
// Factor form shared by the FE kernels.  With h = pi m / N, c = cos h and
// alpha = (1 + omega^m)/2 = c e^{i h}, the factor of a literal with value y is
//     a = (1-p) + p omega^m = alpha (1 + i z),   z = -tan(h) y,
// so one step of a product chain multiplies by (1 + i z): two FMAs.  Since
// |1 + i z| <= 1/c, the segment kernels multiply their running products by
// alpha^RP after every RP literals (RP = 16 for lengths <= 256, else 8), and the
// remaining constant alpha powers are folded into the table (host.cpp,
// append_root_rows).  Padding literals hold y = +1, whose factor
// alpha (1 - i tan h) is exactly 1.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void mul_unit(float &r, float &i, float z)
{
    const float nr = fmaf(-i, z, r);
    i = fmaf(r, z, i);
    r = nr;
}

// ---------------------------------------------------------------------------
// Short constraints (k <= 16): one lane per restart, k known at compile time, the
// whole constraint in registers.  A wave takes 64 restarts and a tile of
// constraints of the bucket.
// ---------------------------------------------------------------------------
template <int K, bool GRAD>
__global__ __launch_bounds__(kBlock) void fe_grad_short(FeArgs A)
{
    const int64_t item = xcd_block() * kWavesPerBlock + wave_id();
    if (item >= A.items) return;
    const int lane = threadIdx.x & 63;
    const int group = (int)(item / A.ntiles);
    const int tile = (int)(item % A.ntiles);
    const int b = group * kWave + lane;
    const bool valid = b < A.B;
    const int bl = valid ? b : A.B - 1;
    const int cbeg = A.c0 + tile * A.tile;
    const int cend = min(cbeg + A.tile, A.c0 + A.nc);
    const float seed = (GRAD && A.dobj) ? A.dobj[bl] : 1.0f;
    float objacc = 0.f;
    for (int c = cbeg; c < cend; ++c) {
        const int slot0 = A.bc_slot0[c];
        const int tab = A.bc_tab[c];
        const float w = A.bc_w[c];
        const float wg = w * seed;
        int lit[K];
        float y[K], adj[K];
#pragma unroll
        for (int i = 0; i < K; ++i) {
            lit[i] = A.slot_lit[slot0 + i];
            const int v = (lit[i] > 0 ? lit[i] : -lit[i]) - 1;
            const float xv = A.x[(int64_t)v * A.B + bl];
            y[i] = lit[i] > 0 ? xv : -xv;
            adj[i] = 0.f;
        }
        const float4 r0 = A.tab[tab];
        float fe = r0.x;
        // Roots one at a time (unrolling them multiplies register use by K/2).
#pragma unroll 1
        for (int m = 1; m <= K / 2; ++m) {
            const float4 ra = A.tab[tab + 2 * m - 1];   // {d alpha^K, Kc}
            const float4 rb = A.tab[tab + 2 * m];       // {-, -, -tan h, -}
            float z[K], pr[K], pi[K];
#pragma unroll
            for (int i = 0; i < K; ++i) z[i] = rb.z * y[i];
            float ur = 1.0f, ui = 0.0f;       // |1 + i z|^K stays far below 2^128 for K <= 16
#pragma unroll
            for (int i = 0; i < K; ++i) {
                pr[i] = ur;
                pi[i] = ui;
                mul_unit(ur, ui, z[i]);
            }
            fe = fmaf(2.0f, ra.x * ur - ra.y * ui, fe);
            if (GRAD) {
                float sr = wg * ra.z, si = wg * ra.w;
#pragma unroll
                for (int i = K - 1; i >= 0; --i) {
                    adj[i] = fmaf(pr[i], sr, adj[i]);
                    adj[i] = fmaf(-pi[i], si, adj[i]);
                    if (i > 0) mul_unit(sr, si, z[i]);
                }
            }
        }
        if (K & 1) {                       // real root omega^(N/2) = -1: factor y_i
            const float dh = r0.y;
            float hp[K], h = 1.0f;
#pragma unroll
            for (int i = 0; i < K; ++i) {
                hp[i] = h;
                h *= y[i];
            }
            fe = fmaf(dh, h, fe);
            if (GRAD) {
                float hs = wg * dh;
#pragma unroll
                for (int i = K - 1; i >= 0; --i) {
                    adj[i] = fmaf(hp[i], hs, adj[i]);
                    hs *= y[i];
                }
            }
        }
        if (valid) {
            if (GRAD) {
#pragma unroll
                for (int i = 0; i < K; ++i)
                    A.adj[(int64_t)(slot0 + i) * A.Bp + b] = lit[i] > 0 ? adj[i] : -adj[i];
            }
            if (A.fe) A.fe[(int64_t)A.bc_orig[c] * A.B + b] = fe;
        }
        objacc = fmaf(w, fe, objacc);
    }
    if (A.part) A.part[(int64_t)(A.tile0 + tile) * A.Bp + b] = objacc;
}

// ---------------------------------------------------------------------------
// Cross-lane products over the J lanes that share one restart.
// Inside a 16-lane row the shifts are DPP row shifts whose out-of-row lanes read
// the identity; groups of 32 or 64 lanes then take the neighbouring rows' totals.
// ---------------------------------------------------------------------------
template <int CTRL>
__device__ __forceinline__ float dpp_mov(float old, float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(old), __float_as_int(v), CTRL, 0xF, 0xF, false));
}

constexpr int kRowShr = 0x110;   // row_shr:n = 0x110 + n
constexpr int kRowShl = 0x100;   // row_shl:n = 0x100 + n

// value of lane j-D of the group (identity below j = D), complex or real
template <int J, int D>
__device__ __forceinline__ float from_below(float v, float ident, int j)
{
    float t = dpp_mov<kRowShr + D>(ident, v);
    if constexpr (J < 16) t = (j >= D) ? t : ident;
    return t;
}

template <int J, int D>
__device__ __forceinline__ float from_above(float v, float ident, int j)
{
    float t = dpp_mov<kRowShl + D>(ident, v);
    if constexpr (J < 16) t = (j + D < J) ? t : ident;
    return t;
}

template <int J, int D = 1>
__device__ __forceinline__ void scan_up_rows(float &r, float &i, int j)
{
    if constexpr (D < J && D < 16) {
        const float tr = from_below<J, D>(r, 1.0f, j), ti = from_below<J, D>(i, 0.0f, j);
        cmul(r, i, tr, ti);
        scan_up_rows<J, 2 * D>(r, i, j);
    }
}

template <int J, int D = 1>
__device__ __forceinline__ void scan_down_rows(float &r, float &i, int j)
{
    if constexpr (D < J && D < 16) {
        const float tr = from_above<J, D>(r, 1.0f, j), ti = from_above<J, D>(i, 0.0f, j);
        cmul(r, i, tr, ti);
        scan_down_rows<J, 2 * D>(r, i, j);
    }
}

// inclusive prefix product: afterwards lane j holds prod_{l <= j}
template <int J>
__device__ __forceinline__ void scan_prefix(float &r, float &i, int lane, int j)
{
    scan_up_rows<J>(r, i, j);
    if constexpr (J >= 32) {                 // odd rows take the total of the row below
        const int src = ((lane | 15) - 16) & 63;
        float tr = __shfl(r, src), ti = __shfl(i, src);
        if (!(lane & 16)) { tr = 1.0f; ti = 0.0f; }
        cmul(r, i, tr, ti);
    }
    if constexpr (J == 64) {                 // rows 2-3 take the total of rows 0-1
        float tr = __shfl(r, 31), ti = __shfl(i, 31);
        if (!(lane & 32)) { tr = 1.0f; ti = 0.0f; }
        cmul(r, i, tr, ti);
    }
}

// inclusive suffix product: afterwards lane j holds prod_{l >= j}
template <int J>
__device__ __forceinline__ void scan_suffix(float &r, float &i, int lane, int j)
{
    scan_down_rows<J>(r, i, j);
    if constexpr (J >= 32) {                 // even rows take the total of the row above
        const int src = ((lane & ~15) + 16) & 63;
        float tr = __shfl(r, src), ti = __shfl(i, src);
        if (lane & 16) { tr = 1.0f; ti = 0.0f; }
        cmul(r, i, tr, ti);
    }
    if constexpr (J == 64) {                 // rows 0-1 take the total of rows 2-3
        float tr = __shfl(r, 32), ti = __shfl(i, 32);
        if (lane & 32) { tr = 1.0f; ti = 0.0f; }
        cmul(r, i, tr, ti);
    }
}

// inclusive -> exclusive (value of lane j-1, identity at j = 0)
template <int J>
__device__ __forceinline__ float prev_lane(float v, float ident, int j)
{
    float t;
    if constexpr (J <= 16) t = dpp_mov<kRowShr + 1>(ident, v);
    else t = __shfl_up(v, 1, J);
    return j == 0 ? ident : t;
}

template <int J>
__device__ __forceinline__ float next_lane(float v, float ident, int j)
{
    float t;
    if constexpr (J <= 16) t = dpp_mov<kRowShl + 1>(ident, v);
    else t = __shfl_down(v, 1, J);
    return j == J - 1 ? ident : t;
}

// Real-valued versions for the root omega^(N/2) = -1 (factor y).
template <int J, int D = 1>
__device__ __forceinline__ void scan_up_rows_real(float &r, int j)
{
    if constexpr (D < J && D < 16) {
        r *= from_below<J, D>(r, 1.0f, j);
        scan_up_rows_real<J, 2 * D>(r, j);
    }
}

template <int J, int D = 1>
__device__ __forceinline__ void scan_down_rows_real(float &r, int j)
{
    if constexpr (D < J && D < 16) {
        r *= from_above<J, D>(r, 1.0f, j);
        scan_down_rows_real<J, 2 * D>(r, j);
    }
}

template <int J>
__device__ __forceinline__ void scan_prefix_real(float &r, int lane, int j)
{
    scan_up_rows_real<J>(r, j);
    if constexpr (J >= 32) {
        const float t = __shfl(r, ((lane | 15) - 16) & 63);
        if (lane & 16) r *= t;
    }
    if constexpr (J == 64) {
        const float t = __shfl(r, 31);
        if (lane & 32) r *= t;
    }
}

template <int J>
__device__ __forceinline__ void scan_suffix_real(float &r, int lane, int j)
{
    scan_down_rows_real<J>(r, j);
    if constexpr (J >= 32) {
        const float t = __shfl(r, ((lane & ~15) + 16) & 63);
        if (!(lane & 16)) r *= t;
    }
    if constexpr (J == 64) {
        const float t = __shfl(r, 32);
        if (!(lane & 32)) r *= t;
    }
}

// ---------------------------------------------------------------------------
// Long constraints: J lanes per restart (64/J restarts per wave), lane j holding
// literals [j*S, j*S + S), S a multiple of 8.  Per root, each lane runs its
// local prefix chain (storing the prefixes) and forms its segment's product;
// exclusive prefix and suffix products across the J lanes then seed the lane's
// suffix chain, which accumulates the adjoint of each literal the lane owns:
// no cross-lane reduction, deterministic order.
// ---------------------------------------------------------------------------
template <int J, int S, bool GRAD>
__global__ __launch_bounds__(kBlock) void fe_grad_seg(FeArgs A)
{
    static_assert(S % 4 == 0 && S >= 8 && S <= 32, "segment length must be 8, 12, ..., 32");
    constexpr int R = kWave / J;
    constexpr int RP = J * S <= 256 ? 16 : 8;     // rescale period (see the table rows)
    const int64_t item = xcd_block() * kWavesPerBlock + wave_id();
    if (item >= A.items) return;
    const int lane = threadIdx.x & 63;
    const int group = (int)(item / A.ntiles);
    const int tile = (int)(item % A.ntiles);
    const int r = lane / J, j = lane % J;
    const int b = group * R + r;
    const bool valid = b < A.B;
    const int bl = valid ? b : A.B - 1;
    const int cbeg = A.c0 + tile * A.tile;
    const int cend = min(cbeg + A.tile, A.c0 + A.nc);
    const int base = j * S;
    const float seed = (GRAD && A.dobj) ? A.dobj[bl] : 1.0f;
    float objacc = 0.f;
    for (int c = cbeg; c < cend; ++c) {
        const int slot0 = A.bc_slot0[c];
        const int k = A.bc_k[c];
        const int tab = A.bc_tab[c];
        const float w = A.bc_w[c];
        const float wg = w * seed;
        unsigned neg = 0;            // bit s: literal s of this lane is negated
        float y[S], adj[S];
#pragma unroll
        for (int s = 0; s < S; ++s) {
            const int i = base + s;
            y[s] = 1.0f;
            adj[s] = 0.f;
            if (i < k) {
                const int lit = A.slot_lit[slot0 + i];
                const int v = (lit > 0 ? lit : -lit) - 1;
                const float xv = A.x[(int64_t)v * A.B + bl];
                y[s] = lit > 0 ? xv : -xv;
                neg |= (lit < 0 ? 1u : 0u) << s;
            }
        }
        const float4 r0 = A.tab[tab];
        float fe = r0.x;
        const int M = k >> 1;
        for (int m = 1; m <= M; ++m) {
            const float4 ra = A.tab[tab + 3 * m - 2];   // {d, Kc}
            const float4 rb = A.tab[tab + 3 * m - 1];   // {alpha^RP, alpha^F}
            const float mt = A.tab[tab + 3 * m].x;      // -tan h
            float z[S], pr[S], pi[S];
#pragma unroll
            for (int s = 0; s < S; ++s) z[s] = mt * y[s];
            float ur = 1.0f, ui = 0.0f;
#pragma unroll
            for (int s = 0; s < S; ++s) {
                if (s > 0 && s % RP == 0) cmul(ur, ui, rb.x, rb.y);
                pr[s] = ur;
                pi[s] = ui;
                mul_unit(ur, ui, z[s]);
            }
            cmul(ur, ui, rb.z, rb.w);                   // the segment's product
            float er = ur, ei = ui;
            scan_prefix<J>(er, ei, lane, j);
            fe = fmaf(2.0f, ra.x * er - ra.y * ei, fe);  // lane J-1: d G
            if (GRAD) {
                float fr = ur, fi = ui;
                scan_suffix<J>(fr, fi, lane, j);
                const float exr = prev_lane<J>(er, 1.0f, j), exi = prev_lane<J>(ei, 0.0f, j);
                const float fxr = next_lane<J>(fr, 1.0f, j), fxi = next_lane<J>(fi, 0.0f, j);
                float sr = wg * ra.z, si = wg * ra.w;
                cmul(sr, si, exr, exi);
                cmul(sr, si, fxr, fxi);
#pragma unroll
                for (int s = S - 1; s >= 0; --s) {
                    adj[s] = fmaf(pr[s], sr, adj[s]);
                    adj[s] = fmaf(-pi[s], si, adj[s]);
                    if (s > 0) {
                        mul_unit(sr, si, z[s]);
                        if (s % RP == 0) cmul(sr, si, rb.x, rb.y);
                    }
                }
            }
        }
        if (k & 1) {
            const float dh = r0.y;
            float q = y[0];
#pragma unroll
            for (int s = 1; s < S; ++s) q *= y[s];
            float e = q;
            scan_prefix_real<J>(e, lane, j);
            fe = fmaf(dh, e, fe);                       // lane J-1: product of all y
            if (GRAD) {
                float f = q;
                scan_suffix_real<J>(f, lane, j);
                e = prev_lane<J>(e, 1.0f, j);
                f = next_lane<J>(f, 1.0f, j);
                float hp[S], h = e;
#pragma unroll
                for (int s = 0; s < S; ++s) {
                    hp[s] = h;
                    h *= y[s];
                }
                float hs = wg * dh * f;
#pragma unroll
                for (int s = S - 1; s >= 0; --s) {
                    adj[s] = fmaf(hp[s], hs, adj[s]);
                    hs *= y[s];
                }
            }
        }
        if (valid) {
            if (GRAD) {
#pragma unroll
                for (int s = 0; s < S; ++s)
                    if (base + s < k)
                        A.adj[(int64_t)(slot0 + base + s) * A.Bp + b] = ((neg >> s) & 1u) ? -adj[s] : adj[s];
            }
            if (A.fe && j == J - 1) A.fe[(int64_t)A.bc_orig[c] * A.B + b] = fe;
        }
        objacc = fmaf(w, fe, objacc);
    }
    if (A.part && j == J - 1) A.part[(int64_t)(A.tile0 + tile) * A.Bp + b] = objacc;
}

template <bool GRAD>
hipError_t dispatch_short(int K, dim3 g, hipStream_t s, const FeArgs &a)
{
#define AFS_SHORT(KK) case KK: hipLaunchKernelGGL((fe_grad_short<KK, GRAD>), g, dim3(kBlock), 0, s, a); break;
    switch (K) {
        AFS_SHORT(1) AFS_SHORT(2) AFS_SHORT(3) AFS_SHORT(4) AFS_SHORT(5) AFS_SHORT(6)
        AFS_SHORT(7) AFS_SHORT(8) AFS_SHORT(9) AFS_SHORT(10) AFS_SHORT(11) AFS_SHORT(12)
        AFS_SHORT(13) AFS_SHORT(14) AFS_SHORT(15) AFS_SHORT(16)
    default: return hipErrorInvalidValue;
    }
#undef AFS_SHORT
    return hipGetLastError();
}

template <int J, bool GRAD>
hipError_t dispatch_seg_s(int S, dim3 g, hipStream_t s, const FeArgs &a)
{
    switch (S) {
    case 8: hipLaunchKernelGGL((fe_grad_seg<J, 8, GRAD>), g, dim3(kBlock), 0, s, a); break;
    case 12: hipLaunchKernelGGL((fe_grad_seg<J, 12, GRAD>), g, dim3(kBlock), 0, s, a); break;
    case 16: hipLaunchKernelGGL((fe_grad_seg<J, 16, GRAD>), g, dim3(kBlock), 0, s, a); break;
    case 20: hipLaunchKernelGGL((fe_grad_seg<J, 20, GRAD>), g, dim3(kBlock), 0, s, a); break;
    case 24: hipLaunchKernelGGL((fe_grad_seg<J, 24, GRAD>), g, dim3(kBlock), 0, s, a); break;
    case 28: hipLaunchKernelGGL((fe_grad_seg<J, 28, GRAD>), g, dim3(kBlock), 0, s, a); break;
    case 32: hipLaunchKernelGGL((fe_grad_seg<J, 32, GRAD>), g, dim3(kBlock), 0, s, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <bool GRAD>
hipError_t dispatch_seg(int J, int S, dim3 g, hipStream_t s, const FeArgs &a)
{
    switch (J) {
    case 2: return dispatch_seg_s<2, GRAD>(S, g, s, a);
    case 4: return dispatch_seg_s<4, GRAD>(S, g, s, a);
    case 8: return dispatch_seg_s<8, GRAD>(S, g, s, a);
    case 16: return dispatch_seg_s<16, GRAD>(S, g, s, a);
    case 32: return dispatch_seg_s<32, GRAD>(S, g, s, a);
    case 64: return dispatch_seg_s<64, GRAD>(S, g, s, a);
    default: return hipErrorInvalidValue;
    }
}

// ---------------------------------------------------------------------------
// Gradient: segmented sum of the per-literal adjoints through the variable ->
// slot transpose.  One wave per (variable, 64 restarts); the slot list is
// wave-uniform and every adjoint row read is a coalesced 256-byte row.
// ---------------------------------------------------------------------------
struct ScatterArgs {
    const float *adj;
    float *grad, *x;
    const int32_t *voff, *vslot, *var_inst;
    int n_inst;
    const uint8_t *fixed, *done;
    uint32_t *bits;
    int32_t *unsat;
    float lr;
    int B, Bp, W, nchunks;
    int64_t items;
};

__device__ __forceinline__ float gather_sum(const ScatterArgs &A, int v, int b)
{
    const int o0 = A.voff[v], o1 = A.voff[v + 1];
    float g = 0.f;
    int o = o0;
    for (; o + 4 <= o1; o += 4) {
        const float a0 = A.adj[(int64_t)A.vslot[o] * A.Bp + b];
        const float a1 = A.adj[(int64_t)A.vslot[o + 1] * A.Bp + b];
        const float a2 = A.adj[(int64_t)A.vslot[o + 2] * A.Bp + b];
        const float a3 = A.adj[(int64_t)A.vslot[o + 3] * A.Bp + b];
        g += a0;
        g += a1;
        g += a2;
        g += a3;
    }
    for (; o < o1; ++o) g += A.adj[(int64_t)A.vslot[o] * A.Bp + b];
    return g;
}

// Projected step of Algorithm 1: x - lr*g clipped to [-1, 1] (NaN stays NaN).
__device__ __forceinline__ float project_step(float xv, float g, float lr)
{
    float t = xv - lr * g;
    t = t > 1.0f ? 1.0f : t;
    t = t < -1.0f ? -1.0f : t;
    return t;
}

__device__ __forceinline__ void store_bits(uint32_t *bits, int v, int W, int chunk, bool neg)
{
    const unsigned long long m = __ballot(neg);
    if ((threadIdx.x & 63) == 0) {
        const int w0 = chunk * 2;
        if (w0 < W) bits[(int64_t)v * W + w0] = (uint32_t)m;
        if (w0 + 1 < W) bits[(int64_t)v * W + w0 + 1] = (uint32_t)(m >> 32);
    }
}

__global__ __launch_bounds__(kBlock) void scatter_grad_kernel(ScatterArgs A)
{
    const int64_t item = (int64_t)blockIdx.x * kWavesPerBlock + wave_id();
    if (item >= A.items) return;
    const int v = (int)(item / A.nchunks), chunk = (int)(item % A.nchunks);
    const int b = chunk * kWave + (threadIdx.x & 63);
    const float g = gather_sum(A, v, b);
    if (b < A.B) A.grad[(int64_t)v * A.B + b] = g;
}

__global__ __launch_bounds__(kBlock) void scatter_step_kernel(ScatterArgs A)
{
    const int64_t item = (int64_t)blockIdx.x * kWavesPerBlock + wave_id();
    if (item >= A.items) return;
    const int v = (int)(item / A.nchunks), chunk = (int)(item % A.nchunks);
    const int b = chunk * kWave + (threadIdx.x & 63);
    const bool valid = b < A.B;
    const float g = gather_sum(A, v, b);
    float xv = 0.f;
    if (valid) {
        const int64_t at = (int64_t)v * A.B + b;
        xv = A.x[at];
        const bool frozen = (A.fixed && A.fixed[v]) || (A.done && A.done[(int64_t)A.var_inst[v] * A.B + b]);
        if (!frozen) {
            xv = project_step(xv, g, A.lr);
            A.x[at] = xv;
        }
        if (v < A.n_inst) A.unsat[(int64_t)v * A.B + b] = 0;
    }
    store_bits(A.bits, v, A.W, chunk, valid && xv < 0.0f);
}

// ---------------------------------------------------------------------------
// Elementwise step, rounding.
// ---------------------------------------------------------------------------
struct EltArgs {
    float *x;
    const float *xin, *grad;
    const int32_t *var_inst;
    int n_inst;
    const uint8_t *fixed, *done;
    uint32_t *bits;
    int32_t *unsat;
    float lr;
    int B, W, nchunks;
    int64_t items;
};

__global__ __launch_bounds__(kBlock) void step_kernel(EltArgs A)
{
    const int64_t item = (int64_t)blockIdx.x * kWavesPerBlock + wave_id();
    if (item >= A.items) return;
    const int v = (int)(item / A.nchunks), chunk = (int)(item % A.nchunks);
    const int b = chunk * kWave + (threadIdx.x & 63);
    if (b >= A.B) return;
    if ((A.fixed && A.fixed[v]) || (A.done && A.done[(int64_t)A.var_inst[v] * A.B + b])) return;
    const int64_t at = (int64_t)v * A.B + b;
    A.x[at] = project_step(A.x[at], A.grad[at], A.lr);
}

__global__ __launch_bounds__(kBlock) void round_kernel(EltArgs A)
{
    const int64_t item = (int64_t)blockIdx.x * kWavesPerBlock + wave_id();
    if (item >= A.items) return;
    const int v = (int)(item / A.nchunks), chunk = (int)(item % A.nchunks);
    const int b = chunk * kWave + (threadIdx.x & 63);
    const bool valid = b < A.B;
    const float xv = valid ? A.xin[(int64_t)v * A.B + b] : 0.f;
    if (valid && v < A.n_inst) A.unsat[(int64_t)v * A.B + b] = 0;
    store_bits(A.bits, v, A.W, chunk, valid && xv < 0.0f);
}

// ---------------------------------------------------------------------------
// Exact verification: per constraint and restart, t = number of true literals
// (variable bit XOR negation), then the integer predicate of its type.
// ---------------------------------------------------------------------------
struct VerifyArgs {
    const uint32_t *bits;
    int32_t *unsat;
    const int32_t *con_off, *lits, *types, *params, *con_inst;
    int B, W, C, tile, ntiles;
    int64_t items;
};


__device__ __forceinline__ bool sat_pred(int type, int k, int param, int t)
{
    switch (type) {
    case 0: return t >= 1;
    case 1: return (t & 1) == (param & 1);
    case 2: return t > 0 && t < k;
    case 3: return t >= param;
    case 4: return t < param;
    case 5: return t <= 1;
    case 6: return t == 1;
    default: return t == param;
    }
}

__global__ __launch_bounds__(kBlock) void verify_kernel(VerifyArgs A)
{
    const int64_t item = xcd_block() * kWavesPerBlock + wave_id();
    if (item >= A.items) return;
    const int group = (int)(item / A.ntiles), tile = (int)(item % A.ntiles);
    const int b = group * kWave + (threadIdx.x & 63);
    const bool valid = b < A.B;
    const int wi = (valid ? b : A.B - 1) >> 5;
    const int sh = b & 31;
    const int cbeg = tile * A.tile, cend = min(cbeg + A.tile, A.C);
    int cnt = 0;
    int inst = cbeg < cend ? A.con_inst[cbeg] : 0;
    for (int c = cbeg; c < cend; ++c) {
        const int ci = A.con_inst[c];
        if (ci != inst) {                        // constraints of one sub-instance are contiguous
            if (valid && cnt) atomicAdd(&A.unsat[(int64_t)inst * A.B + b], cnt);
            cnt = 0;
            inst = ci;
        }
        const int o0 = A.con_off[c], o1 = A.con_off[c + 1];
        int t = 0;
#pragma unroll 4
        for (int o = o0; o < o1; ++o) {
            const int l = A.lits[o];
            const int v = (l > 0 ? l : -l) - 1;
            const uint32_t word = A.bits[(int64_t)v * A.W + wi];
            t += (int)((word >> sh) & 1u) ^ (l < 0 ? 1 : 0);
        }
        cnt += sat_pred(A.types[c], o1 - o0, A.params[c], t) ? 0 : 1;
    }
    if (valid && cnt) atomicAdd(&A.unsat[(int64_t)inst * A.B + b], cnt);
}

// One block: done / first_sat bookkeeping and the {t, number done} counter.
__global__ __launch_bounds__(1024) void finalize_kernel(int count, const int32_t *unsat, uint8_t *done,
                                                        int32_t *first_sat, int32_t *counter, int mode)
{
    __shared__ int red[1024 / kWave];
    const int t = (mode == FIN_STEP) ? counter[0] + 1 : 0;
    __syncthreads();
    int cnt = 0;
    for (int b = threadIdx.x; b < count; b += blockDim.x) {
        const bool ok = unsat[b] == 0;
        if (mode == FIN_INIT) {
            done[b] = ok ? 1 : 0;
            first_sat[b] = ok ? 0 : -1;
            cnt += ok;
        } else if (mode == FIN_STEP) {
            uint8_t d = done[b];
            if (!d && ok) {
                done[b] = d = 1;
                first_sat[b] = t;
            }
            cnt += d;
        } else {
            if (ok) done[b] = 1;
        }
    }
    if (mode == FIN_VERIFY) return;
    for (int off = 32; off > 0; off >>= 1) cnt += __shfl_down(cnt, off);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = cnt;
    __syncthreads();
    if (threadIdx.x == 0) {
        int total = 0;
        for (int i = 0; i < (int)(blockDim.x / kWave); ++i) total += red[i];
        counter[0] = t;
        counter[1] = total;
    }
}

// ---------------------------------------------------------------------------
// Objective: fixed-order two-pass sum of the per-tile partials.
// ---------------------------------------------------------------------------
constexpr int kRedGroup = 32;

__global__ __launch_bounds__(kWave) void obj_reduce1(int tiles, int Bp, const float *part, float *part2)
{
    const int chunk = blockIdx.x, g = blockIdx.y;
    const int b = chunk * kWave + threadIdx.x;
    const int t0 = g * kRedGroup, t1 = min(t0 + kRedGroup, tiles);
    float s = 0.f;
    for (int t = t0; t < t1; ++t) s += part[(int64_t)t * Bp + b];
    part2[(int64_t)g * Bp + b] = s;
}

__global__ __launch_bounds__(kBlock) void obj_reduce2(int groups, int B, int Bp, const float *part2, float *obj)
{
    const int b = blockIdx.x * kBlock + threadIdx.x;
    if (b >= B) return;
    float s = 0.f;
    for (int g = 0; g < groups; ++g) s += part2[(int64_t)g * Bp + b];
    obj[b] = s;
}

__global__ __launch_bounds__(kBlock) void permute_adj_kernel(const float *adj, float *out,
                                                             const int32_t *slot_to_lit, int B, int Bp,
                                                             int nchunks, int64_t items)
{
    const int64_t item = (int64_t)blockIdx.x * kWavesPerBlock + wave_id();
    if (item >= items) return;
    const int64_t s = item / nchunks;
    const int chunk = (int)(item % nchunks);
    const int b = chunk * kWave + (threadIdx.x & 63);
    if (b < B) out[(int64_t)slot_to_lit[s] * B + b] = adj[s * Bp + b];
}

inline dim3 grid_for_waves(int64_t items)
{
    return dim3((unsigned)((items + kWavesPerBlock - 1) / kWavesPerBlock));
}

}  // namespace

hipError_t launch_fe_grad(const DevInstance &I, const BucketLaunch &bk, int B, int Bp,
                          const float *x, float *adj, float *part, float *fe, const float *dobj,
                          bool grad, hipStream_t s)
{
    if (bk.nc == 0 || B == 0) return hipSuccess;
    FeArgs a;
    a.x = x; a.adj = adj; a.part = part; a.fe = fe; a.dobj = dobj;
    a.bc_slot0 = I.bc_slot0; a.bc_k = I.bc_k; a.bc_tab = I.bc_tab; a.bc_orig = I.bc_orig;
    a.bc_w = I.bc_w; a.slot_lit = I.slot_lit; a.tab = I.tab;
    a.B = B; a.Bp = Bp;
    a.c0 = bk.c0; a.nc = bk.nc; a.tile = bk.tile; a.ntiles = bk.ntiles; a.tile0 = bk.tile0;
    const int R = kWave / bk.J;
    const int64_t groups = (B + R - 1) / R;
    a.items = groups * bk.ntiles;
    const dim3 g = grid_for_waves(a.items);
    if (grad) return bk.J == 1 ? dispatch_short<true>(bk.S, g, s, a) : dispatch_seg<true>(bk.J, bk.S, g, s, a);
    return bk.J == 1 ? dispatch_short<false>(bk.S, g, s, a) : dispatch_seg<false>(bk.J, bk.S, g, s, a);
}

static ScatterArgs scatter_args(const DevInstance &I, int B, int Bp, const float *adj)
{
    ScatterArgs a{};
    a.adj = adj;
    a.voff = I.voff; a.vslot = I.vslot; a.var_inst = I.var_inst; a.n_inst = I.n_inst;
    a.B = B; a.Bp = Bp; a.W = (B + 31) / 32;
    a.nchunks = Bp / kWave;
    a.items = (int64_t)I.n * a.nchunks;
    return a;
}

hipError_t launch_scatter(const DevInstance &I, int B, int Bp, const float *adj, float *grad,
                          hipStream_t s)
{
    if (B == 0) return hipSuccess;
    ScatterArgs a = scatter_args(I, B, Bp, adj);
    a.grad = grad;
    hipLaunchKernelGGL(scatter_grad_kernel, grid_for_waves(a.items), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_scatter_step(const DevInstance &I, int B, int Bp, const float *adj, float *x,
                               float lr, const uint8_t *fixed, const uint8_t *done,
                               uint32_t *bits, int32_t *unsat, hipStream_t s)
{
    if (B == 0) return hipSuccess;
    ScatterArgs a = scatter_args(I, B, Bp, adj);
    a.x = x; a.lr = lr; a.fixed = fixed; a.done = done; a.bits = bits; a.unsat = unsat;
    hipLaunchKernelGGL(scatter_step_kernel, grid_for_waves(a.items), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_obj_reduce(int tiles, int B, int Bp, const float *part, float *part2,
                             float *obj, hipStream_t s)
{
    if (B == 0) return hipSuccess;
    const int groups = (tiles + kRedGroup - 1) / kRedGroup;
    if (groups > 0)
        hipLaunchKernelGGL(obj_reduce1, dim3(Bp / kWave, groups), dim3(kWave), 0, s, tiles, Bp, part, part2);
    hipLaunchKernelGGL(obj_reduce2, dim3((B + kBlock - 1) / kBlock), dim3(kBlock), 0, s, groups, B, Bp,
                       part2, obj);
    return hipGetLastError();
}

static EltArgs elt_args(int n, int B)
{
    EltArgs a{};
    a.B = B;
    a.W = (B + 31) / 32;
    a.nchunks = (B + kWave - 1) / kWave;
    a.items = (int64_t)n * a.nchunks;
    return a;
}

hipError_t launch_step(const DevInstance &I, int B, float *x, const float *grad, float lr,
                       const uint8_t *fixed, const uint8_t *done, hipStream_t s)
{
    if (B == 0) return hipSuccess;
    EltArgs a = elt_args(I.n, B);
    a.x = x; a.grad = grad; a.lr = lr; a.fixed = fixed; a.done = done;
    a.var_inst = I.var_inst; a.n_inst = I.n_inst;
    hipLaunchKernelGGL(step_kernel, grid_for_waves(a.items), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_round(const DevInstance &I, int B, const float *x, uint32_t *bits, int32_t *unsat,
                        hipStream_t s)
{
    if (B == 0) return hipSuccess;
    EltArgs a = elt_args(I.n, B);
    a.xin = x; a.bits = bits; a.unsat = unsat;
    a.var_inst = I.var_inst; a.n_inst = I.n_inst;
    hipLaunchKernelGGL(round_kernel, grid_for_waves(a.items), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_verify(const DevInstance &I, int B, const uint32_t *bits, int32_t *unsat,
                         hipStream_t s)
{
    if (B == 0 || I.C == 0) return hipSuccess;
    VerifyArgs a{};
    a.bits = bits; a.unsat = unsat;
    a.con_off = I.con_off; a.lits = I.lits; a.types = I.types; a.params = I.params;
    a.con_inst = I.con_inst;
    a.B = B; a.W = (B + 31) / 32; a.C = I.C;
    a.tile = 32;
    a.ntiles = (I.C + a.tile - 1) / a.tile;
    a.items = (int64_t)((B + kWave - 1) / kWave) * a.ntiles;
    hipLaunchKernelGGL(verify_kernel, grid_for_waves(a.items), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_finalize(int count, const int32_t *unsat, uint8_t *done, int32_t *first_sat,
                           int32_t *counter, int mode, hipStream_t s)
{
    if (count == 0) return hipSuccess;
    hipLaunchKernelGGL(finalize_kernel, dim3(1), dim3(1024), 0, s, count, unsat, done, first_sat, counter, mode);
    return hipGetLastError();
}

hipError_t launch_permute_adj(const DevInstance &I, int B, int Bp, const float *adj,
                              float *adj_out, hipStream_t s)
{
    if (B == 0 || I.L == 0) return hipSuccess;
    const int nchunks = Bp / kWave;
    const int64_t items = I.L * nchunks;
    hipLaunchKernelGGL(permute_adj_kernel, grid_for_waves(items), dim3(kBlock), 0, s, adj, adj_out,
                       I.slot_to_lit, B, Bp, nchunks, items);
    return hipGetLastError();
}

}  // namespace afs
