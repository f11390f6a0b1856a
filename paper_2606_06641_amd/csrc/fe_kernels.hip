// fe_kernels.hip -- FE and adjoint kernels for gfx950 (CDNA4, wave64).
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

#include <cstdint>

#include "device_common.hpp"

namespace afs {

namespace {

using namespace dev;

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
    const uint8_t *skip;        // per restart: nonzero = not needed (NULL: all needed)
    const int32_t *bc_slot0, *bc_k, *bc_tab, *bc_orig;
    const float *bc_w;
    const int32_t *slot_lit;
    const float4 *tab;
    int64_t tab_rows;            // rows of tab
    int B, Bp;
    int32_t c0, nc, tile, ntiles, tile0;
    int64_t items, item0;        // all items; first item of this launch
};

// ---------------------------------------------------------------------------
// Factor form shared by the FE kernels.  With h = pi m / N, c = cos h and
// alpha = (1 + omega^m)/2 = c e^{i h}, the factor of a literal with value y is
//     a = (1-p) + p omega^m = alpha (1 + i z),   z = -tan(h) y,
// so one step of a product chain multiplies by (1 + i z): two FMAs.  Since
// |1 + i z| <= 1/c, the segment kernels multiply their running products by the
// real c^RP after every RP literals (RP = 16 for lengths <= 256, else 8) and by
// c^F at the end of the segment; every phase e^{i n h} of the alpha powers is a
// constant folded into the table rows (host.cpp, append_root_rows).  Padding
// literals hold y = +1, whose factor alpha (1 - i tan h) is exactly 1.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void mul_unit(float &r, float &i, float z)
{
    const float nr = fmaf(-i, z, r);
    i = fmaf(r, z, i);
    r = nr;
}

// A wave-uniform value (a table entry read through the scalar cache) copied
// into a vector register once per root, so that the per-literal instructions
// that use it read no scalar register: gfx950 issues a VALU instruction with a
// scalar-register operand at half the rate of one with vector operands only.
__device__ __forceinline__ float in_vgpr(float s)
{
    float v;
    asm("v_mov_b32 %0, %1" : "=v"(v) : "s"(s));
    return v;
}

// The table seen as a buffer resource of tab_rows 16-byte rows (fewer than 2^27:
// the packing refuses more; the fourth word is the raw-buffer setting for this
// architecture): a read through it is an intrinsic call, which the compiler
// does not merge into other reads, and a read past the end returns zero.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t table_rsrc(const float4 *T, int64_t rows)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<float4 *>(T), (short)0, (int)(rows * 16), 0x00020000);
}

typedef float f32x2 __attribute__((ext_vector_type(2)));

// The first two constants of table row `row` into vector registers.  The
// segment kernels with long segments read the next root's -tan h and rescale
// factor this way while the current root runs: the first per-literal products
// of a root then need no scalar-cache read, whose wait would cover every scalar
// read in flight.
__device__ __forceinline__ f32x2 row_head(__amdgpu_buffer_rsrc_t rs, int row)
{
    return __builtin_bit_cast(f32x2, __builtin_amdgcn_raw_buffer_load_b64(rs, row * 16, 0, 0));
}

// The same step for a product held as (re, -im) =: (r, n): re' = r + n z and
// -im' = n - r z.  The suffix chains are held this way so that the adjoint
// contraction Re(P S) = Pr Sr + Pi n takes two plain multiply-accumulates
// (v_fmac_f32, which gfx950 issues at twice the rate of the three-address
// v_fma_f32 that a negated operand needs).  Negation is exact, so the values
// are those of mul_unit bit for bit.
__device__ __forceinline__ void mul_unit_conj(float &r, float &n, float z)
{
    const float nn = fmaf(-r, z, n);
    r = fmaf(n, z, r);
    n = nn;
}

// ---------------------------------------------------------------------------
// Short constraints (k <= 16): one lane per RPL consecutive restarts, k known at
// compile time, the whole constraint in registers.  A wave takes 64*RPL restarts
// and a tile of constraints of the bucket; with RPL = 2 or 4 (B a multiple of
// RPL) the x rows are read and the adjoint rows written as 8- or 16-byte vectors
// and the constraint's metadata, literal addresses and table rows serve RPL
// restarts.  The weight (and the adjoint seed) multiplies each literal's adjoint
// once, after the roots.
// ---------------------------------------------------------------------------
template <int RPL>
struct Lanes {
    float v[RPL];
};

template <int RPL>
__device__ __forceinline__ void load_lanes(const float *p, Lanes<RPL> &out)
{
    if constexpr (RPL == 4) {
        const float4 q = *reinterpret_cast<const float4 *>(p);
        out.v[0] = q.x; out.v[1] = q.y; out.v[2] = q.z; out.v[3] = q.w;
    } else if constexpr (RPL == 2) {
        const float2 q = *reinterpret_cast<const float2 *>(p);
        out.v[0] = q.x; out.v[1] = q.y;
    } else {
#pragma unroll
        for (int e = 0; e < RPL; ++e) out.v[e] = p[e];
    }
}

typedef float f32x4 __attribute__((ext_vector_type(4)));

template <int RPL>
__device__ __forceinline__ void store_lanes_stream(float *p, const Lanes<RPL> &in)
{
    if constexpr (RPL == 4) {
        f32x4 q = {in.v[0], in.v[1], in.v[2], in.v[3]};
        __builtin_nontemporal_store(q, reinterpret_cast<f32x4 *>(p));
    } else if constexpr (RPL == 2) {
        f32x2 q = {in.v[0], in.v[1]};
        __builtin_nontemporal_store(q, reinterpret_cast<f32x2 *>(p));
    } else {
#pragma unroll
        for (int e = 0; e < RPL; ++e) __builtin_nontemporal_store(in.v[e], p + e);
    }
}

template <int K, int RPL, bool GRAD>
__global__ __launch_bounds__(kBlock) void fe_grad_short(FeArgs A, const float4 *__restrict__ T)
{
    const uint32_t item = (uint32_t)A.item0 + xcd_block() * kWavesPerBlock + wave_id();
    if (item >= (uint32_t)A.items) return;
    const int lane = threadIdx.x & 63;
    const uint32_t group = item / (uint32_t)A.ntiles;
    const int tile = (int)(item - group * (uint32_t)A.ntiles);
    const int b0 = ((int)group * kWave + lane) * RPL;          // first restart of the lane
    const bool valid = b0 < A.B;                               // RPL divides B
    const int bl = valid ? b0 : A.B - RPL;
    if (A.skip) {                                              // a wave whose restarts are all skipped
        bool need = false;
#pragma unroll
        for (int e = 0; e < RPL; ++e) need |= valid && !A.skip[b0 + e];
        if (__ballot(need) == 0) return;
    }
    const int cbeg = A.c0 + tile * A.tile;
    const int cend = min(cbeg + A.tile, A.c0 + A.nc);
    Lanes<RPL> seed;
#pragma unroll
    for (int e = 0; e < RPL; ++e) seed.v[e] = (GRAD && A.dobj) ? A.dobj[bl + e] : 1.0f;
    float objacc[RPL];
#pragma unroll
    for (int e = 0; e < RPL; ++e) objacc[e] = 0.f;
    for (int c = cbeg; c < cend; ++c) {
        const int slot0 = A.bc_slot0[c];
        const int tab = A.bc_tab[c];
        const float w = A.bc_w[c];
        int lit[K];
        Lanes<RPL> y[K], adj[K];
#pragma unroll
        for (int i = 0; i < K; ++i) {
            lit[i] = A.slot_lit[slot0 + i];
            const int v = (lit[i] > 0 ? lit[i] : -lit[i]) - 1;
            load_lanes<RPL>(A.x + (int64_t)v * A.B + bl, y[i]);
#pragma unroll
            for (int e = 0; e < RPL; ++e) {
                y[i].v[e] = lit[i] > 0 ? y[i].v[e] : -y[i].v[e];
                adj[i].v[e] = 0.f;
            }
        }
        const float4 r0 = T[tab];
        float fe[RPL];
#pragma unroll
        for (int e = 0; e < RPL; ++e) fe[e] = r0.x;
        // Roots one at a time (unrolling them multiplies register use by K/2).
#pragma unroll 1
        for (int m = 1; m <= K / 2; ++m) {
            const float4 ra = T[tab + 2 * m - 1];       // {2 d alpha^K, Kc}
            const float4 rb = T[tab + 2 * m];           // {-, -, -tan h, -}
            const float mt = in_vgpr(rb.z);
#pragma unroll
            for (int e = 0; e < RPL; ++e) {
                float z[K], pr[K], pi[K];
#pragma unroll
                for (int i = 0; i < K; ++i) z[i] = mt * y[i].v[e];
                // |1 + i z|^K stays far below 2^128 for K <= 16; the prefix of literal 0
                // is exactly 1 and the running product after it exactly (1, z_0)
                float ur = 1.0f, ui = z[0];
#pragma unroll
                for (int i = 1; i < K; ++i) {
                    pr[i] = ur;
                    pi[i] = ui;
                    mul_unit(ur, ui, z[i]);
                }
                fe[e] = fmaf(ra.x, ur, fe[e]);          // Re(2 d alpha^K G)
                fe[e] = fmaf(-ra.y, ui, fe[e]);
                if (GRAD) {
                    float sr = ra.z, sn = -ra.w;        // suffix chain, held as (re, -im)
#pragma unroll
                    for (int i = K - 1; i >= 1; --i) {
                        adj[i].v[e] = fmaf(pr[i], sr, adj[i].v[e]);
                        adj[i].v[e] = fmaf(pi[i], sn, adj[i].v[e]);
                        mul_unit_conj(sr, sn, z[i]);
                    }
                    adj[0].v[e] += sr;
                }
            }
        }
        if (K & 1) {                       // real root omega^(N/2) = -1: factor y_i
            const float dh = r0.y;
#pragma unroll
            for (int e = 0; e < RPL; ++e) {
                float hp[K], h = 1.0f;
#pragma unroll
                for (int i = 0; i < K; ++i) {
                    hp[i] = h;
                    h *= y[i].v[e];
                }
                fe[e] = fmaf(dh, h, fe[e]);
                if (GRAD) {
                    float hs = dh;
#pragma unroll
                    for (int i = K - 1; i >= 0; --i) {
                        adj[i].v[e] = fmaf(hp[i], hs, adj[i].v[e]);
                        hs *= y[i].v[e];
                    }
                }
            }
        }
        if (valid) {
            if (GRAD) {
#pragma unroll
                for (int i = 0; i < K; ++i) {
                    const float ws = lit[i] > 0 ? w : -w;
#pragma unroll
                    for (int e = 0; e < RPL; ++e) adj[i].v[e] *= ws * seed.v[e];
                    store_lanes_stream<RPL>(A.adj + (int64_t)(slot0 + i) * A.Bp + b0, adj[i]);
                }
            }
            if (A.fe) {
#pragma unroll
                for (int e = 0; e < RPL; ++e) A.fe[(int64_t)A.bc_orig[c] * A.B + b0 + e] = fe[e];
            }
        }
#pragma unroll
        for (int e = 0; e < RPL; ++e) objacc[e] = fmaf(w, fe[e], objacc[e]);
    }
    if (A.part && valid) {
#pragma unroll
        for (int e = 0; e < RPL; ++e) A.part[(int64_t)(A.tile0 + tile) * A.Bp + b0 + e] = objacc[e];
    }
}

// ---------------------------------------------------------------------------
// Cross-lane products over the J lanes that share one restart, as a butterfly:
// at level D every lane takes the running product of the partner half-group
// (lanes differing in bit D) and multiplies it both into the group total and
// into the product of the lanes other than itself.  The partner half-groups of
// the log2(J) levels partition the other lanes, so afterwards every lane holds
// the total and the product of all segments but its own -- the two quantities
// the FE and the adjoint need -- without separate prefix and suffix scans.
// Levels 1, 2, 4 and 8 stay inside a 16-lane row (DPP quad_perm and the row
// mirrors); 16 uses ds_swizzle, 32 a bpermute.
// ---------------------------------------------------------------------------
// DPP permutation inside 16-lane rows.  Every lane reads a lane of its own row,
// so no lane keeps its previous value and none is passed in: the move needs no
// copy of its source first.
template <int CTRL>
__device__ __forceinline__ float row_perm(float v)
{
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, false));
}

// value held by some lane of the other half of this lane's 2D-group
template <int D>
__device__ __forceinline__ float partner(float v)
{
    if constexpr (D == 1) return row_perm<0xB1>(v);         // quad_perm [1,0,3,2]
    else if constexpr (D == 2) return row_perm<0x4E>(v);    // quad_perm [2,3,0,1]
    else if constexpr (D == 4) return row_perm<0x141>(v);   // row_half_mirror: i -> 7-i
    else if constexpr (D == 8) return row_perm<0x140>(v);   // row_mirror: i -> 15-i
    else if constexpr (D == 16)                            // swizzle xor 16 within 32 lanes
        return __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(v), 0x401F));
    else return __shfl_xor(v, 32);
}

// (gr, gi): own segment product in, group total out; (xr, xi): product of the other lanes
template <int J, int D = 1>
__device__ __forceinline__ void butterfly(float &gr, float &gi, float &xr, float &xi)
{
    if constexpr (D < J) {
        const float wr = partner<D>(gr), wi = partner<D>(gi);
        if constexpr (D == 1) {
            xr = wr;
            xi = wi;
        } else {
            cmul(xr, xi, wr, wi);
        }
        cmul(gr, gi, wr, wi);
        butterfly<J, 2 * D>(gr, gi, xr, xi);
    }
}

// Real-valued version for the root omega^(N/2) = -1 (factor y).
template <int J, int D = 1>
__device__ __forceinline__ void butterfly_real(float &g, float &x)
{
    if constexpr (D < J) {
        const float w = partner<D>(g);
        x = D == 1 ? w : x * w;
        g *= w;
        butterfly_real<J, 2 * D>(g, x);
    }
}

// ---------------------------------------------------------------------------
// Long constraints: J lanes per restart (64/J restarts per wave), lane j holding
// literals [j*S, j*S + S), S even in [4, 32].  Per root, each lane
// runs its local prefix chain (storing the prefixes) and forms its segment's
// product; the butterfly gives every lane the total and the product of the other
// lanes' segments, which seeds the lane's suffix chain; that chain accumulates
// the adjoint of each literal the lane owns: no cross-lane reduction of
// adjoints, deterministic order.
// ---------------------------------------------------------------------------
// The points of this lane's literals of constraint c, unsigned (x as stored; the
// signs go into neg, bit s for literal s), padding literals 1.  The sign is
// applied when the values are used, so the loads can stay in flight meanwhile.
template <int S>
__device__ __forceinline__ void fetch_points(const FeArgs &A, int c, int base, int bl, float (&xv)[S], unsigned &neg)
{
    const int slot0 = A.bc_slot0[c];
    const int k = A.bc_k[c];
    neg = 0;
#pragma unroll
    for (int s = 0; s < S; ++s) {
        const int i = base + s;
        xv[s] = 1.0f;
        if (i < k) {
            const int lit = A.slot_lit[slot0 + i];
            const int v = (lit > 0 ? lit : -lit) - 1;
            xv[s] = A.x[(int64_t)v * A.B + bl];
            neg |= (lit < 0 ? 1u : 0u) << s;
        }
    }
}

// Minimum resident waves per SIMD asked of the compiler for a segment length.
// Left to itself it gives segments of 22 literals 155 VGPRs (three waves) and
// of 26 to 32 literals 177 to 215 (two waves).  Asked for one wave more, it
// fits 22 in 128 VGPRs and 26 to 32 in 168, spilling 28 bytes per lane for 22,
// none for 26 and 28, 32 for 30 and 264 for 32, and the kernels still run
// faster: the segment of 32 by about a tenth.  The same request for 24 (four
// waves) or for 16 to 20 (five) loses.  J = 64 is left alone.
constexpr int seg_min_waves(int J, int S)
{
    if (J > 32) return 1;
    if (S == 22) return 4;
    if (S >= 26) return 3;
    return 1;
}

template <int J, int S, bool GRAD>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(seg_min_waves(J, S)))) void fe_grad_seg(FeArgs A, const float4 *__restrict__ T)
{
    static_assert(S % 2 == 0 && S >= 4 && S <= 32, "segment length must be even, 4 to 32");
    constexpr int R = kWave / J;
    constexpr int RP = J * S <= 256 ? 16 : 8;     // rescale period (see the table rows)
    const uint32_t item = (uint32_t)A.item0 + xcd_block() * kWavesPerBlock + wave_id();
    if (item >= (uint32_t)A.items) return;
    const int lane = threadIdx.x & 63;
    // The kWavesPerBlock waves of a block take consecutive restart groups of one
    // tile, so that together they write whole 128-byte lines of each adjoint row;
    // blocks then run over the tiles, and over groups of kWavesPerBlock groups last.
    const uint32_t per = kWavesPerBlock * (uint32_t)A.ntiles;
    const uint32_t gb = item / per, rem = item - gb * per;
    const int tile = (int)(rem / kWavesPerBlock);
    const int group = (int)(gb * kWavesPerBlock + rem % kWavesPerBlock);
    if (group * R >= A.B) return;                 // padding group past the last restart
    const int r = lane / J, j = lane % J;
    const int b = group * R + r;
    const bool valid = b < A.B;
    const int bl = valid ? b : A.B - 1;
    if (A.skip && __ballot(valid && !A.skip[b]) == 0) return;   // every restart of the wave skipped
    const int cbeg = A.c0 + tile * A.tile;
    const int cend = min(cbeg + A.tile, A.c0 + A.nc);
    const int base = j * S;
    const float seed = (GRAD && A.dobj) ? A.dobj[bl] : 1.0f;
    // Long segments read the next root's first constants through the vector path
    // (a vector read's latency, a few hundred cycles, needs a root of 18 or more
    // literals per lane to hide; shorter ones wait on the scalar read instead).
    constexpr bool kHeadAhead = S >= 18;
    const __amdgpu_buffer_rsrc_t rs = table_rsrc(T, A.tab_rows);
    // With several constraints per wave and short segments (few registers), the
    // next constraint's points are gathered while this one's roots run.
    constexpr bool kAhead = J <= 4 && S <= 12;
    float xn[S];
    unsigned negn = 0;
    if (kAhead && cbeg < cend) fetch_points<S>(A, cbeg, base, bl, xn, negn);
    float objacc = 0.f;
    for (int c = cbeg; c < cend; ++c) {
        const int slot0 = A.bc_slot0[c];
        const int k = A.bc_k[c];
        const int tab = A.bc_tab[c];
        const float w = A.bc_w[c];
        const float wg = w * seed;
        unsigned neg = 0;            // bit s: literal s of this lane is negated
        float y[S], adj[S];
        if constexpr (kAhead) {
            neg = negn;
#pragma unroll
            for (int s = 0; s < S; ++s) {
                y[s] = ((neg >> s) & 1u) ? -xn[s] : xn[s];
                adj[s] = 0.f;
            }
            if (c + 1 < cend) fetch_points<S>(A, c + 1, base, bl, xn, negn);
        } else {
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
        }
        const float4 r0 = T[tab];
        float fe = r0.x;
        const int M = k >> 1;                          // >= 8: k > 16 here
        f32x2 nh = {0.f, 0.f};                         // {-tan h, c^RP} of the next root
        if constexpr (kHeadAhead) nh = row_head(rs, tab + 2);
        for (int m = 1; m <= M; ++m) {
            const float4 ra = T[tab + 2 * m - 1];       // {2 d', Kc}
            const float4 rb = T[tab + 2 * m];           // {-tan h, c^RP, c^F, 0}
            float mt, crp;
            if constexpr (kHeadAhead) {
                mt = nh.x;
                crp = nh.y;
                nh = row_head(rs, tab + 2 * min(m + 1, M));
                __builtin_amdgcn_sched_barrier(0);      // the read goes out before the root's work
            } else {
                mt = in_vgpr(rb.x);
                crp = in_vgpr(rb.y);
            }
            float z[S], pr[S], pi[S];
#pragma unroll
            for (int s = 0; s < S; ++s) z[s] = mt * y[s];
            // prefix chain; the prefix of literal 0 is exactly 1, and after it the
            // running product is exactly (1, z_0)
            float ur = 1.0f, ui = z[0];
#pragma unroll
            for (int s = 1; s < S; ++s) {
                if (s % RP == 0) {                      // real rescale; its phase is in the rows
                    ur *= crp;
                    ui *= crp;
                }
                pr[s] = ur;
                pi[s] = ui;
                mul_unit(ur, ui, z[s]);
            }
            ur *= rb.z;                                 // the segment's product, scaled by c^F
            ui *= rb.z;
            float gr = ur, gi = ui, xr = 1.0f, xi = 0.0f;
            butterfly<J>(gr, gi, xr, xi);
            fe = fmaf(ra.x, gr, fe);                    // Re(2 d' G)
            fe = fmaf(-ra.y, gi, fe);
            if (GRAD) {
                float sr = ra.z, si = ra.w;
                cmul(sr, si, xr, xi);
                float sn = -si;                         // suffix chain, held as (re, -im)
#pragma unroll
                for (int s = S - 1; s >= 1; --s) {
                    adj[s] = fmaf(pr[s], sr, adj[s]);
                    adj[s] = fmaf(pi[s], sn, adj[s]);
                    mul_unit_conj(sr, sn, z[s]);
                    if (s % RP == 0) {
                        sr *= crp;
                        sn *= crp;
                    }
                }
                adj[0] += sr;                           // prefix of literal 0: exactly 1
            }
        }
        if (k & 1) {
            const float dh = r0.y;
            float q = y[0];
#pragma unroll
            for (int s = 1; s < S; ++s) q *= y[s];
            float x = 1.0f;
            butterfly_real<J>(q, x);
            fe = fmaf(dh, q, fe);                       // d_{N/2} times the product of all y
            if (GRAD) {
                float hp[S], h = 1.0f;
#pragma unroll
                for (int s = 0; s < S; ++s) {
                    hp[s] = h;
                    h *= y[s];
                }
                float hs = dh * x;
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
                        A.adj[(int64_t)(slot0 + base + s) * A.Bp + b] = ((neg >> s) & 1u) ? -wg * adj[s] : wg * adj[s];
            }
            if (A.fe && j == J - 1) A.fe[(int64_t)A.bc_orig[c] * A.B + b] = fe;
        }
        objacc = fmaf(w, fe, objacc);
    }
    if (A.part && j == J - 1) A.part[(int64_t)(A.tile0 + tile) * A.Bp + b] = objacc;
}

template <bool GRAD>
hipError_t dispatch_short(int K, int rpl, dim3 g, hipStream_t s, const FeArgs &a)
{
#define AFS_SHORT(KK) case KK:                                                                        \
    if constexpr (KK <= 8) {                                                                         \
        if (rpl == 4) {                                                                              \
            hipLaunchKernelGGL((fe_grad_short<KK, 4, GRAD>), g, dim3(kBlock), 0, s, a, a.tab);              \
            break;                                                                                   \
        }                                                                                            \
    }                                                                                                \
    if (rpl == 2) {                                                                                  \
        hipLaunchKernelGGL((fe_grad_short<KK, 2, GRAD>), g, dim3(kBlock), 0, s, a, a.tab);                  \
        break;                                                                                       \
    }                                                                                                \
    hipLaunchKernelGGL((fe_grad_short<KK, 1, GRAD>), g, dim3(kBlock), 0, s, a, a.tab);                      \
    break;
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
    case 4: hipLaunchKernelGGL((fe_grad_seg<J, 4, GRAD>), g, dim3(kBlock), 0, s, a, a.tab); break;
    case 6: hipLaunchKernelGGL((fe_grad_seg<J, 6, GRAD>), g, dim3(kBlock), 0, s, a, a.tab); break;
    case 8: hipLaunchKernelGGL((fe_grad_seg<J, 8, GRAD>), g, dim3(kBlock), 0, s, a, a.tab); break;
    case 10: hipLaunchKernelGGL((fe_grad_seg<J, 10, GRAD>), g, dim3(kBlock), 0, s, a, a.tab); break;
    case 12: hipLaunchKernelGGL((fe_grad_seg<J, 12, GRAD>), g, dim3(kBlock), 0, s, a, a.tab); break;
    case 14: hipLaunchKernelGGL((fe_grad_seg<J, 14, GRAD>), g, dim3(kBlock), 0, s, a, a.tab); break;
    case 16: hipLaunchKernelGGL((fe_grad_seg<J, 16, GRAD>), g, dim3(kBlock), 0, s, a, a.tab); break;
    case 18: hipLaunchKernelGGL((fe_grad_seg<J, 18, GRAD>), g, dim3(kBlock), 0, s, a, a.tab); break;
    case 20: hipLaunchKernelGGL((fe_grad_seg<J, 20, GRAD>), g, dim3(kBlock), 0, s, a, a.tab); break;
    case 22: hipLaunchKernelGGL((fe_grad_seg<J, 22, GRAD>), g, dim3(kBlock), 0, s, a, a.tab); break;
    case 24: hipLaunchKernelGGL((fe_grad_seg<J, 24, GRAD>), g, dim3(kBlock), 0, s, a, a.tab); break;
    case 26: hipLaunchKernelGGL((fe_grad_seg<J, 26, GRAD>), g, dim3(kBlock), 0, s, a, a.tab); break;
    case 28: hipLaunchKernelGGL((fe_grad_seg<J, 28, GRAD>), g, dim3(kBlock), 0, s, a, a.tab); break;
    case 30: hipLaunchKernelGGL((fe_grad_seg<J, 30, GRAD>), g, dim3(kBlock), 0, s, a, a.tab); break;
    case 32: hipLaunchKernelGGL((fe_grad_seg<J, 32, GRAD>), g, dim3(kBlock), 0, s, a, a.tab); break;
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

}  // namespace

hipError_t launch_fe_grad(const DevInstance &I, const BucketLaunch &bk, int B, int Bp,
                          const float *x, float *adj, float *part, float *fe, const float *dobj,
                          bool grad, hipStream_t s, const uint8_t *skip)
{
    if (bk.nc == 0 || B == 0) return hipSuccess;
    FeArgs a;
    a.x = x; a.adj = adj; a.part = part; a.fe = fe; a.dobj = dobj; a.skip = skip;
    a.bc_slot0 = I.bc_slot0; a.bc_k = I.bc_k; a.bc_tab = I.bc_tab; a.bc_orig = I.bc_orig;
    a.bc_w = I.bc_w; a.slot_lit = I.slot_lit; a.tab = I.tab; a.tab_rows = I.tab_rows;
    a.B = B; a.Bp = Bp;
    a.c0 = bk.c0; a.nc = bk.nc; a.tile = bk.tile; a.ntiles = bk.ntiles; a.tile0 = bk.tile0;
    // several restarts per lane for short constraints when B and the rows allow
    // 4*rpl-byte access (else one)
    int rpl = 1;
    if (bk.J == 1) {
        const int want = bk.rpl > 0 ? bk.rpl : (bk.S <= 8 ? 4 : 1);
        const uintptr_t al = (uintptr_t)(4 * want);
        if ((want == 2 || (want == 4 && bk.S <= 8)) && B % want == 0 &&
            reinterpret_cast<uintptr_t>(x) % al == 0 && (!dobj || reinterpret_cast<uintptr_t>(dobj) % al == 0))
            rpl = want;
    }
    const int R = bk.J == 1 ? kWave * rpl : kWave / bk.J;      // restarts per wave
    int64_t groups = (B + R - 1) / R;
    if (bk.J > 1) groups = (groups + kWavesPerBlock - 1) / kWavesPerBlock * kWavesPerBlock;
    a.items = groups * bk.ntiles;
    if (a.items > INT32_MAX) return hipErrorInvalidValue;
    hipError_t err = hipSuccess;
    const hipError_t e = for_launch_chunks(a.items, [&](int64_t first, int64_t count) {
        a.item0 = first;
        const dim3 g = grid_for_waves(count);
        hipError_t r;
        if (grad) r = bk.J == 1 ? dispatch_short<true>(bk.S, rpl, g, s, a) : dispatch_seg<true>(bk.J, bk.S, g, s, a);
        else r = bk.J == 1 ? dispatch_short<false>(bk.S, rpl, g, s, a) : dispatch_seg<false>(bk.J, bk.S, g, s, a);
        if (r != hipSuccess && err == hipSuccess) err = r;
    });
    return err != hipSuccess ? err : e;
}

}  // namespace afs
