// update_kernels.hip -- gradient gather, projected step, rounding, exact
// verification and bookkeeping kernels for gfx950 (CDNA4, wave64).
//
// Layouts: x [n][B] f32 (restart contiguous); adj [L][Bp] f32 in slot order with
// Bp = B rounded up to 64; bits [n][ceil(B/32)] u32.

#include "kernels.hpp"

#include <algorithm>

#include "afsat.h"
#include "device_common.hpp"

namespace afs {

namespace {

using namespace dev;

// ---------------------------------------------------------------------------
// Gradient: segmented sum of the per-literal adjoints through the variable ->
// slot transpose.  One wave per (variable, 256 restarts), four consecutive
// restarts per lane: the slot list is wave-uniform and every adjoint row read
// is a coalesced 1 KiB row of 16-byte loads.  Each restart sums its slots in
// ascending order, so the result does not depend on the launch shape.
// ---------------------------------------------------------------------------
constexpr int kRestartsPerLane = 4;
constexpr int kScatterChunk = kWave * kRestartsPerLane;

struct ScatterArgs {
    const float *adj;
    float *grad, *x;
    const int32_t *voff, *vslot, *var_inst;
    int n_inst;
    const uint8_t *fixed, *done;  // fixed [n_partial][n]
    int n, n_partial;
    uint32_t *bits;
    int32_t *unsat;
    uint8_t *moved;              // [n_inst][B]: set where some variable moves by >= eps (NULL: not tracked)
    float *vel;                  // [n][B] heavy-ball velocity (NULL: plain step)
    float lr, eps, mu;
    int B, Bp, W, nchunks;
    int64_t items, item0;        // all items; first item of this launch
};

__device__ __forceinline__ void add4(float4 &g, const float4 a)
{
    g.x += a.x;
    g.y += a.y;
    g.z += a.z;
    g.w += a.w;
}

// adjoint rows are read once: non-temporal loads keep them from evicting x
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float4 load_stream(const float *p)
{
    const f32x4 v = __builtin_nontemporal_load(reinterpret_cast<const f32x4 *>(p));
    return make_float4(v.x, v.y, v.z, v.w);
}

// restarts b0..b0+3 of variable v (zero where b0 >= Bp)
__device__ __forceinline__ float4 gather_sum4(const ScatterArgs &A, int v, int b0)
{
    float4 g = make_float4(0.f, 0.f, 0.f, 0.f);
    if (b0 >= A.Bp) return g;
    const int o0 = A.voff[v], o1 = A.voff[v + 1];
    const float *col = A.adj + b0;
    int o = o0;
    for (; o + 4 <= o1; o += 4) {
        const float4 a0 = load_stream(col + (int64_t)A.vslot[o] * A.Bp);
        const float4 a1 = load_stream(col + (int64_t)A.vslot[o + 1] * A.Bp);
        const float4 a2 = load_stream(col + (int64_t)A.vslot[o + 2] * A.Bp);
        const float4 a3 = load_stream(col + (int64_t)A.vslot[o + 3] * A.Bp);
        add4(g, a0);
        add4(g, a1);
        add4(g, a2);
        add4(g, a3);
    }
    for (; o < o1; ++o) add4(g, load_stream(col + (int64_t)A.vslot[o] * A.Bp));
    return g;
}

__device__ __forceinline__ float elem(const float4 &g, int e)
{
    return e == 0 ? g.x : e == 1 ? g.y : e == 2 ? g.z : g.w;
}

// Projected step of Algorithm 1: x - lr*g clipped to [-1, 1] (NaN stays NaN).
__device__ __forceinline__ float project_step(float xv, float g, float lr)
{
    float t = xv - lr * g;
    t = t > 1.0f ? 1.0f : t;
    t = t < -1.0f ? -1.0f : t;
    return t;
}

// 64 restarts per wave, one per lane: word pair of the chunk from a ballot
__device__ __forceinline__ void store_bits(uint32_t *bits, int v, int W, int chunk, bool neg)
{
    const unsigned long long m = __ballot(neg);
    if ((threadIdx.x & 63) == 0) {
        const int w0 = chunk * 2;
        if (w0 < W) bits[(int64_t)v * W + w0] = (uint32_t)m;
        if (w0 + 1 < W) bits[(int64_t)v * W + w0 + 1] = (uint32_t)(m >> 32);
    }
}

template <int CTRL>
__device__ __forceinline__ uint32_t dpp_mov_u(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, CTRL, 0xF, 0xF, false);
}

// Four restarts per lane (a nibble): the eight lanes 8q..8q+7 form one 32-bit
// word, gathered by row shifts inside the 16-lane row; lane 8q ends up with it.
__device__ __forceinline__ uint32_t gather_nibbles(uint32_t nib)
{
    uint32_t t = nib | (dpp_mov_u<0x101>(nib) << 4);      // row_shl:1
    t |= dpp_mov_u<0x102>(t) << 8;                        // row_shl:2
    t |= dpp_mov_u<0x104>(t) << 16;                       // row_shl:4
    return t;
}

// 256 restarts per wave; lane 8q stores word q of the chunk.
__device__ __forceinline__ void store_bits4(uint32_t *bits, int v, int W, int chunk, uint32_t nib)
{
    const uint32_t t = gather_nibbles(nib);
    const int lane = threadIdx.x & 63;
    const int w = chunk * (kScatterChunk / 32) + (lane >> 3);
    if ((lane & 7) == 0 && w < W) bits[(int64_t)v * W + w] = t;
}

__global__ __launch_bounds__(kBlock) void scatter_grad_kernel(ScatterArgs A)
{
    const int64_t item = A.item0 + (int64_t)blockIdx.x * kWavesPerBlock + wave_id();
    if (item >= A.items) return;
    const int v = (int)(item / A.nchunks), chunk = (int)(item % A.nchunks);
    const int b0 = chunk * kScatterChunk + (threadIdx.x & 63) * kRestartsPerLane;
    const float4 g = gather_sum4(A, v, b0);
#pragma unroll
    for (int e = 0; e < kRestartsPerLane; ++e)
        if (b0 + e < A.B) A.grad[(int64_t)v * A.B + b0 + e] = elem(g, e);
}

__global__ __launch_bounds__(kBlock) void scatter_step_kernel(ScatterArgs A)
{
    const int64_t item = A.item0 + (int64_t)blockIdx.x * kWavesPerBlock + wave_id();
    if (item >= A.items) return;
    const int v = (int)(item / A.nchunks), chunk = (int)(item % A.nchunks);
    const int b0 = chunk * kScatterChunk + (threadIdx.x & 63) * kRestartsPerLane;
    const float4 g = gather_sum4(A, v, b0);
    const uint8_t *done = A.done ? A.done + (int64_t)A.var_inst[v] * A.B : nullptr;
    uint32_t nib = 0;
#pragma unroll
    for (int e = 0; e < kRestartsPerLane; ++e) {
        const int b = b0 + e;
        if (b < A.B) {
            const int64_t at = (int64_t)v * A.B + b;
            float xv = A.x[at];
            if (!is_fixed(A.fixed, A.n_partial, A.n, A.B, v, b) && !(done && done[b])) {
                const float x0 = xv;
                float d = elem(g, e);
                if (A.vel) {                            // v = mu v + g, and the step follows v
                    d = fmaf(A.mu, A.vel[at], d);
                    A.vel[at] = d;
                }
                xv = project_step(xv, d, A.lr);
                A.x[at] = xv;
                // several variables may store 1 into one flag: every store writes the same value
                if (A.moved && fabsf(xv - x0) >= A.eps) A.moved[(int64_t)A.var_inst[v] * A.B + b] = 1;
            }
            if (v < A.n_inst) A.unsat[(int64_t)v * A.B + b] = 0;
            nib |= (xv < 0.0f ? 1u : 0u) << e;
        }
    }
    store_bits4(A.bits, v, A.W, chunk, nib);
}

// ---------------------------------------------------------------------------
// Elementwise step, rounding.
// ---------------------------------------------------------------------------
struct EltArgs {
    float *x;
    const float *xin, *grad;
    const int32_t *var_inst;
    int n_inst;
    const uint8_t *fixed, *done;  // fixed [n_partial][n]
    int n, n_partial;
    uint32_t *bits;
    int32_t *unsat;
    float lr;
    int B, W, nchunks;
    int64_t items, item0;        // all items; first item of this launch
};

__global__ __launch_bounds__(kBlock) void step_kernel(EltArgs A)
{
    const int64_t item = A.item0 + (int64_t)blockIdx.x * kWavesPerBlock + wave_id();
    if (item >= A.items) return;
    const int v = (int)(item / A.nchunks), chunk = (int)(item % A.nchunks);
    const int b = chunk * kWave + (threadIdx.x & 63);
    if (b >= A.B) return;
    if (is_fixed(A.fixed, A.n_partial, A.n, A.B, v, b) || (A.done && A.done[(int64_t)A.var_inst[v] * A.B + b]))
        return;
    const int64_t at = (int64_t)v * A.B + b;
    A.x[at] = project_step(A.x[at], A.grad[at], A.lr);
}

__global__ __launch_bounds__(kBlock) void round_kernel(EltArgs A)
{
    const int64_t item = A.item0 + (int64_t)blockIdx.x * kWavesPerBlock + wave_id();
    if (item >= A.items) return;
    const int v = (int)(item / A.nchunks), chunk = (int)(item % A.nchunks);
    const int b = chunk * kWave + (threadIdx.x & 63);
    const bool valid = b < A.B;
    const float xv = valid ? A.xin[(int64_t)v * A.B + b] : 0.f;
    if (valid && v < A.n_inst) A.unsat[(int64_t)v * A.B + b] = 0;
    store_bits(A.bits, v, A.W, chunk, valid && xv < 0.0f);
}

// ---------------------------------------------------------------------------
// Exact verification in two passes over the rounded assignments bits [n][W]
// (bit b%32 of word b/32 set when x[v][b] < 0, i.e. variable v True in restart b).
// Pass one stores a 32-restart violation mask per (constraint, word) in
// viol [W][Cp] (Cp = C rounded up to 4); pass two sums each restart's bits.
//
// violation_kernel (every type but the counted ones): one lane per (constraint,
// word), lanes of a wave on consecutive words so that each literal's load is a
// coalesced row.  Bitwise over the 32 restarts the lane keeps any (t >= 1),
// all (t == k), two (t >= 2) and the parity of t, which decide OR, XOR, NAE,
// AMO and EO.
//
// violation_count_kernel (CARD >= K, CARD < K, EK): the same lane mapping over
// the list of counted constraints.  A lane counts the true literals of its 32
// restarts bit-sliced: plane j holds bit j of the 32 counts, and each literal's
// word is added with a carry through the planes (k <= 1024, so 11 planes); the
// counts are then compared with K plane by plane from the top.
//
// Both read the literals of a constraint in batches of 16 so that every load of
// a batch is in flight at once; the literal array carries kLitPad trailing
// zeros, so a batch never reads past it.
//
// count_kernel: one lane per restart and a tile of constraints; sums the
// restart's violation bits and adds them to unsat of the constraint's
// sub-instance (integer atomics, so the order does not matter).
// ---------------------------------------------------------------------------
constexpr int kLitBatch = 16;

__device__ __forceinline__ bool counted_type(int type)
{
    return type == AFS_CARD_GE || type == AFS_CARD_LT || type == AFS_EK;
}

struct ViolArgs {
    const uint32_t *bits;
    uint32_t *viol;
    const int32_t *con_off, *lits, *types, *params, *counted;
    int B, W, C, Cp, wpw, cpw, wchunks, n_counted;
    int64_t items, item0;        // all items; first item of this launch
};

__global__ __launch_bounds__(kBlock) void violation_kernel(ViolArgs A)
{
    const int64_t item = A.item0 + (int64_t)blockIdx.x * kWavesPerBlock + wave_id();
    if (item >= A.items) return;
    const int lane = threadIdx.x & 63;
    const int cl = lane / A.wpw, wl = lane % A.wpw;
    const int64_t c = (item / A.wchunks) * A.cpw + cl;
    const int w = (int)(item % A.wchunks) * kWave + wl;
    if (cl >= A.cpw || c >= A.C || w >= A.W) return;
    const int type = A.types[c];
    if (counted_type(type)) return;                  // violation_count_kernel's
    const int o0 = A.con_off[c], o1 = A.con_off[c + 1];
    uint32_t any = 0u, all = ~0u, two = 0u, par = 0u;
    for (int o = o0; o < o1; o += kLitBatch) {
        int l[kLitBatch];
        uint32_t tv[kLitBatch];
#pragma unroll
        for (int i = 0; i < kLitBatch; ++i) l[i] = A.lits[o + i];     // padded: past o1 stays in bounds
#pragma unroll
        for (int i = 0; i < kLitBatch; ++i) {
            const int v = (l[i] > 0 ? l[i] : -l[i]) - 1;
            tv[i] = A.bits[(int64_t)(v > 0 ? v : 0) * A.W + w];             // 1: variable True
        }
#pragma unroll
        for (int i = 0; i < kLitBatch; ++i) {
            const bool in = o + i < o1;
            const uint32_t lt = in ? (l[i] > 0 ? tv[i] : ~tv[i]) : 0u;       // 1: literal True
            two |= any & lt;
            any |= lt;
            all &= in ? lt : ~0u;
            par ^= lt;
        }
    }
    uint32_t viol;
    switch (type) {
    case AFS_OR: viol = ~any; break;
    case AFS_XOR: viol = par ^ ((A.params[c] & 1) ? ~0u : 0u); break;
    case AFS_NAE: viol = ~any | all; break;
    case AFS_AMO: viol = two; break;
    default: viol = ~any | two; break;               // AFS_EO
    }
    A.viol[(int64_t)w * A.Cp + c] = viol;
}

constexpr int kPlanes = 11;                          // counts up to 2047 >= AFS_MAX_LEN
static_assert((1 << kPlanes) > AFS_MAX_LEN, "bit planes too few for the longest constraint");

__global__ __launch_bounds__(kBlock) void violation_count_kernel(ViolArgs A)
{
    const int64_t item = A.item0 + (int64_t)blockIdx.x * kWavesPerBlock + wave_id();
    if (item >= A.items) return;
    const int lane = threadIdx.x & 63;
    const int cl = lane / A.wpw, wl = lane % A.wpw;
    const int64_t ci = (item / A.wchunks) * A.cpw + cl;       // index into the counted list
    const int w = (int)(item % A.wchunks) * kWave + wl;
    if (cl >= A.cpw || ci >= A.n_counted || w >= A.W) return;
    const int c = A.counted[ci];
    const int o0 = A.con_off[c], o1 = A.con_off[c + 1];
    uint32_t plane[kPlanes];
#pragma unroll
    for (int j = 0; j < kPlanes; ++j) plane[j] = 0u;
    for (int o = o0; o < o1; o += kLitBatch) {
        int l[kLitBatch];
        uint32_t tv[kLitBatch];
#pragma unroll
        for (int i = 0; i < kLitBatch; ++i) l[i] = A.lits[o + i];     // padded: past o1 stays in bounds
#pragma unroll
        for (int i = 0; i < kLitBatch; ++i) {
            const int v = (l[i] > 0 ? l[i] : -l[i]) - 1;
            tv[i] = A.bits[(int64_t)(v > 0 ? v : 0) * A.W + w];             // 1: variable True
        }
#pragma unroll
        for (int i = 0; i < kLitBatch; ++i) {
            uint32_t carry = o + i < o1 ? (l[i] > 0 ? tv[i] : ~tv[i]) : 0u;  // 1: literal True
#pragma unroll
            for (int j = 0; j < kPlanes; ++j) {
                const uint32_t t = plane[j] & carry;
                plane[j] ^= carry;
                carry = t;
            }
        }
    }
    const int type = A.types[c], K = A.params[c], k = o1 - o0;
    uint32_t viol;
    if (K <= 0 || K > k) {
        // constant predicates: t >= K holds for every t when K <= 0 and for none when
        // K > k; t == K for none unless K == 0
        const bool ge_all = K <= 0;
        if (type == AFS_EK && K == 0) {
            uint32_t any = 0u;
#pragma unroll
            for (int j = 0; j < kPlanes; ++j) any |= plane[j];
            viol = any;                                  // violated where t != 0
        } else if (type == AFS_EK) {
            viol = ~0u;
        } else {
            const bool sat = type == AFS_CARD_GE ? ge_all : !ge_all;
            viol = sat ? 0u : ~0u;
        }
    } else {
        // 1 <= K <= k < 2^kPlanes: compare the counts with K from the top plane down
        uint32_t eq = ~0u, gt = 0u;
#pragma unroll
        for (int j = kPlanes - 1; j >= 0; --j) {
            const uint32_t kb = ((K >> j) & 1) ? ~0u : 0u;
            gt |= eq & plane[j] & ~kb;
            eq &= ~(plane[j] ^ kb);
        }
        const uint32_t ge = gt | eq;
        viol = type == AFS_CARD_GE ? ~ge : type == AFS_CARD_LT ? ge : ~eq;
    }
    A.viol[(int64_t)w * A.Cp + c] = viol;
}

struct CountArgs {
    const uint32_t *viol;
    int32_t *unsat;
    const int32_t *con_inst;
    int n_inst, B, W, C, Cp, tile, tblocks;
};

__device__ __forceinline__ void add_unsat(const CountArgs &A, int inst, int b, bool valid, int cnt)
{
    if (valid && cnt) atomicAdd(&A.unsat[(int64_t)inst * A.B + b], cnt);
}

__device__ __forceinline__ int bit_at(uint32_t v, int sh, bool in)
{
    return in ? (int)((v >> sh) & 1u) : 0;
}

// viol is [W][Cp] (Cp = C rounded up to 4): four constraints per 16-byte load,
// shared by the 32 lanes of one word.  A block of kCountWaves waves takes one
// group of 64 restarts and kCountWaves consecutive tiles (tiles start at
// multiples of 16); when its constraints lie in one sub-instance the waves'
// counts are summed in LDS and added with one atomic per restart.
constexpr int kCountWaves = 16;

__device__ __forceinline__ int count_tile(const uint32_t *row, int cbeg, int cend, int sh)
{
    int cnt = 0;
    for (int c = cbeg; c < cend; c += 16) {
        uint4 q[4];
#pragma unroll
        for (int i = 0; i < 4; ++i)
            q[i] = c + 4 * i < cend ? *reinterpret_cast<const uint4 *>(row + c + 4 * i) : make_uint4(0, 0, 0, 0);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int c4 = c + 4 * i;
            cnt += bit_at(q[i].x, sh, c4 < cend) + bit_at(q[i].y, sh, c4 + 1 < cend) +
                   bit_at(q[i].z, sh, c4 + 2 < cend) + bit_at(q[i].w, sh, c4 + 3 < cend);
        }
    }
    return cnt;
}

__global__ __launch_bounds__(kCountWaves * kWave) void count_kernel(CountArgs A)
{
    __shared__ int red[kCountWaves][kWave];
    const int64_t blk = xcd_block();
    const int group = (int)(blk / A.tblocks), tb = (int)(blk % A.tblocks);
    const int wv = wave_id(), lane = threadIdx.x & 63;
    const int b = group * kWave + lane;
    const bool valid = b < A.B;
    const int wi = (valid ? b : A.B - 1) >> 5;
    const int sh = b & 31;
    const int bbeg = tb * kCountWaves * A.tile, bend = min(bbeg + kCountWaves * A.tile, A.C);
    const int cbeg = min(bbeg + wv * A.tile, A.C), cend = min(cbeg + A.tile, A.C);
    const uint32_t *row = A.viol + (int64_t)wi * A.Cp;
    const int first = A.n_inst == 1 ? 0 : A.con_inst[bbeg];
    if (A.n_inst == 1 || A.con_inst[bend - 1] == first) {     // block-uniform
        red[wv][lane] = count_tile(row, cbeg, cend, sh);
        __syncthreads();
        if (wv == 0) {
            int cnt = 0;
#pragma unroll
            for (int i = 0; i < kCountWaves; ++i) cnt += red[i][lane];
            add_unsat(A, first, b, valid, cnt);
        }
        return;
    }
    // The tile spans sub-instances: the constraints of one sub-instance are
    // contiguous (con_inst is non-decreasing), so each run's end is found by a
    // binary search and the run counted like a whole tile.
    for (int c = cbeg; c < cend;) {
        const int inst = A.con_inst[c];
        int lo = c + 1, hi = cend;               // first index in (c, cend] of another sub-instance
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (A.con_inst[mid] == inst) lo = mid + 1;
            else hi = mid;
        }
        int cnt = 0, h = c;
        for (; h < lo && (h & 3); ++h) cnt += (int)((row[h] >> sh) & 1u);   // up to a 16-byte boundary
        if (h < lo) cnt += count_tile(row, h, lo, sh);
        add_unsat(A, inst, b, valid, cnt);
        c = lo;
    }
}

// One block: done / first_sat bookkeeping and the {t, number done} counter.
// done: 0 searching, 1 verified, 2 converged (the step length fell below delta,
// Algorithm 1's eta < delta); both freeze the restart.  counter = {t, verified,
// frozen, 0}.  The step length of pair i is eta[i % B] (a line search on a
// plain instance) or eta_const (constant step); delta <= 0 turns the test off.
__global__ __launch_bounds__(1024) void finalize_kernel(int count, int B, const int32_t *unsat, uint8_t *done,
                                                        int32_t *first_sat, int32_t *counter, int mode,
                                                        const float *eta, float eta_const, float delta,
                                                        uint8_t *moved, float eps)
{
    __shared__ int red[2][1024 / kWave];
    const int t = (mode == FIN_STEP) ? counter[0] + 1 : 0;
    __syncthreads();
    int nsat = 0, nfrozen = 0;
    for (int b = threadIdx.x; b < count; b += blockDim.x) {
        const bool ok = unsat[b] == 0;
        if (mode == FIN_INIT) {
            done[b] = ok ? 1 : 0;
            first_sat[b] = ok ? 0 : -1;
            if (moved) moved[b] = 0;
            nsat += ok;
            nfrozen += ok;
        } else if (mode == FIN_STEP) {
            uint8_t d = done[b];
            if (!d && ok) {
                done[b] = d = 1;
                first_sat[b] = t;
            }
            if (!d && delta > 0.0f && (eta ? eta[b % B] : eta_const) < delta) done[b] = d = 2;
            if (moved) {
                // within eps of the previous point in every variable; cleared for the next step
                if (!d && eps > 0.0f && !moved[b]) done[b] = d = 2;
                moved[b] = 0;
            }
            nsat += d == 1;
            nfrozen += d != 0;
        } else {
            if (ok) done[b] = 1;
        }
    }
    if (mode == FIN_VERIFY) return;
    for (int off = 32; off > 0; off >>= 1) {
        nsat += __shfl_down(nsat, off);
        nfrozen += __shfl_down(nfrozen, off);
    }
    if ((threadIdx.x & 63) == 0) {
        red[0][threadIdx.x >> 6] = nsat;
        red[1][threadIdx.x >> 6] = nfrozen;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int s0 = 0, s1 = 0;
        for (int i = 0; i < (int)(blockDim.x / kWave); ++i) {
            s0 += red[0][i];
            s1 += red[1][i];
        }
        counter[0] = t;
        counter[1] = s0;
        counter[2] = s1;
        counter[3] = 0;
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

// one block of kRed2Waves waves per 64 restarts: wave w sums the groups
// w, w + kRed2Waves, ... in ascending order, then lane b of wave 0 adds the
// waves' sums in wave order (a fixed order, whatever the launch)
constexpr int kRed2Waves = 16;

__global__ __launch_bounds__(kRed2Waves * kWave) void obj_reduce2(int groups, int B, int Bp, const float *part2,
                                                                 float *obj)
{
    __shared__ float red[kRed2Waves][kWave];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int b = blockIdx.x * kWave + lane;           // < Bp
    float s = 0.f;
    for (int g = w; g < groups; g += kRed2Waves) s += part2[(int64_t)g * Bp + b];
    red[w][lane] = s;
    __syncthreads();
    if (w == 0 && b < B) {
        float t = red[0][lane];
        for (int i = 1; i < kRed2Waves; ++i) t += red[i][lane];
        obj[b] = t;
    }
}

__global__ __launch_bounds__(kBlock) void permute_adj_kernel(const float *adj, float *out,
                                                             const int32_t *slot_to_lit, int B, int Bp,
                                                             int nchunks, int64_t items, int64_t item0)
{
    const int64_t item = item0 + (int64_t)blockIdx.x * kWavesPerBlock + wave_id();
    if (item >= items) return;
    const int64_t s = item / nchunks;
    const int chunk = (int)(item % nchunks);
    const int b = chunk * kWave + (threadIdx.x & 63);
    if (b < B) out[(int64_t)slot_to_lit[s] * B + b] = adj[s * Bp + b];
}

}  // namespace

static ScatterArgs scatter_args(const DevInstance &I, int B, int Bp, const float *adj)
{
    ScatterArgs a{};
    a.adj = adj;
    a.voff = I.voff; a.vslot = I.vslot; a.var_inst = I.var_inst; a.n_inst = I.n_inst;
    a.B = B; a.Bp = Bp; a.W = (B + 31) / 32;
    a.nchunks = (B + kScatterChunk - 1) / kScatterChunk;
    a.items = (int64_t)I.n * a.nchunks;
    return a;
}

hipError_t launch_scatter(const DevInstance &I, int B, int Bp, const float *adj, float *grad,
                          hipStream_t s)
{
    if (B == 0) return hipSuccess;
    ScatterArgs a = scatter_args(I, B, Bp, adj);
    a.grad = grad;
    return for_launch_chunks(a.items, [&](int64_t first, int64_t count) {
        a.item0 = first;
        hipLaunchKernelGGL(scatter_grad_kernel, grid_for_waves(count), dim3(kBlock), 0, s, a);
    });
}

hipError_t launch_scatter_step(const DevInstance &I, int B, int Bp, const float *adj, float *x,
                               float lr, const uint8_t *fixed, int n_partial, const uint8_t *done,
                               uint32_t *bits, int32_t *unsat, hipStream_t s, uint8_t *moved, float eps,
                               float *vel, float mu)
{
    if (B == 0) return hipSuccess;
    ScatterArgs a = scatter_args(I, B, Bp, adj);
    a.x = x; a.lr = lr; a.fixed = fixed; a.done = done; a.bits = bits; a.unsat = unsat;
    a.moved = moved; a.eps = eps; a.vel = vel; a.mu = mu;
    a.n = I.n; a.n_partial = n_partial;
    return for_launch_chunks(a.items, [&](int64_t first, int64_t count) {
        a.item0 = first;
        hipLaunchKernelGGL(scatter_step_kernel, grid_for_waves(count), dim3(kBlock), 0, s, a);
    });
}

hipError_t launch_obj_reduce(int tiles, int B, int Bp, const float *part, float *part2,
                             float *obj, hipStream_t s)
{
    if (B == 0) return hipSuccess;
    const int groups = (tiles + kRedGroup - 1) / kRedGroup;
    if (groups > 0)
        hipLaunchKernelGGL(obj_reduce1, dim3(Bp / kWave, groups), dim3(kWave), 0, s, tiles, Bp, part, part2);
    hipLaunchKernelGGL(obj_reduce2, dim3(Bp / kWave), dim3(kRed2Waves * kWave), 0, s, groups, B, Bp, part2, obj);
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
                       const uint8_t *fixed, int n_partial, const uint8_t *done, hipStream_t s)
{
    if (B == 0) return hipSuccess;
    EltArgs a = elt_args(I.n, B);
    a.x = x; a.grad = grad; a.lr = lr; a.fixed = fixed; a.done = done;
    a.n = I.n; a.n_partial = n_partial;
    a.var_inst = I.var_inst; a.n_inst = I.n_inst;
    return for_launch_chunks(a.items, [&](int64_t first, int64_t count) {
        a.item0 = first;
        hipLaunchKernelGGL(step_kernel, grid_for_waves(count), dim3(kBlock), 0, s, a);
    });
}

hipError_t launch_round(const DevInstance &I, int B, const float *x, uint32_t *bits, int32_t *unsat,
                        hipStream_t s)
{
    if (B == 0) return hipSuccess;
    EltArgs a = elt_args(I.n, B);
    a.xin = x; a.bits = bits; a.unsat = unsat;
    a.var_inst = I.var_inst; a.n_inst = I.n_inst;
    return for_launch_chunks(a.items, [&](int64_t first, int64_t count) {
        a.item0 = first;
        hipLaunchKernelGGL(round_kernel, grid_for_waves(count), dim3(kBlock), 0, s, a);
    });
}

hipError_t launch_verify(const DevInstance &I, int B, const uint32_t *bits, uint32_t *viol,
                         int32_t *unsat, hipStream_t s)
{
    if (B == 0 || I.C == 0) return hipSuccess;
    ViolArgs v{};
    v.bits = bits; v.viol = viol;
    v.con_off = I.con_off; v.lits = I.lits; v.types = I.types; v.params = I.params;
    v.counted = I.counted;
    v.B = B; v.W = (B + 31) / 32; v.C = I.C; v.Cp = (I.C + 3) / 4 * 4;
    v.wpw = v.W < kWave ? v.W : kWave;
    v.cpw = kWave / v.wpw;
    v.wchunks = (v.W + kWave - 1) / kWave;
    v.items = (int64_t)((I.C + v.cpw - 1) / v.cpw) * v.wchunks;
    hipError_t e = for_launch_chunks(v.items, [&](int64_t first, int64_t count) {
        v.item0 = first;
        hipLaunchKernelGGL(violation_kernel, grid_for_waves(count), dim3(kBlock), 0, s, v);
    });
    if (e != hipSuccess) return e;
    if (I.n_counted > 0) {
        v.n_counted = I.n_counted;
        v.items = (int64_t)((I.n_counted + v.cpw - 1) / v.cpw) * v.wchunks;
        e = for_launch_chunks(v.items, [&](int64_t first, int64_t count) {
            v.item0 = first;
            hipLaunchKernelGGL(violation_count_kernel, grid_for_waves(count), dim3(kBlock), 0, s, v);
        });
        if (e != hipSuccess) return e;
    }
    CountArgs a{};
    a.viol = viol; a.unsat = unsat; a.con_inst = I.con_inst; a.n_inst = I.n_inst;
    a.B = B; a.W = v.W; a.C = I.C; a.Cp = v.Cp;
    const int groups = (B + kWave - 1) / kWave;
    const int want = (8192 + groups - 1) / groups;             // tiles for about 8k waves
    a.tile = std::max(64, ((I.C + want - 1) / want + 15) / 16 * 16);
    const int ntiles = (I.C + a.tile - 1) / a.tile;
    a.tblocks = (ntiles + kCountWaves - 1) / kCountWaves;
    hipLaunchKernelGGL(count_kernel, dim3((unsigned)((int64_t)groups * a.tblocks)), dim3(kCountWaves * kWave), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_finalize(int count, int B, const int32_t *unsat, uint8_t *done, int32_t *first_sat,
                           int32_t *counter, int mode, hipStream_t s, const float *eta, float eta_const,
                           float delta, uint8_t *moved, float eps)
{
    if (count == 0) return hipSuccess;
    hipLaunchKernelGGL(finalize_kernel, dim3(1), dim3(1024), 0, s, count, B, unsat, done, first_sat, counter, mode,
                       eta, eta_const, delta, moved, eps);
    return hipGetLastError();
}

hipError_t launch_permute_adj(const DevInstance &I, int B, int Bp, const float *adj,
                              float *adj_out, hipStream_t s)
{
    if (B == 0 || I.L == 0) return hipSuccess;
    const int nchunks = Bp / kWave;
    const int64_t items = I.L * nchunks;
    return for_launch_chunks(items, [&](int64_t first, int64_t count) {
        hipLaunchKernelGGL(permute_adj_kernel, grid_for_waves(count), dim3(kBlock), 0, s, adj, adj_out,
                           I.slot_to_lit, B, Bp, nchunks, items, first);
    });
}

}  // namespace afs
