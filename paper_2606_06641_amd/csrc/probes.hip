// probes.hip -- peak probes for the roofline denominators (gfx950).
//
// Three small kernels that measure what this build's code can reach on the
// device, reported beside the published peaks:
//   - plain FP32 FMA issue: independent v_fma_f32 chains (the library is built
//     without packed FP32 instructions, so this is the ceiling of its VALU code);
//   - dense BF16 MFMA: v_mfma_f32_16x16x32_bf16 with independent accumulators;
//   - HBM streaming: a 16-byte-per-lane copy with non-temporal loads and stores.
// Each kernel writes a value derived from all of its work so that nothing is
// optimised away.  The caller times the launch on `stream` (HIP events).

#include <hip/hip_runtime.h>

#include <cstdint>

#include "afsat.h"

namespace {

constexpr int kProbeBlock = 256;
constexpr int kChains = 16;            // independent FMA chains per lane

// V = 0: v_fma_f32 chains acc = acc * a + b (a, b uniform);
// V = 1: v_fmac_f32 chains acc += x * y with x, y per-lane registers;
// V = 2: v_mul_f32 chains acc *= x;
// V = 3: the product step of the FE kernels, (r, i) <- (r - i z, i + r z), two
//        dependent FMAs per step, kChains / 2 independent complex chains;
// V = 4: v_fma_f32 chains acc = acc * x + y with per-lane x, y (three-address
//        form, all operands in vector registers, no modifiers);
// V = 5: v_mul_f32 chains acc *= a with a uniform (a scalar-register operand);
// V = 6: v_fmac_f32 chains acc += a * x with a uniform, x per lane.
// Flops counted: 2 per FMA, 1 per multiply.
template <int V>
__global__ __launch_bounds__(kProbeBlock) void probe_fma_kernel(float *out, int iters, float a, float b)
{
    float acc[kChains];
#pragma unroll
    for (int j = 0; j < kChains; ++j) acc[j] = (float)(threadIdx.x + j) * 1e-3f;
    const float x = a + (float)(threadIdx.x & 1) * 1e-9f, y = b + (float)(threadIdx.x & 2) * 1e-9f;
#pragma unroll 2
    for (int i = 0; i < iters; ++i) {
        if constexpr (V == 3) {
#pragma unroll
            for (int j = 0; j < kChains; j += 2) {
                const float r = fmaf(-acc[j + 1], y, acc[j]);
                acc[j + 1] = fmaf(acc[j], y, acc[j + 1]);
                acc[j] = r;
            }
        } else {
#pragma unroll
            for (int j = 0; j < kChains; ++j) {
                if constexpr (V == 0) acc[j] = fmaf(acc[j], a, b);
                else if constexpr (V == 1) acc[j] = fmaf(x, y, acc[j]);
                else if constexpr (V == 4) acc[j] = fmaf(acc[j], x, y);
                else if constexpr (V == 5) acc[j] *= a;
                else if constexpr (V == 6) acc[j] = fmaf(a, x, acc[j]);
                else acc[j] *= x;
            }
        }
    }
    float s = 0.f;
#pragma unroll
    for (int j = 0; j < kChains; ++j) s += acc[j];
    out[(size_t)blockIdx.x * kProbeBlock + threadIdx.x] = s;
}

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
constexpr int kAcc = 8;                // independent MFMA accumulators per wave

__global__ __launch_bounds__(kProbeBlock) void probe_mfma_kernel(float *out, int iters)
{
    bf16x8 a, b;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        a[e] = (__bf16)(1e-3f * (float)((threadIdx.x + e) & 7));
        b[e] = (__bf16)(1e-3f * (float)((threadIdx.x * 3 + e) & 7));
    }
    f32x4 acc[kAcc];
#pragma unroll
    for (int t = 0; t < kAcc; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int t = 0; t < kAcc; ++t) acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[t], 0, 0, 0);
    }
    float s = 0.f;
#pragma unroll
    for (int t = 0; t < kAcc; ++t) s += acc[t][0] + acc[t][1] + acc[t][2] + acc[t][3];
    out[(size_t)blockIdx.x * kProbeBlock + threadIdx.x] = s;
}

__global__ __launch_bounds__(kProbeBlock) void probe_copy_kernel(const f32x4 *__restrict__ src, f32x4 *__restrict__ dst,
                                                                 int64_t n4)
{
    const int64_t stride = (int64_t)gridDim.x * kProbeBlock;
    for (int64_t i = (int64_t)blockIdx.x * kProbeBlock + threadIdx.x; i < n4; i += stride) {
        const f32x4 v = __builtin_nontemporal_load(src + i);
        __builtin_nontemporal_store(v, dst + i);
    }
}

}  // namespace

extern "C" {

afs_status afs_probe_fma(int32_t variant, int32_t blocks, int32_t iters, float *out, double *flops, void *stream)
{
    if (blocks <= 0 || iters <= 0 || !out || variant < 0 || variant > 6) return AFS_EINVAL;
    const dim3 g(blocks), t(kProbeBlock);
    hipStream_t s = (hipStream_t)stream;
    switch (variant) {
    case 0: hipLaunchKernelGGL(probe_fma_kernel<0>, g, t, 0, s, out, iters, 0.999999f, 1e-7f); break;
    case 1: hipLaunchKernelGGL(probe_fma_kernel<1>, g, t, 0, s, out, iters, 1e-4f, 1e-4f); break;
    case 2: hipLaunchKernelGGL(probe_fma_kernel<2>, g, t, 0, s, out, iters, 0.9999999f, 0.f); break;
    case 3: hipLaunchKernelGGL(probe_fma_kernel<3>, g, t, 0, s, out, iters, 0.f, 1e-4f); break;
    case 4: hipLaunchKernelGGL(probe_fma_kernel<4>, g, t, 0, s, out, iters, 0.999999f, 1e-7f); break;
    case 5: hipLaunchKernelGGL(probe_fma_kernel<5>, g, t, 0, s, out, iters, 0.9999999f, 0.f); break;
    default: hipLaunchKernelGGL(probe_fma_kernel<6>, g, t, 0, s, out, iters, 1e-4f, 1e-4f); break;
    }
    if (hipGetLastError() != hipSuccess) return AFS_EDEVICE;
    const double per = (variant == 2 || variant == 5) ? 1.0 : 2.0;        // flops per operation
    if (flops) *flops = per * kChains * (double)iters * (double)blocks * kProbeBlock;
    return AFS_OK;
}

afs_status afs_probe_mfma_bf16(int32_t blocks, int32_t iters, float *out, double *flops, void *stream)
{
    if (blocks <= 0 || iters <= 0 || !out) return AFS_EINVAL;
    hipLaunchKernelGGL(probe_mfma_kernel, dim3(blocks), dim3(kProbeBlock), 0, (hipStream_t)stream, out, iters);
    if (hipGetLastError() != hipSuccess) return AFS_EDEVICE;
    // one 16x16x32 product per instruction: 2 * 16 * 16 * 32 flops, per wave
    if (flops) *flops = 2.0 * 16 * 16 * 32 * kAcc * (double)iters * (double)blocks * (kProbeBlock / 64);
    return AFS_OK;
}

afs_status afs_probe_copy(const void *src, void *dst, int64_t bytes, int32_t blocks, void *stream)
{
    if (!src || !dst || bytes <= 0 || bytes % 16 || blocks <= 0) return AFS_EINVAL;
    if (reinterpret_cast<uintptr_t>(src) % 16 || reinterpret_cast<uintptr_t>(dst) % 16) return AFS_EINVAL;
    hipLaunchKernelGGL(probe_copy_kernel, dim3(blocks), dim3(kProbeBlock), 0, (hipStream_t)stream,
                       static_cast<const f32x4 *>(src), static_cast<f32x4 *>(dst), bytes / 16);
    return hipGetLastError() == hipSuccess ? AFS_OK : AFS_EDEVICE;
}

}  // extern "C"
