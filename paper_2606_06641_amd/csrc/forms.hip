// forms.hip -- plain evaluation of FE(y) = Re sum_m d_m prod_i (alpha_m + beta_m y_i)
// in FP32 or FP64, for the precision study of the two DFT forms (the tables come
// from forms.cpp).  One lane per point, roots and literals in sequence, no
// rescaling: the arithmetic the form implies and nothing else.

#include "kernels.hpp"

#include "device_common.hpp"

namespace afs {

namespace {

using namespace dev;

// tab [N][6]: alpha (re, im), beta (re, im), d (re, im); y [k][B]
template <class T>
__global__ __launch_bounds__(kBlock) void fe_generic_kernel(int k, const double *tab, int B, const double *y,
                                                            double *fe)
{
    const int b = blockIdx.x * kBlock + threadIdx.x;
    if (b >= B) return;
    const int N = k + 1;
    T sum = 0;
    for (int m = 0; m < N; ++m) {
        const T ar = (T)tab[6 * m], ai = (T)tab[6 * m + 1];
        const T br = (T)tab[6 * m + 2], bi = (T)tab[6 * m + 3];
        T pr = 1, pi = 0;
        for (int i = 0; i < k; ++i) {
            const T yi = (T)y[(int64_t)i * B + b];
            const T fr = ar + br * yi, fi = ai + bi * yi;
            const T r = pr * fr - pi * fi;
            pi = pr * fi + pi * fr;
            pr = r;
        }
        sum += (T)tab[6 * m + 4] * pr - (T)tab[6 * m + 5] * pi;
    }
    fe[b] = (double)sum;
}

}  // namespace

hipError_t launch_fe_generic(int k, const double *tab, bool fp64, int B, const double *y, double *fe, hipStream_t s)
{
    if (B == 0) return hipSuccess;
    const dim3 grid((B + kBlock - 1) / kBlock);
    if (fp64)
        hipLaunchKernelGGL(fe_generic_kernel<double>, grid, dim3(kBlock), 0, s, k, tab, B, y, fe);
    else
        hipLaunchKernelGGL(fe_generic_kernel<float>, grid, dim3(kBlock), 0, s, k, tab, B, y, fe);
    return hipGetLastError();
}

}  // namespace afs
