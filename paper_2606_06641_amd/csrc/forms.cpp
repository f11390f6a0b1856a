// forms.cpp -- the two DFT evaluation forms of the precision study (Sec. 2.1.2
// for the method, Sec. 3.5 for the length ceiling it runs into).
//
// Form A, the paper's: the elementary symmetric polynomials of the literal values
// come from sampling Q(z) = prod_i (z + y_i) at the N = k + 1 roots of unity, so
//   FE(y) = Re sum_m c_m prod_i (omega^m + y_i),
//   c_m   = (1/N) sum_j fhat_(k-j) omega^(-m j),
// where fhat_t is the Walsh-Fourier coefficient shared by every literal set of
// size t (Sec. 2.1).  Near a corner the products range from about 2^k down to
// about eps^k, and the inverse DFT cancels them: the paper's ceiling near k = 50
// in FP64.
//
// Form B, the count basis the library's FE kernels use (in rotated, rescaled
// form): the factor of a literal is its true/false probability pair,
//   FE(y) = Re sum_m d_m prod_i (alpha_m + beta_m y_i),
//   alpha_m = (1 + omega^m)/2, beta_m = (1 - omega^m)/2,
//   d_m = (1/N) sum_t g(t) omega^(-m t),
// whose factors have modulus at most 1, so nothing overflows or cancels.
//
// fhat_t = 2^-k sum_s g(s) K_t(s), K_t(s) = sum_j (-1)^j C(t, j) C(k - t, s - j)
// (g(s) = -1 satisfied / +1 violated with s true literals; a true literal is
// y = -1).  The sum is exact in 128-bit integers (|sum| <= 2^k) and divided by
// 2^k only at the end, as Sec. 3.5.1 prescribes arbitrary-precision
// combinatorics with the division deferred.

#include "afsat.h"

#include <hip/hip_runtime_api.h>

#include <string>
#include <vector>

#include "host.hpp"
#include "instance.hpp"
#include "kernels.hpp"

namespace {

using afs::set_last_error;

constexpr int kFormAMaxLen = 120;     // 128-bit exactness of the Krawtchouk sums

// Walsh-Fourier coefficient per set size, t = 0..k
std::vector<long double> walsh_by_size(int type, int k, int param)
{
    typedef __int128 i128;
    std::vector<std::vector<i128>> C(k + 1, std::vector<i128>(k + 1, 0));
    for (int a = 0; a <= k; ++a) {
        C[a][0] = 1;
        for (int b = 1; b <= a; ++b) C[a][b] = C[a - 1][b - 1] + (b <= a - 1 ? C[a - 1][b] : 0);
    }
    std::vector<long double> out(k + 1);
    const long double scale = ldexpl(1.0L, -k);
    for (int t = 0; t <= k; ++t) {
        i128 acc = 0;
        for (int s = 0; s <= k; ++s) {
            i128 kr = 0;
            for (int j = 0; j <= t && j <= s; ++j) {
                if (s - j > k - t) continue;
                const i128 term = C[t][j] * C[k - t][s - j];
                kr += (j & 1) ? -term : term;
            }
            acc += afs::satisfied(type, k, param, s) == 1 ? -kr : kr;
        }
        out[t] = (long double)acc * scale;
    }
    return out;
}

}  // namespace

extern "C" {

afs_status afs_form_tables(int32_t type, int32_t k, int32_t param, int32_t form, double *alpha, double *beta,
                           double *d)
{
    if (!alpha || !beta || !d) return set_last_error(AFS_EINVAL, "output is NULL");
    if (type < 0 || type > 7) return set_last_error(AFS_EINVAL, "unknown type");
    if (form != AFS_FORM_A && form != AFS_FORM_B) return set_last_error(AFS_EINVAL, "unknown form");
    if (k < 1 || k > afs::kMaxLen) return set_last_error(AFS_EINVAL, "k out of range");
    if (form == AFS_FORM_A && k > kFormAMaxLen)
        return set_last_error(AFS_EINVAL, "form A tables are exact up to k = " + std::to_string(kFormAMaxLen));
    const int N = k + 1;
    std::vector<long double> c, s;
    afs::roots(N, c, s);
    if (form == AFS_FORM_B) {
        std::vector<double> re(N), im(N);
        afs::coefficients(type, k, param, re.data(), im.data());
        for (int m = 0; m < N; ++m) {
            alpha[2 * m] = (double)((1.0L + c[m]) / 2.0L);
            alpha[2 * m + 1] = (double)(s[m] / 2.0L);
            beta[2 * m] = (double)((1.0L - c[m]) / 2.0L);
            beta[2 * m + 1] = (double)(-s[m] / 2.0L);
            d[2 * m] = re[m];
            d[2 * m + 1] = im[m];
        }
        return AFS_OK;
    }
    const std::vector<long double> fh = walsh_by_size(type, k, param);
    for (int m = 0; m < N; ++m) {
        long double ar = 0.0L, ai = 0.0L;
        for (int j = 0; j <= k; ++j) {
            const int r = (int)(((int64_t)m * j) % N);
            ar += fh[k - j] * c[r];
            ai -= fh[k - j] * s[r];
        }
        alpha[2 * m] = (double)c[m];
        alpha[2 * m + 1] = (double)s[m];
        beta[2 * m] = 1.0;
        beta[2 * m + 1] = 0.0;
        d[2 * m] = (double)(ar / N);
        d[2 * m + 1] = (double)(ai / N);
    }
    return AFS_OK;
}

afs_status afs_fe_generic(int32_t k, const double *alpha, const double *beta, const double *d, int32_t fp64,
                          int32_t B, const double *y, double *fe, int32_t device, void *stream)
{
    if (!alpha || !beta || !d) return set_last_error(AFS_EINVAL, "table is NULL");
    if (k < 1 || k > afs::kMaxLen) return set_last_error(AFS_EINVAL, "k out of range");
    if (B < 0) return set_last_error(AFS_EINVAL, "B must be >= 0");
    if (B > 0 && (!y || !fe)) return set_last_error(AFS_EINVAL, "y or fe is NULL");
    if (B == 0) return AFS_OK;
    int prev = -1;
    if (hipGetDevice(&prev) != hipSuccess || hipSetDevice(device) != hipSuccess)
        return set_last_error(AFS_EDEVICE, "no HIP device " + std::to_string(device));
    const int N = k + 1;
    std::vector<double> tab((size_t)N * 6);
    for (int m = 0; m < N; ++m) {
        tab[6 * m + 0] = alpha[2 * m];
        tab[6 * m + 1] = alpha[2 * m + 1];
        tab[6 * m + 2] = beta[2 * m];
        tab[6 * m + 3] = beta[2 * m + 1];
        tab[6 * m + 4] = d[2 * m];
        tab[6 * m + 5] = d[2 * m + 1];
    }
    void *dtab = nullptr;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipMalloc(&dtab, tab.size() * sizeof(double));
    if (e == hipSuccess) e = hipMemcpy(dtab, tab.data(), tab.size() * sizeof(double), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = afs::launch_fe_generic(k, static_cast<const double *>(dtab), fp64 != 0, B, y, fe, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (dtab) (void)hipFree(dtab);
    (void)hipSetDevice(prev);
    if (e != hipSuccess) return set_last_error(AFS_EDEVICE, std::string("generic FE: ") + hipGetErrorString(e));
    return AFS_OK;
}

}  // extern "C"
