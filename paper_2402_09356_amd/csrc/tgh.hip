// Tukey g-and-h random fields (paper Section 4.2.2): T = xi + omega tau(Z),
// tau(z) = (exp(g z) - 1)/g exp(h z^2/2) (g = 0: z exp(h z^2/2)), Z a
// standard Gaussian random field.  For h >= 0 tau is strictly increasing and
// the log-likelihood of observations t follows by the change of variables:
//     l_TGH = l_Gauss(z) - sum_i log(omega tau'(z_i)),  z_i = tau^-1((t_i - xi)/omega).
//
// k_tgh_inverse: one thread per observation.  h = 0 has the closed form
// z = log1p(g y)/g; otherwise Newton's method on tau(z) - y inside a bracket
// [lo, hi] with tau(lo) <= y <= tau(hi) (grown by doubling from [-1, 1]),
// falling back to the bracket's midpoint whenever a step leaves the bracket
// or tau overflows, until the step is below a few ulps of z.  A value with
// no preimage (h = 0, g y <= -1) or not finite gives z = NaN.
//
// k_tgh_combine: one work-group, a fixed-order reduction of
// log(omega tau'(z_i)) = log omega + h z^2/2 + log(exp(g z) + h z expm1(g z)/g),
// then l_TGH = l_Gauss - that sum in place of out[2] (and the sum in out[3]);
// -inf when either part is not finite.  The tree is the same on every call,
// so results are bitwise reproducible.
#include "kernels.h"
#include "ktimer.h"

namespace tlr {
namespace {

__device__ inline double tgh_core(double z, double g) {  // (exp(g z) - 1)/g, z at g = 0
    return (g == 0.0) ? z : expm1(g * z) / g;
}

__device__ inline double tgh_tau(double z, double g, double h) { return tgh_core(z, g) * exp(0.5 * h * z * z); }

__global__ __launch_bounds__(256) void k_tgh_inverse(const double *__restrict__ t, int64_t n, double xi, double omega,
                                                     double g, double h, double *__restrict__ z) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double y = (t[i] - xi) / omega;
    double out = __builtin_nan("");
    if (isfinite(y)) {
        if (h == 0.0) {
            if (g == 0.0)
                out = y;
            else if (g * y > -1.0)
                out = log1p(g * y) / g;
        } else {
            double lo = -1.0, hi = 1.0;
            for (int it = 0; it < 64 && tgh_tau(lo, g, h) > y; ++it) lo *= 2.0;
            for (int it = 0; it < 64 && tgh_tau(hi, g, h) < y; ++it) hi *= 2.0;
            // start from the h = 0 solution where it exists, clipped into the bracket
            double x = (g != 0.0 && g * y > -1.0) ? log1p(g * y) / g : y;
            x = fmin(fmax(x, lo), hi);
            for (int it = 0; it < 200; ++it) {
                const double e = exp(0.5 * h * x * x), core = tgh_core(x, g);
                const double f = core * e - y;
                if (f == 0.0) break;
                if (f < 0.0)
                    lo = x;
                else
                    hi = x;
                const double fp = e * (exp(g * x) + h * x * core);
                double xn = x - f / fp;
                if (!(xn > lo && xn < hi)) xn = 0.5 * (lo + hi);  // outside, or not finite
                const double step = fabs(xn - x);
                x = xn;
                if (step <= 4.0 * 2.220446049250313e-16 * fabs(x) || hi - lo <= 4.0 * 2.220446049250313e-16 * fabs(x))
                    break;
            }
            out = x;
        }
    }
    z[i] = out;
}

__global__ __launch_bounds__(1024) void k_tgh_combine(const double *__restrict__ z, int64_t n, double omega, double g,
                                                      double h, double *__restrict__ out) {
    __shared__ double s[1024];
    const int tid = threadIdx.x;
    double acc = 0.0;
    for (int64_t i = tid; i < n; i += 1024) {
        const double x = z[i];
        const double inner = (g == 0.0) ? 1.0 + h * x * x : exp(g * x) + h * x * (expm1(g * x) / g);
        acc += 0.5 * h * x * x + log(inner);
    }
    s[tid] = acc;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
        if (tid < w) s[tid] += s[tid + w];
        __syncthreads();
    }
    if (tid == 0) {
        const double logjac = (double)n * log(omega) + s[0];
        const double lg = out[2];
        out[3] = logjac;
        out[2] = (isfinite(lg) && isfinite(logjac)) ? lg - logjac : -INFINITY;
    }
}

}  // namespace

tlr_status tgh_inverse(const double *t, int64_t n, double xi, double omega, double g, double h, double *z,
                       hipStream_t s) {
    if (n <= 0) return TLR_OK;
    static const int cls = ktimer_class("k_tgh_inverse");
    KTimer kt(cls, s, 0.0, 16.0 * (double)n, true);
    hipLaunchKernelGGL(k_tgh_inverse, dim3((unsigned)cdiv(n, 256)), dim3(256), 0, s, t, n, xi, omega, g, h, z);
    TLR_HIP(hipGetLastError());
    return TLR_OK;
}

tlr_status tgh_combine(const double *z, int64_t n, double omega, double g, double h, double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_tgh_combine, dim3(1), dim3(1024), 0, s, z, n, omega, g, h, out);
    TLR_HIP(hipGetLastError());
    return TLR_OK;
}

}  // namespace tlr
