// Matern covariance on the device (paper Section 4.1, eq. "maternkernel"):
//   C(d) = sigma2 / (Gamma(nu) 2^(nu-1)) * (d/beta)^nu * K_nu(d/beta),  C(0) = sigma2.
//
// nu = 1/2, 3/2, 5/2 use the exact elementary forms of x^nu K_nu(x).  Any
// other nu evaluates K_nu(x) itself:
//  * x < 2: Temme's series (N. M. Temme, J. Comput. Phys. 19, 1975) for
//    K_mu and K_{mu+1}, |mu| <= 1/2, followed by the upward recurrence
//    K_{v+1} = K_{v-1} + (2v/x) K_v up to nu = mu + N;
//  * x >= 2: the integral K_nu(x) = int_0^inf exp(-x cosh t) cosh(nu t) dt by
//    the trapezoidal rule, which converges geometrically for this analytic,
//    doubly-exponentially decaying integrand; the step shrinks like 1/sqrt(x)
//    to resolve the peak at t = 0.
// The theta-only constants (Gamma values of mu and nu) are computed once per
// parameter vector on the host.
#pragma once

#include <hip/hip_runtime.h>

namespace tlr {

struct MaternConst {
    double sigma2;
    double beta;
    double nu;
    double mu;      // nu - N, in [-1/2, 1/2)
    double coef;    // sigma2 / (Gamma(nu) 2^(nu-1))
    double gam1;    // (1/Gamma(1-mu) - 1/Gamma(1+mu)) / (2 mu), limit -gamma_E at mu = 0
    double gam2;    // (1/Gamma(1-mu) + 1/Gamma(1+mu)) / 2
    double gp;      // Gamma(1+mu)
    double gm;      // Gamma(1-mu)
    double fact;    // mu pi / sin(mu pi), 1 at mu = 0
    int N;          // number of upward recurrence steps
    int kind;       // 0 general, 1 nu=1/2, 2 nu=3/2, 3 nu=5/2
    // general nu: piecewise Chebyshev table of h(s) = log(x^nu K_nu(x)) + x,
    // s = log x, on [s_lo, s_lo + nint / inv_w], kChebDeg+1 coefficients per piece
    const double *tab;
    double s_lo, inv_w;
    int nint;
};

// Parsimonious bivariate Matern model (paper Section 4.2.1, eq. "bivmatern"):
// the three functions C_11, C_12, C_22 as univariate Matern constants (one
// range a; nu_12 = (nu_11 + nu_22)/2; the variance field of C_12 is
// rho_12 sigma_11 sigma_22, which may be zero or negative).  Matrix entry
// 2p + v is variable v at location p; on = 0 for the univariate model.
struct BivConst {
    MaternConst m[3];  // C_11, C_12, C_22 (index v + w)
    int32_t on;
    int32_t pad;
};

constexpr int kChebDeg = 10;
constexpr int kChebPieces = 160;
constexpr double kTabXlo = 1e-6;
constexpr double kTabXhi = 745.0;

// Host: constants of one theta.  Returns false for invalid theta.
bool make_matern_const(double sigma2, double beta, double nu, MaternConst *out);
// Host: the three functions of a bivariate theta (tables not yet attached).
// False for invalid theta (a variance, the range or a smoothness not
// positive, |beta_12| > 1, anything not finite).
bool make_biv_const(double s11, double s22, double a, double nu11, double nu22, double beta12, BivConst *out);

__device__ inline void temme_k(double mu, double x, const MaternConst &c, double *kmu, double *kmu1) {
    const double L = log(2.0 / x);
    const double sig = mu * L;
    const double shs = (sig == 0.0) ? 1.0 : sinh(sig) / sig;
    double f = c.fact * (cosh(sig) * c.gam1 + shs * L * c.gam2);
    const double es = exp(sig);
    double p = 0.5 * es * c.gp;
    double q = 0.5 / es * c.gm;
    double ck = 1.0;
    double s0 = f, s1 = p;
    const double x2 = 0.25 * x * x;
    for (int k = 1; k < 64; ++k) {
        const double kd = (double)k;
        f = (kd * f + p + q) / (kd * kd - mu * mu);
        p /= (kd - mu);
        q /= (kd + mu);
        ck *= x2 / kd;
        const double tf = ck * f;
        s0 += tf;
        s1 += ck * (p - kd * f);
        if (fabs(tf) < 1e-17 * fabs(s0)) break;
    }
    *kmu = s0;
    *kmu1 = s1 * (2.0 / x);
}

// exp(x) * K_nu(x) for x >= 2 by the trapezoidal rule on the cosh integral.
__device__ inline double scaled_k_integral(double nu, double x) {
    const double h = fmin(0.2, 0.6 * rsqrt(x));
    const double T = acosh(1.0 + 45.0 / x);
    const int npts = (int)ceil(T / h);
    double s = 0.5;
    for (int k = 1; k <= npts; ++k) {
        const double t = h * (double)k;
        const double sh = sinh(0.5 * t);
        s += exp(-2.0 * x * sh * sh) * cosh(nu * t);  // cosh t - 1 = 2 sinh^2(t/2)
    }
    return h * s;
}

// x^nu K_nu(x), x > 0, general nu.
__device__ inline double xnu_knu(double x, const MaternConst &c) {
    if (x >= 2.0) {
        return exp(c.nu * log(x) - x) * scaled_k_integral(c.nu, x);
    }
    double k0, k1;
    temme_k(c.mu, x, c, &k0, &k1);
    for (int j = 0; j < c.N; ++j) {
        const double k2 = k0 + 2.0 * (c.mu + (double)j + 1.0) / x * k1;
        k0 = k1;
        k1 = k2;
    }
    return pow(x, c.nu) * k0;
}

// h(s) = log(x^nu K_nu(x)) + x by the accurate evaluator (table nodes).
__device__ inline double log_xnu_knu_scaled(double x, const MaternConst &c) {
    if (x >= 2.0) return c.nu * log(x) + log(scaled_k_integral(c.nu, x));
    return log(xnu_knu(x, c)) + x;
}

// x^nu K_nu(x) from the table (x in [kTabXlo, kTabXhi]).
__device__ inline double xnu_knu_tab(double x, const MaternConst &c) {
    const double u = (log(x) - c.s_lo) * c.inv_w;
    int idx = (int)u;
    idx = idx < 0 ? 0 : (idx >= c.nint ? c.nint - 1 : idx);
    const double t = 2.0 * (u - (double)idx) - 1.0;
    const double *cf = c.tab + idx * (kChebDeg + 1);
    double b1 = 0.0, b2 = 0.0;
#pragma unroll
    for (int m = kChebDeg; m >= 1; --m) {
        const double b0 = cf[m] + 2.0 * t * b1 - b2;
        b2 = b1;
        b1 = b0;
    }
    const double h = cf[0] + t * b1 - b2;
    // exp(h) exp(-x): each factor keeps its own relative accuracy, unlike
    // exp(h - x) whose large argument carries |h - x| ulp of rounding
    return (x < 700.0) ? exp(h) * exp(-x) : exp(h - x);
}

__device__ inline double matern_cov(double d, const MaternConst &c) {
    const double x = d / c.beta;
    switch (c.kind) {
        case 1:
            return c.sigma2 * exp(-x);
        case 2:
            return c.sigma2 * (1.0 + x) * exp(-x);
        case 3:
            return c.sigma2 * (1.0 + x + x * x / 3.0) * exp(-x);
        default:
            if (x == 0.0) return c.sigma2;
            if (x > 745.0) return 0.0;
            return c.coef * xnu_knu(x, c);
    }
}

}  // namespace tlr
