// Host-side numerics: REXI coefficients, per-mode operator coefficients and
// the geometric checks on a pole set.  Plain C++ in extended precision.
#include <cmath>
#include <complex>
#include <cstring>
#include <string>

#include "internal.h"

namespace rexi {

using cld = std::complex<long double>;

namespace {

// f(z) for exp and the exponential-integrator functions of Section 4.3.
// Near z = 0 psi_1, psi_2 use their Taylor series (the removable singularity
// the paper treats with L'Hopital's rule).
cld eval_fn(int fn, cld z) {
    if (fn == REXI_FN_EXP) return std::exp(z);
    const long double az = std::abs(z);
    if (az < 1e-3L) {
        // psi_1 = sum z^k/(k+1)!, psi_2 = sum z^k/(k+2)!
        cld term = 1.0L, sum = 0.0L;
        const int shift = fn == REXI_FN_PSI1 ? 1 : 2;
        long double fact = 1.0L;
        for (int k = 1; k <= shift; ++k) fact *= k;
        term = 1.0L / fact;
        for (int k = 0; k < 12; ++k) {
            sum += term;
            term *= z / static_cast<long double>(k + shift + 1);
        }
        return sum;
    }
    if (fn == REXI_FN_PSI1) return (std::exp(z) - 1.0L) / z;
    return (std::exp(z) - 1.0L - z) / (z * z);
}

}  // namespace

int coefficients(int fn, int N, double p0, double y, double* alpha, double* beta,
                 double* r_out, double* mu_out) {
    if (fn != REXI_FN_EXP && fn != REXI_FN_PSI1 && fn != REXI_FN_PSI2)
        return fail(REXI_EINVAL, "rexi_coefficients: unknown function id");
    if (N < 2 || (N & 1) || N > (1 << 20))
        return fail(REXI_EINVAL, "rexi_coefficients: N must be even and in [2, 2^20]");
    if (!(p0 > 0.0) || !(y > 0.0) || !std::isfinite(p0) || !std::isfinite(y))
        return fail(REXI_EINVAL, "rexi_coefficients: p0 and y must be positive and finite");
    if (!alpha || !beta) return fail(REXI_EINVAL, "rexi_coefficients: NULL output array");

    const long double P0 = p0, Y = y;
    const long double r = (P0 * P0 + Y * Y) / (2.0L * P0);   // circle through p0, +-iy
    const long double mu = P0 - r;
    const long double pi = 4.0L * std::atan(1.0L);
    for (int n = 0; n < N; ++n) {
        const long double th = 2.0L * pi * (static_cast<long double>(n) + 0.5L) / N;
        const cld w = std::polar(r, th);        // r e^{i theta_n}
        const cld z = w + mu;                   // point on the contour
        const cld a = -z;
        const cld b = -(w * eval_fn(fn, z)) / static_cast<long double>(N);
        alpha[2 * n] = static_cast<double>(a.real());
        alpha[2 * n + 1] = static_cast<double>(a.imag());
        beta[2 * n] = static_cast<double>(b.real());
        beta[2 * n + 1] = static_cast<double>(b.imag());
    }
    if (r_out) *r_out = static_cast<double>(r);
    if (mu_out) *mu_out = static_cast<double>(mu);
    return REXI_OK;
}

void build_mode_coef(int L, double a, double g, double Omega, ModeCoef* out) {
    const long double tw = 2.0L * Omega;
    for (int m = 0; m <= L; ++m) {
        const int kmin = m > 1 ? m : 1;
        for (int k = m; k <= L; ++k) {
            ModeCoef c{0.0, 0.0, 0.0, 0.0};
            const long double K = k;
            auto eps = [m](int l) -> long double {
                if (l <= m || l <= 0) return 0.0L;
                const long double L2 = static_cast<long double>(l) * l;
                return std::sqrt((L2 - static_cast<long double>(m) * m) / (4.0L * L2 - 1.0L));
            };
            if (k >= 1) {
                const long double Nk = K * (K + 1.0L);
                c.s = static_cast<double>(tw * m / Nk);
                c.gN = static_cast<double>(static_cast<long double>(g) * Nk /
                                           (static_cast<long double>(a) * a));
                if (k - 1 >= kmin) c.cm = static_cast<double>(tw * (K + 1.0L) / K * eps(k));
                if (k + 1 <= L) c.cp = static_cast<double>(tw * K / (K + 1.0L) * eps(k + 1));
            }
            out[mode_index(L, k, m)] = c;
        }
    }
}

void build_pole_data(const double* alpha, const double* beta, int N, PoleData* pd) {
    for (int n = 0; n < N; ++n) {
        const cld z(-static_cast<long double>(alpha[2 * n]), -static_cast<long double>(alpha[2 * n + 1]));
        const cld zi = 1.0L / z;
        pd[n].zr = static_cast<double>(z.real());
        pd[n].zi = static_cast<double>(z.imag());
        pd[n].zir = static_cast<double>(zi.real());
        pd[n].zii = static_cast<double>(zi.imag());
        pd[n].wr = -beta[2 * n];
        pd[n].wi = -beta[2 * n + 1];
    }
}

int winding_number(const PoleData* pd, int N, double x, double y) {
    // Sum of the turning angles of the closed polygon seen from (x, y).
    long double total = 0.0L;
    for (int n = 0; n < N; ++n) {
        const int k = (n + 1) % N;
        const long double ax = pd[n].zr - x, ay = pd[n].zi - y;
        const long double bx = pd[k].zr - x, by = pd[k].zi - y;
        total += std::atan2(ax * by - ay * bx, ax * bx + ay * by);
    }
    const long double pi = 4.0L * std::atan(1.0L);
    return static_cast<int>(std::lround(total / (2.0L * pi)));
}

double min_distance_to_segment(const PoleData* pd, int N, double rho) {
    double best = INFINITY;
    for (int n = 0; n < N; ++n) {
        const double yc = std::fmax(-rho, std::fmin(rho, pd[n].zi));
        const double d = std::hypot(pd[n].zr, pd[n].zi - yc);
        best = std::fmin(best, d);
    }
    return best;
}

}  // namespace rexi
