// Host-side tables of the spherical-harmonic transforms, in extended precision:
// Gauss-Legendre nodes and weights, the three-term recurrence coefficients of
// the normalised associated Legendre functions, their seeds Pbar_mm(mu_j) split
// into mantissa and base-2 exponent, and the FFT twiddle factors.
#include <cmath>
#include <vector>

#include "internal.h"

namespace rexi {

namespace {

// eps_l^m = sqrt((l^2 - m^2) / (4 l^2 - 1)), zero for l <= m.
long double eps_lm(int l, int m) {
    if (l <= m || l <= 0) return 0.0L;
    const long double L2 = static_cast<long double>(l) * l;
    return std::sqrt((L2 - static_cast<long double>(m) * m) / (4.0L * L2 - 1.0L));
}

}  // namespace

// Gauss-Legendre nodes of the northern hemisphere in 80-bit arithmetic.  The
// unknown is the colatitude theta; P_n(cos theta) is evaluated through
// t = 1 - cos(theta) = 2 sin^2(theta/2) with Reinsch's form of the three-term
// recurrence (it carries D_k = P_k - P_{k-1}), so sin(theta) and the weight keep
// full relative accuracy next to the pole.  w = 2 sin^2(theta) / (n (t P_n - D_n))^2.
void gauss_north(int n, std::vector<long double>& mu, std::vector<long double>& sint,
                 std::vector<long double>& w) {
    const int half = n / 2;
    mu.resize(half);
    sint.resize(half);
    w.resize(half);
    const long double pi = 4.0L * std::atan(1.0L);
    auto pn = [n](long double t, long double& D) {
        long double P = 1.0L - t;
        D = -t;
        for (int k = 2; k <= n; ++k) {
            D = ((k - 1) * D - (2 * k - 1) * t * P) / k;
            P += D;
        }
        return P;
    };
    for (int j = 0; j < half; ++j) {
        long double th = pi * (j + 0.75L) / (n + 0.5L);
        for (int it = 0; it < 100; ++it) {
            const long double sh = std::sin(0.5L * th);
            const long double t = 2.0L * sh * sh;
            long double D;
            const long double P = pn(t, D);
            const long double dP = -n * (t * P - D) / std::sin(th);   // d/dtheta P_n(cos theta)
            const long double d = P / dP;
            th -= d;
            if (std::fabs(d) < 1e-22L * (1.0L + th)) break;
        }
        const long double sh = std::sin(0.5L * th);
        const long double t = 2.0L * sh * sh;
        long double D;
        const long double P = pn(t, D);
        const long double s = std::sin(th);
        const long double q = n * (t * P - D);
        mu[j] = std::cos(th);
        sint[j] = s;
        w[j] = 2.0L * s * s / (q * q);
    }
}

void build_legendre_tables(int L, int nlat, double a, ShtHost& out) {
    std::vector<long double> mu, sint, w;
    gauss_north(nlat, mu, sint, w);
    const int half = nlat / 2;
    out.half = half;
    out.mu.resize(half);
    out.sint.resize(half);
    out.w.resize(half);
    for (int j = 0; j < half; ++j) {
        out.mu[j] = static_cast<double>(mu[j]);
        out.sint[j] = static_cast<double>(sint[j]);
        out.w[j] = static_cast<double>(w[j]);
    }

    // recurrence coefficients per (l, m), m-major like the spectral state
    const int modes = n_modes(L);
    out.rec.assign(modes, LegCoef{0, 0, 0, 0});
    for (int m = 0; m <= L; ++m) {
        for (int l = m; l <= L; ++l) {
            const long double e1 = eps_lm(l + 1, m), e0 = eps_lm(l, m);
            LegCoef c;
            c.A = static_cast<double>(1.0L / e1);
            c.B = static_cast<double>(e0 / e1);
            c.hA = static_cast<double>(-static_cast<long double>(l) * e1);
            c.hB = static_cast<double>((l + 1.0L) * e0);
            out.rec[mode_index(L, l, m)] = c;
        }
    }
    // per-degree factors: a / (l(l+1)) and l(l+1) / a^2 (0 for l = 0)
    out.a_over_n.assign(L + 2, 0.0);
    out.n_over_a2.assign(L + 2, 0.0);
    for (int l = 1; l <= L + 1; ++l) {
        const long double N = static_cast<long double>(l) * (l + 1);
        out.a_over_n[l] = static_cast<double>(static_cast<long double>(a) / N);
        out.n_over_a2[l] = static_cast<double>(N / (static_cast<long double>(a) * a));
    }
    // seeds Pbar_mm(mu_j) = c_m sin(theta_j)^m, c_0 = 1/sqrt(2), c_m = c_{m-1} sqrt((2m+1)/(2m)),
    // stored as mantissa * 2^exponent with exponent <= 0 only when the value is below 2^-960
    out.seed_m.assign(static_cast<size_t>(L + 1) * half, 0.0);
    out.seed_e.assign(static_cast<size_t>(L + 1) * half, 0);
    long double log2c = -0.5L;
    for (int m = 0; m <= L; ++m) {
        if (m > 0) log2c += 0.5L * std::log2((2.0L * m + 1.0L) / (2.0L * m));
        for (int j = 0; j < half; ++j) {
            const long double lg = log2c + m * std::log2(sint[j]);
            const size_t i = static_cast<size_t>(m) * half + j;
            if (lg >= -960.0L) {
                out.seed_m[i] = static_cast<double>(std::exp2(lg));
                out.seed_e[i] = 0;
            } else {
                const long double e = std::floor(lg) + 1.0L;
                out.seed_m[i] = static_cast<double>(std::exp2(lg - e));
                out.seed_e[i] = static_cast<int>(e);
            }
        }
    }
}

void build_twiddles(int M, std::vector<double>& tw) {
    // tw[2k], tw[2k+1] = cos, sin of -2 pi k / M  (forward sign)
    tw.resize(2 * static_cast<size_t>(M));
    const long double pi = 4.0L * std::atan(1.0L);
    for (int k = 0; k < M; ++k) {
        const long double ang = -2.0L * pi * k / M;
        tw[2 * k] = static_cast<double>(std::cos(ang));
        tw[2 * k + 1] = static_cast<double>(std::sin(ang));
    }
}

}  // namespace rexi
