// Host-side tables of the spherical-harmonic transforms, in extended precision:
// Gauss-Legendre nodes and weights, the three-term recurrence coefficients of
// the normalised associated Legendre functions, their seeds Pbar_mm(mu_j) split
// into mantissa and base-2 exponent, and the FFT twiddle factors.
#include <algorithm>
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
    out.mu_ld = mu;
    out.sint_ld = sint;
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
}

void build_segments(int L, int seg_len, const ShtHost& sh, SegHost& out) {
    const int half = sh.half;
    out.seg_len = seg_len;
    out.segbase.assign(L + 2, 0);
    out.seg_m.clear();
    out.seg_i0.clear();
    out.seg_n.clear();
    for (int m = 0; m <= L; ++m) {
        out.segbase[m] = static_cast<int>(out.seg_m.size());
        const int Lm = L - m + 1;
        for (int i0 = 0; i0 < Lm; i0 += seg_len) {
            out.seg_m.push_back(m);
            out.seg_i0.push_back(i0);
            out.seg_n.push_back(std::min(seg_len, Lm - i0));
        }
    }
    out.nseg = static_cast<int>(out.seg_m.size());
    out.segbase[L + 1] = out.nseg;
    out.seed_pm.assign(static_cast<size_t>(out.nseg) * half, 0.0);
    out.seed_p.assign(static_cast<size_t>(out.nseg) * half, 0.0);
    out.seed_e.assign(static_cast<size_t>(out.nseg) * half, 0);
    // 80-bit recurrence from Pbar_mm = c_m sin^m (representable in long double even
    // where it underflows double), recording (Pbar_{k0-1}, Pbar_{k0}) at each segment start
    long double log2c = -0.5L;
    for (int m = 0; m <= L; ++m) {
        if (m > 0) log2c += 0.5L * std::log2((2.0L * m + 1.0L) / (2.0L * m));
        const int Lm = L - m + 1;
        std::vector<long double> A(Lm), B(Lm);
        for (int i = 0; i < Lm; ++i) {
            const int l = m + i;
            const long double e1 = eps_lm(l + 1, m), e0 = eps_lm(l, m);
            A[i] = 1.0L / e1;
            B[i] = e0 / e1;
        }
        for (int j = 0; j < half; ++j) {
            const long double mu = sh.mu_ld[j];
            long double pm = 0.0L;
            long double p = std::exp2(log2c + m * std::log2(sh.sint_ld[j]));
            for (int i = 0; i < Lm; ++i) {
                if (i % seg_len == 0) {
                    const size_t k = static_cast<size_t>(out.segbase[m] + i / seg_len) * half + j;
                    const long double big = std::max(std::fabs(pm), std::fabs(p));
                    int e = 0;
                    if (big > 0.0L && big < 0x1p-960L) e = std::ilogb(big) + 1;
                    out.seed_pm[k] = static_cast<double>(std::ldexp(pm, -e));
                    out.seed_p[k] = static_cast<double>(std::ldexp(p, -e));
                    out.seed_e[k] = e;
                }
                const long double pn = A[i] * mu * p - B[i] * pm;
                pm = p;
                p = pn;
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
