// Host-side numerics: REXI coefficients, per-mode operator coefficients and
// the geometric checks on a pole set.  Plain C++ in extended precision.
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

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

void coupling_row_max(int L, double Omega, std::vector<double>& out) {
    std::vector<ModeCoef> c(static_cast<size_t>(n_modes(L)));
    build_mode_coef(L, 1.0, 1.0, Omega, c.data());
    out.assign(static_cast<size_t>(L + 1), 0.0);
    for (int m = 0; m <= L; ++m)
        for (int k = m; k <= L; ++k) {
            const ModeCoef& q = c[mode_index(L, k, m)];
            out[k] = std::fmax(out[k], std::fabs(q.cm) + std::fabs(q.cp));
        }
}

int check_poles(const OperatorBounds& op, const PoleData* pd, int N, double dt, bool chain, const char* who,
                double* margin) {
    for (int n = 0; n < N; ++n) {
        const PoleData& q = pd[n];
        if (!std::isfinite(q.zr) || !std::isfinite(q.zi) || !std::isfinite(q.wr) || !std::isfinite(q.wi))
            return fail(REXI_EINVAL, std::string(who) + ": non-finite alpha or beta");
    }
    const double rho = dt * (std::sqrt(op.g * op.H * op.L * (op.L + 1.0)) / op.a + 2.0 * op.Omega);
    const double probes[5] = {-rho, -0.5 * rho, 0.0, 0.5 * rho, rho};
    for (double w : probes) {
        const int wn = winding_number(pd, N, 0.0, w);
        if (wn != 1 && wn != -1) {
            char buf[200];
            std::snprintf(buf, sizeof buf,
                          "%s: the poles do not enclose the spectrum of dt L "
                          "(winding %d around %.6g i; rho = %.6g)", who, wn, w, rho);
            return fail(REXI_ENUMERIC, buf);
        }
    }
    if (!(min_distance_to_segment(pd, N, rho) > 1e-6 * (1.0 + rho)))
        return fail(REXI_ENUMERIC, std::string(who) + ": a pole lies on the spectrum of dt L");
    // diagonal dominance of the chain rows, degree by degree (see check_poles in internal.h)
    auto dist = [](double x, double y, double top) {          // |(x, y) - i [0, top]|
        return std::hypot(x, y - std::fmax(0.0, std::fmin(top, y)));
    };
    double worst = INFINITY;
    int nworst = 0, kworst = 0;
    for (int k = 0; k <= op.L; ++k) {
        const double off = dt * op.off[k];
        if (!(off > 0.0)) continue;
        const double top = dt * 2.0 * op.Omega / (k + 1.0);
        const double g2 = dt * dt * op.H * op.g * k * (k + 1.0) / (op.a * op.a);
        for (int n = 0; n < N; ++n) {
            const PoleData& q = pd[n];
            const double bz = dist(q.zr, q.zi, top);
            const double bd = dist(std::fma(g2, q.zir, q.zr), std::fma(g2, q.zii, q.zi), top);
            const double r = std::fmin(bz, bd) / off;
            if (r < worst) {
                worst = r;
                nworst = n;
                kworst = k;
            }
        }
    }
    if (margin) *margin = worst;
    if (chain && !(worst > 1.0)) {
        char buf[300];
        std::snprintf(buf, sizeof buf,
                      "%s: the chain systems are not diagonally dominant (pole %d, degree %d: diagonal bound / "
                      "off-diagonal sum = %.4g); the unpivoted elimination is not guaranteed stable",
                      who, nworst, kworst, worst);
        return fail(REXI_ENUMERIC, buf);
    }
    return REXI_OK;
}

double spectral_radius(int L, double dt, double a, double g, double H, double Omega) {
    return dt * (std::sqrt(g * H * L * (L + 1.0)) / a + 2.0 * Omega);
}

void contour_error(const double* alpha, const double* beta, int N, double rho, int npts, double* approx,
                   double* kappa) {
    using cd = std::complex<double>;
    double emax = 0.0, kmax = 0.0;
    for (int k = 0; k < npts; ++k) {
        const double w = -rho + 2.0 * rho * static_cast<double>(k) / static_cast<double>(npts - 1);
        const cd x(0.0, w);
        cd sum(0.0, 0.0);
        double ks = 0.0;
        for (int n = 0; n < N; ++n) {
            const cd a(alpha[2 * n], alpha[2 * n + 1]), b(beta[2 * n], beta[2 * n + 1]);
            const cd d = x + a;
            sum += b / d;
            ks += std::abs(b) / std::abs(d);
        }
        if (approx) emax = std::fmax(emax, std::abs(sum - std::exp(x)));
        kmax = std::fmax(kmax, ks);
    }
    if (approx) *approx = emax;
    if (kappa) *kappa = kmax;
}

namespace {

// approx (1601 points) + u kappa (401 points) of the contour (p0, y, N) on
// i[-rho, rho]; +inf when the coefficients cannot be formed.
double predicted_error(double p0, double y, int N, double rho, double u, std::vector<double>& al,
                       std::vector<double>& be) {
    al.resize(2 * static_cast<size_t>(N));
    be.resize(2 * static_cast<size_t>(N));
    if (coefficients(REXI_FN_EXP, N, p0, y, al.data(), be.data(), nullptr, nullptr) != REXI_OK) return INFINITY;
    double approx = 0.0, kap = 0.0;
    contour_error(al.data(), be.data(), N, rho, 1601, &approx, nullptr);
    contour_error(al.data(), be.data(), N, rho, 401, nullptr, &kap);
    const double e = approx + u * kap;
    return std::isfinite(e) ? e : INFINITY;
}

}  // namespace

int choose_contour(double rho, double target, int prec, int N_fixed, const double* grid, int n_grid, int n_max,
                   double* p0_out, double* y_out, int* N_out, double* pred_out) {
    static const double kGrid[] = {2.0, 3.0, 4.0, 5.0, 6.0, 8.0, 10.0, 12.0, 14.0, 16.0, 20.0, 24.0, 28.0, 32.0};
    if (!grid) {
        grid = kGrid;
        n_grid = static_cast<int>(sizeof(kGrid) / sizeof(kGrid[0]));
    }
    const double u = (prec & REXI_PREC_FP32_SOLVE) ? std::ldexp(1.0, -24) : std::ldexp(1.0, -53);
    const double y = std::sqrt(2.0) * 1.05 * rho;
    std::vector<double> al, be;
    double best_p0 = 0.0, best_e = INFINITY;
    int best_N = 0;
    if (N_fixed > 0) {
        for (int i = 0; i < n_grid; ++i) {
            const double e = predicted_error(grid[i], y, N_fixed, rho, u, al, be);
            if (e < best_e) {
                best_e = e;
                best_p0 = grid[i];
            }
        }
        if (best_p0 == 0.0) return fail(REXI_ENUMERIC, "rexi_choose_contour: no shift of the grid gives finite coefficients");
        best_N = N_fixed;
    } else {
        for (int i = 0; i < n_grid; ++i) {
            const double p0 = grid[i];
            if (!(predicted_error(p0, y, n_max, rho, u, al, be) <= target)) continue;
            int lo = 1, hi = n_max / 2;            // N = 2 k, k in (lo, hi]
            if (best_N) hi = std::min(hi, best_N / 2);
            while (hi - lo > 1) {
                const int mid = (lo + hi) / 2;
                if (predicted_error(p0, y, 2 * mid, rho, u, al, be) <= target) hi = mid;
                else lo = mid;
            }
            const int N = 2 * hi;
            const double e = predicted_error(p0, y, N, rho, u, al, be);
            if (e <= target && (!best_N || N < best_N)) {
                best_N = N;
                best_p0 = p0;
                best_e = e;
            }
        }
        if (!best_N) {
            char buf[200];
            std::snprintf(buf, sizeof buf,
                          "rexi_choose_contour: no shift of the grid reaches %.3g with at most %d poles", target, n_max);
            return fail(REXI_ENUMERIC, buf);
        }
    }
    *p0_out = best_p0;
    *y_out = y;
    *N_out = best_N;
    *pred_out = best_e;
    return REXI_OK;
}

}  // namespace rexi
