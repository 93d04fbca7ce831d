/*
 * rexi_swe.h -- C-ABI of the MI355X (gfx950) library for REXI time stepping of
 * the shallow-water equations on the rotating sphere (Schreiber, Schaeffer &
 * Loft, arXiv:1805.06557).
 *
 * Conventions shared by every call
 * --------------------------------
 * - Every function returns an int status: REXI_OK (0) or a negative REXI_E*
 *   code.  Nothing aborts, throws or exits.  rexi_last_error() returns a
 *   thread-local message describing the last failure on the calling thread.
 * - Spectral states are device arrays of complex128 stored as interleaved
 *   (re, im) doubles.  A state holds 3 fields (h, zeta, delta) = (height
 *   perturbation h' = Phi'/g [m], relative vorticity [1/s], divergence [1/s]),
 *   field-major: field f occupies doubles [2 f modes, 2 (f + 1) modes).
 *   Within a field the (l, m) coefficient with 0 <= m <= l <= L sits at
 *   idx(l, m) = m (2L + 3 - m) / 2 + (l - m)   (m-major; modes = (L+1)(L+2)/2).
 *   Only m >= 0 is stored; the fields are real in physical space, so the
 *   m = 0 coefficients are real.  Normalisation: integral over [-1, 1] of
 *   Pbar_lm(mu)^2 dmu = 1, no Condon-Shortley phase, e^{+i m lambda}.
 * - Grid fields are device float64 arrays [nf][nlat][nlon]: Gauss-Legendre
 *   latitudes ordered north to south, longitudes lambda_k = 2 pi k / nlon.
 * - Device pointers are caller-owned; the library never frees them.  Calls
 *   that take a hipStream_t enqueue their work on that stream and return
 *   without waiting; device buffers must stay valid until that work is done.
 *   Errors found by the host (bad arguments, a contour that does not enclose
 *   the spectrum) are returned at once; nothing is enqueued in that case.
 * - A context (swe_ctx) owns its device tables, cached REXI coefficients and
 *   workspaces.  It is bound to the device that was current at swe_create.
 *   Calls on one context must not run concurrently from several host threads.
 */
#ifndef REXI_SWE_H
#define REXI_SWE_H

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    REXI_OK = 0,
    REXI_EINVAL = -1,   /* invalid argument (size, pointer, parameter) */
    REXI_ENOMEM = -2,   /* device or host allocation failed */
    REXI_EDEVICE = -3,  /* HIP runtime error (launch, copy, no device) */
    REXI_ENOTSUP = -4,  /* operation not available for this context */
    REXI_ENUMERIC = -5  /* numerically invalid set-up (contour, dominance) */
};

/* Functions approximated by the rational sum (Section 4.3: psi_0 = exp,
 * psi_1(z) = (e^z - 1)/z, psi_2(z) = (e^z - 1 - z)/z^2). */
enum { REXI_FN_EXP = 0, REXI_FN_PSI1 = 1, REXI_FN_PSI2 = 2 };

/* Precision modes of a context (bit flags; 0 = everything in FP64).
 * REXI_PREC_FP32_SOLVE: the banded REXI solves run in complex FP32.  The
 *   pole-independent row data (couplings, dt terms, right-hand sides) are
 *   formed in FP64 and rounded once to FP32; the pole-dependent diagonal
 *   z + dt^2 g H l(l+1)/(a^2 z) - i dt m q_l and right-hand-side term t/z are
 *   formed in FP32 from z and 1/z rounded to FP32, and the pivot reciprocal is
 *   the hardware's FP32 reciprocal without refinement (a backward error of a
 *   few FP32 units relative to the diagonal, the size the FP32 sweep makes
 *   anyway).  Each pole's solution is weighted in FP32 (by -beta_n rounded to
 *   FP32 once) and the weighted solutions of the (at most two) poles a GPU
 *   lane carries are added in FP32; that sum is widened to FP64, and the sum
 *   over all poles accumulates in FP64 (Section 4.2.2: the sum cancels; its
 *   terms are up to kappa = sum |beta_n| / |x + alpha_n| times larger than the
 *   result).
 * REXI_PREC_BF16_SPLIT, REXI_PREC_FP16_SPLIT (exclusive): the Legendre
 *   contractions of the transforms (Section 3.2) run on the matrix cores with
 *   every operand split into two 16-bit values (hi + lo) and three products
 *   accumulated in FP32: relative error per product about 2^-16 (BF16) or
 *   2^-22 (FP16; data columns scaled by exact powers of two into FP16's
 *   range), plus FP32 accumulation over the latitudes or degrees.  FFTs,
 *   products and the time stepping stay FP64. */
enum {
    REXI_PREC_FP64 = 0,
    REXI_PREC_FP32_SOLVE = 1,
    REXI_PREC_BF16_SPLIT = 2,
    REXI_PREC_FP16_SPLIT = 4
};

typedef struct swe_ctx swe_ctx;

/*
 * rexi_coefficients -- poles and weights of the rational approximation
 *   f(x) ~ sum_{n<N} beta_n / (x + alpha_n)
 * from the N-point trapezoidal rule of the Cauchy integral on the circle
 * through p0 > 0 and +-i y (Section 4.2.1, Eq. cauchy_alpha and Eq.
 * cauchy_beta; circle from Section 4.2.2: r = (p0^2 + y^2) / (2 p0),
 * centre mu = p0 - r):
 *   theta_n = 2 pi (n + 1/2) / N,  alpha_n = -(r e^{i theta_n} + mu),
 *   beta_n  = -(1/N) r e^{i theta_n} f(r e^{i theta_n} + mu).
 * Host only; touches no device.  Computed in extended precision and rounded
 * once.  fn: REXI_FN_*.  N: even, 2 <= N <= 1<<20.  alpha, beta:
 * caller-owned host arrays of 2N doubles (interleaved re, im).  r, mu: may be
 * NULL; otherwise receive the radius and centre.
 * Errors: REXI_EINVAL for a bad fn, odd/out-of-range N, p0 <= 0, y <= 0 or a
 * NULL alpha/beta.
 */
int rexi_coefficients(int fn, int N, double p0, double y,
                      double* alpha, double* beta, double* r, double* mu);

/*
 * rexi_check_contour -- the host checks that rexi_linear_step applies to a
 * coefficient set before it enqueues anything, without a context or device:
 * alpha, beta finite; the polygon of the poles z_n = -alpha_n winds once
 * around the segment i[-rho, rho], rho = dt (sqrt(g H L(L+1))/a + 2 Omega),
 * which holds the spectrum of dt L (Section 4.2.1: the contour must enclose
 * the spectrum); and every row of every chain system of the banded solve
 * (z_n I - dt L_m with h eliminated) is strictly diagonally dominant, the
 * condition under which its unpivoted elimination is stable.  Per degree l
 * the orders m <= l shift the diagonal by dt m q_l, q_l = 2 Omega/(l(l+1)),
 * within i[0, dt 2 Omega/(l+1)]: the zeta-row diagonal z - i dt m q_l is at
 * least the distance of z from that segment and the delta-row diagonal
 * z + dt^2 g H l(l+1)/(a^2 z) - i dt m q_l at least the distance of
 * z + dt^2 g H l(l+1)/(a^2 z) from it, while the row's off-diagonals (the
 * Coriolis couplings to degrees l -+ 1) sum to at most dt max_m (|c^-| + |c^+|).
 * margin (may be NULL) receives the smallest ratio of the two over poles and
 * degrees (> 1 passes).  alpha, beta: host arrays of 2N doubles.
 * Host only.
 * Errors: REXI_EINVAL (bad sizes or constants, NULL arrays, non-finite
 * coefficients), REXI_ENUMERIC (a check fails; *margin is still written when
 * the winding check passed).
 */
int rexi_check_contour(int L, double a, double g, double H, double Omega, double dt,
                       const double* alpha, const double* beta, int N, double* margin);

/*
 * rexi_spectral_radius -- rho = dt (sqrt(g H L(L+1))/a + 2 Omega), a bound on
 * |lambda| over the spectrum of dt L (L = L_g + L_c; gravity-wave frequencies
 * plus the Coriolis term).  Host only.  Errors: REXI_EINVAL.
 */
int rexi_spectral_radius(int L, double dt, double a, double g, double H, double Omega, double* rho);

/*
 * rexi_contour_error -- the accuracy of a coefficient set (alpha, beta: host,
 * 2N doubles) on the spectrum segment i[-rho, rho] (Section 4.2.2):
 *   *approx = max_w |S(i w) - e^{i w}|,  *kappa = max_w sum_n |beta_n| / |i w + alpha_n|,
 * over npts (>= 2) equally spaced w in [-rho, rho], S(x) = sum_n beta_n / (x + alpha_n)
 * summed in FP64 in pole order.  kappa is the cancellation factor of the sum:
 * a solve with unit roundoff u carries an error of about u kappa.  Host only.
 * Errors: REXI_EINVAL.
 */
int rexi_contour_error(const double* alpha, const double* beta, int N, double rho, int npts,
                       double* approx, double* kappa);

/*
 * rexi_choose_contour -- a contour for a target accuracy on i[-rho, rho]
 * (the contour must enclose the spectrum, Section 4.2.1; the shift trades the
 * trapezoidal rule's error against the cancellation of the sum, Section
 * 4.2.2): y = sqrt(2) 1.05 rho, and p0 from p0_grid (n_p0 values; NULL: 2, 3,
 * 4, 5, 6, 8, 10, 12, 14, 16, 20, 24, 28, 32).  The predicted error of a
 * contour is approx + u kappa (rexi_contour_error with 1601 points for approx
 * and 401 for kappa; u = 2^-53 for prec 0, 2^-24 with REXI_PREC_FP32_SOLVE).
 * N_fixed == 0: the contour with the fewest even N <= n_max whose prediction
 * is <= target (ties: the first p0 of the grid).  N_fixed > 0 (even): the p0 of
 * the grid with the smallest prediction at that N (target and n_max unused).
 * Outputs (host): *p0, *y, *N, *predicted.  Host only.
 * Errors: REXI_EINVAL; REXI_ENUMERIC when no p0 of the grid meets the target.
 */
int rexi_choose_contour(double rho, double target, int prec, int N_fixed, const double* p0_grid, int n_p0,
                        int n_max, double* p0, double* y, int* N, double* predicted);

/*
 * swe_create -- context for truncation L on an nlat x nlon Gauss grid with
 * planet radius a [m], gravity g [m/s^2], mean depth H [m], rotation rate
 * Omega [1/s] and precision flags prec (REXI_PREC_*).
 * nlat = nlon = 0 makes a linear-only context (no transforms, no nonlinear
 * step).  Otherwise nlat > L, nlat even, nlon > 2L and nlon a multiple of 4.
 * 1 <= L <= 1023.  On success *out receives the context.
 * Errors: REXI_EINVAL, REXI_ENOMEM, REXI_EDEVICE.
 */
int swe_create(int L, int nlat, int nlon, double a, double g, double H,
               double Omega, int prec, swe_ctx** out);

/* swe_destroy -- waits for the context's work and frees it.  NULL is a no-op. */
int swe_destroy(swe_ctx* ctx);

/*
 * rexi_linear_step -- the REXI linear stage (Section 4.2, Eq. rexi):
 *   U1 = sum_{n<N} beta_n (dt L + alpha_n I)^{-1} U0,  L = L_g + L_c,
 * the paper's sign convention, with alpha/beta as from rexi_coefficients.
 * L_g: h_t = -H delta, delta_t = -g lap h.  L_c: the Coriolis terms with
 * f = 2 Omega sin(phi) (Section 3), which couple degree l to l +- 1 within
 * each zonal order m: every (pole, m) system is banded and is solved on the
 * device as two complex tridiagonal chains after eliminating h.
 * alpha, beta: host arrays of 2N doubles; they are copied to the device and
 * cached inside the context (keyed by their contents and dt), together with
 * the chain factorization when a streaming schedule is selected
 * (swe_set_tuning); the cache is written on the stream of the call that
 * rebuilds it, so a later call on another stream must be ordered after that
 * call by the caller.  U0, U1: device states [3][modes] complex128; they must
 * not overlap.
 * Before enqueueing, the host applies the checks of rexi_check_contour (the
 * poles enclose the spectrum; the chain systems are diagonally dominant, so
 * the unpivoted elimination is stable); otherwise REXI_ENUMERIC.
 * Non-finite outputs are reported by swe_sync.
 * Errors: REXI_EINVAL (N odd or < 2, dt <= 0, NULL pointers), REXI_ENUMERIC,
 * REXI_ENOMEM, REXI_EDEVICE.
 */
int rexi_linear_step(swe_ctx* ctx, const double* alpha, const double* beta,
                     int N, double dt, const double* U0, double* U1,
                     hipStream_t stream);

/*
 * rexi_lg_step -- the REXI stage of the gravity-wave part L_g alone (Section 3:
 * L_g couples h and delta of one degree, zeta is left alone):
 *   U1 = sum_n beta_n (dt L_g + alpha_n)^-1 U0,
 * computed per degree from two sums over the poles and applied per mode
 * (no banded solve).  U1 may equal U0.  Same contour checks and errors as
 * rexi_linear_step, without the dominance check (there is no chain solve).
 */
int rexi_lg_step(swe_ctx* ctx, const double* alpha, const double* beta, int N, double dt,
                 const double* U0, double* U1, hipStream_t stream);

/*
 * rexi_lg_step_noalloc -- rexi_lg_step for callers that cannot allocate device
 * memory: code being captured into a HIP graph, tight serving loops, harnesses
 * that forbid hipMalloc.  Same kernels and the same result bits as
 * rexi_lg_step; the pole table and the per-degree sums live in a static
 * device array of the library (229 408 bytes per device, held until the
 * process ends) instead of context allocations, so the call allocates
 * nothing on the device.  Limits: N <= 4096 (and L <= 1023, as for every
 * context).  The array keeps the last call's contents: a call whose
 * (alpha, beta, N, dt) differ from the previous call's on that device uploads
 * the new pole table on `stream` and waits for the stream; a call with the
 * same set only enqueues the two kernels.  Every call on one device shares the
 * array, so calls that may overlap on one device (several streams or host
 * threads) race; the caller orders them.
 * Errors: REXI_EINVAL (as rexi_lg_step, and N > 4096), REXI_ENUMERIC,
 * REXI_ENOTSUP, REXI_EDEVICE.
 */
int rexi_lg_step_noalloc(swe_ctx* ctx, const double* alpha, const double* beta, int N, double dt,
                         const double* U0, double* U1, hipStream_t stream);

/*
 * rexi_linear_step_batched -- the REXI linear stage (Section 4.2, Eq. rexi)
 * of an ensemble of independent problems, each with its own context (own
 * truncation), coefficients, pole count and dt, in one row-record launch, one
 * fused chain-solve launch over the work items of every member (longest
 * chains first) and one pole-sum launch.  Per member the result is bit for
 * bit that of rexi_linear_step with the launch shape of members[0].ctx (which
 * is the shape used for all).  All members need distinct contexts on one
 * device with the same solve precision.  The argument and work-item tables
 * are cached in members[0].ctx and re-uploaded only when a member's pointers,
 * N, dt, coefficients or the launch shape change; with nothing changed the
 * call only enqueues kernels, so it can be captured into a HIP graph after
 * one eager call.
 * Errors: REXI_EINVAL (count outside [1, 4096], NULL pointers, a context used
 * twice, mixed device or precision, bad N or dt, overlapping U0/U1),
 * REXI_ENUMERIC, REXI_ENOMEM, REXI_ENOTSUP, REXI_EDEVICE.
 */
typedef struct {
    swe_ctx* ctx;
    const double* alpha;   /* host, 2N doubles */
    const double* beta;    /* host, 2N doubles */
    int N;
    double dt;
    const double* U0;      /* device [3][modes(ctx)] complex128 */
    double* U1;            /* device [3][modes(ctx)] complex128 */
} rexi_member;
int rexi_linear_step_batched(const rexi_member* members, int count, hipStream_t stream);

/*
 * sh_synthesis -- spectral to grid for nf scalar fields (Section 3.2):
 *   f(lambda_k, mu_j) = sum_l Pbar_l0 Re f_l0 + 2 Re sum_{m>=1} sum_l f_lm Pbar_lm(mu_j) e^{i m lambda_k}.
 * spec: device complex128 [nf][modes]; grid: device float64 [nf][nlat][nlon].
 * Errors: REXI_ENOTSUP for a linear-only context, REXI_EINVAL, REXI_EDEVICE.
 */
int sh_synthesis(swe_ctx* ctx, const double* spec, double* grid, int nf,
                 hipStream_t stream);

/*
 * sh_analysis -- grid to spectral for nf scalar fields by Gauss quadrature:
 *   f_lm = sum_j w_j Pbar_lm(mu_j) (1/nlon) sum_k f_jk e^{-i m lambda_k}.
 * grid: device float64 [nf][nlat][nlon]; spec: device complex128 [nf][modes].
 * Errors: as sh_synthesis.
 */
int sh_analysis(swe_ctx* ctx, const double* grid, double* spec, int nf,
                hipStream_t stream);

/*
 * swe_nonlinear_step -- integrates dU/dt = N(U) over tau with the
 * second-order explicit Runge-Kutta method of Heun (Section 4.1 and Table 2,
 * ``erk``):  U1 = U0 + tau/2 (N(U0) + N(U0 + tau N(U0))), where (Section 3)
 *   N_h = -div(h V),  N_zeta = -div(zeta V),  N_delta = k.curl(zeta V) - lap(|V|^2 / 2)
 * are formed pseudo-spectrally on the context's grid.  U0, U1: device states
 * [3][modes]; U1 may equal U0 (in place).
 * Errors: REXI_ENOTSUP for a linear-only context, REXI_EINVAL, REXI_EDEVICE.
 */
int swe_nonlinear_step(swe_ctx* ctx, double tau, const double* U0, double* U1,
                       hipStream_t stream);

/*
 * swe_strang_step -- one step of l_rexi_n_erk_ver1 (Section 4.4, version 1):
 *   U1 = N^{dt/2} o REXI^{dt} o N^{dt/2} (U0), 2 Heun steps and 1 REXI stage.
 * Arguments as rexi_linear_step / swe_nonlinear_step; U1 may equal U0.
 */
int swe_strang_step(swe_ctx* ctx, const double* alpha, const double* beta,
                    int N, double dt, const double* U0, double* U1,
                    hipStream_t stream);

/*
 * swe_strang_steps -- nsteps (>= 1) consecutive swe_strang_step steps from U0,
 * the result in U1 (U1 may equal U0).  Same result bits as nsteps separate
 * calls; in split-precision contexts with fusion on (swe_set_fusion) the last
 * analysis of each step is fused with the first synthesis of the next, which
 * separate calls cannot do.  The states between steps are kept in U1 and in
 * the context's own buffer.
 * Errors: as swe_strang_step; REXI_EINVAL for nsteps < 1.
 */
int swe_strang_steps(swe_ctx* ctx, const double* alpha, const double* beta,
                     int N, double dt, int nsteps, const double* U0, double* U1,
                     hipStream_t stream);

/* swe_sync -- waits for all work on the context's device; returns REXI_EDEVICE
 * if the device reported an error, and REXI_ENUMERIC if any kernel of this
 * context wrote a non-finite value (NaN or infinity) into an output since the
 * last swe_sync: the REXI/linear stage outputs, the non-linear step outputs
 * and the transform outputs set a device-side flag word (the error text names
 * which); the flag is cleared by the call that reports it. */
int swe_sync(swe_ctx* ctx);

/* rexi_last_error -- thread-local text of the last error ("" if none).  The
 * pointer stays valid until the next library call on the same thread. */
const char* rexi_last_error(void);

/*
 * swe_cn_step -- the Crank-Nicolson step of the linear part (Section 4.1,
 * the implicit baseline ``irk``): U1 = (I - dt/2 L)^-1 (I + dt/2 L) U0 with
 * L = L_g + L_c, computed as -U0 + 4 (2 I - dt L)^-1 U0 by the same banded
 * chain solve with one real shift.  U0, U1: device states [3][modes], must
 * not overlap.  Errors: REXI_EINVAL, REXI_ENOMEM, REXI_EDEVICE.
 */
int swe_cn_step(swe_ctx* ctx, double dt, const double* U0, double* U1, hipStream_t stream);

/*
 * swe_split_step -- one Strang-split step of the full equations (Section 4.4)
 * with the non-linear part by Heun (``erk``):
 *   REXI_SPLIT_REXI_V1  l_rexi_n_erk_ver1: N^{dt/2} o REXI^{dt} o N^{dt/2}
 *   REXI_SPLIT_REXI_V0  l_rexi_n_erk_ver0: REXI^{dt/2} o N^{dt} o REXI^{dt/2}
 *   REXI_SPLIT_CN_V1    l_irk_n_erk_ver1:  N^{dt/2} o CN^{dt} o N^{dt/2}
 *   REXI_SPLIT_CN_V0    l_irk_n_erk_ver0:  CN^{dt/2} o N^{dt} o CN^{dt/2}
 *   REXI_SPLIT_LG_REXI_V1  lg_rexi_lc_n_erk_ver1: REXI on the gravity-wave part
 *                       L_g alone (rexi_lg_step), the Coriolis part L_c joined to
 *                       N and formed on the grid through the absolute vorticity
 *                       (Section 3 splitting, Section 5.3 fastest REXI variant)
 * For the REXI schemes alpha, beta (host, 2N doubles) must approximate exp on
 * the spectrum of the linear step's length (dt for version 1, dt/2 for
 * version 0); the CN schemes ignore them (they may be NULL).  U1 may equal U0.
 * Errors: REXI_ENOTSUP for a linear-only context, REXI_EINVAL, REXI_ENUMERIC,
 * REXI_ENOMEM, REXI_EDEVICE.
 */
enum { REXI_SPLIT_REXI_V1 = 0, REXI_SPLIT_REXI_V0 = 1, REXI_SPLIT_CN_V1 = 2, REXI_SPLIT_CN_V0 = 3,
       REXI_SPLIT_LG_REXI_V1 = 4 };
int swe_split_step(swe_ctx* ctx, int scheme, const double* alpha, const double* beta, int N, double dt,
                   const double* U0, double* U1, hipStream_t stream);

/*
 * swe_etdrk2_step -- one step of l_rexi_n_etdrk, the second-order exponential
 * time differencing Runge-Kutta scheme (Section 4.3, Eq. etdrk) with
 * L = L_g + L_c applied through REXI and N explicit:
 *   A  = psi_0(dt L) U0 + dt psi_1(dt L) N(U0)
 *   U1 = A + dt psi_2(dt L) (N(A) - N(U0)),
 * psi_0 = exp, psi_1(K) = K^-1 (exp(K) - I), psi_2(K) = K^-2 (exp(K) - I - K).
 * alpha: the poles of one contour; beta0, beta1, beta2: the weights of psi_0,
 * psi_1, psi_2 on it (rexi_coefficients with REXI_FN_EXP, REXI_FN_PSI1,
 * REXI_FN_PSI2 and the same N, p0, y); host arrays of 2N doubles.  U0, U1:
 * device states [3][modes]; U1 may equal U0.  Two non-linear evaluations and
 * three REXI stages; the three coefficient sets stay cached in the context.
 * Errors: REXI_ENOTSUP for a linear-only context, REXI_EINVAL, REXI_ENUMERIC,
 * REXI_ENOMEM, REXI_EDEVICE.
 */
int swe_etdrk2_step(swe_ctx* ctx, const double* alpha, const double* beta0, const double* beta1,
                    const double* beta2, int N, double dt, const double* U0, double* U1,
                    hipStream_t stream);

/*
 * Per-kernel timing (tracing).  swe_profile(ctx, 1) starts recording a HIP
 * event pair on the launch stream around every launch of the given kernels
 * (up to 4096 launches per kernel between reads); swe_profile(ctx, 0) stops.
 * swe_profile_read waits for the recorded events, returns the summed device
 * duration [ms] and the launch count of one kernel since the last read, and
 * resets that kernel's record.  kernel: REXI_KERNEL_*.
 * Errors: REXI_EINVAL (NULL, bad kernel id), REXI_EDEVICE.
 */
enum {
    REXI_KERNEL_SOLVE = 0,       /* banded chain solves + per-wave pole sums */
    REXI_KERNEL_REDUCE = 1,      /* sum of the pole-block partial sums */
    REXI_KERNEL_LEG_SYNTH = 2,   /* Legendre synthesis (spectral -> Fourier) */
    REXI_KERNEL_RING = 3,        /* longitude FFTs and pointwise products */
    REXI_KERNEL_LEG_ANAL = 4,    /* Legendre analysis (Fourier -> spectral) */
    REXI_KERNEL_FACTOR = 5,      /* pivots of the chain factorization (once per coefficient set and dt) */
    REXI_KERNEL_LEG_FUSED = 6,   /* split precision: a Heun step's first analysis fused with the next synthesis */
    REXI_KERNEL_COUNT = 7
};
int swe_profile(swe_ctx* ctx, int enable);
/* The same for a subset: bit k of mask records kernel k (0 stops recording).
 * Errors: REXI_EINVAL for a NULL context. */
int swe_profile_kernels(swe_ctx* ctx, unsigned mask);
int swe_profile_read(swe_ctx* ctx, int kernel, double* total_ms, int* launches);

/*
 * Schedules of the REXI chain solve.  All three give bit-identical results.
 *   REXI_SOLVER_FUSED:  the pivots are recomputed in both sweeps; nothing but
 *                       the state and the tables is read (arithmetic bound).
 *   REXI_SOLVER_STREAM: the pivots of every (pole, chain row) are computed
 *                       once per coefficient set and dt into a cache held by
 *                       the context (2 modes x N x 8 B in FP32, 16 B in FP64)
 *                       and read by both sweeps (HBM bound).
 *   REXI_SOLVER_HYBRID: the forward sweep reads the cached pivots, the backward
 *                       pass recomputes them.
 * The cache is rebuilt when alpha, beta, N, dt or the solve precision change.
 */
enum { REXI_SOLVER_FUSED = 1, REXI_SOLVER_STREAM = 2, REXI_SOLVER_HYBRID = 3 };

/*
 * swe_set_tuning -- choose the schedule and launch shape of the REXI solve:
 * solver = REXI_SOLVER_*, seg_rows = rows per register-resident segment of
 * the chain sweep, waves = waves per workgroup (1, 2 or 4), poles_per_lane =
 * poles whose sweeps one lane interleaves (1 or 2).  seg_rows is 16 or 32 with
 * one pole per lane and 8 or 16 with two; another pairing makes the next
 * solve fail with REXI_ENOTSUP.
 * 0 keeps the current value.  The schedule, seg_rows and waves never change
 * the result bits; poles_per_lane regroups the pole sum (results agree to
 * rounding).
 * Errors: REXI_EINVAL for an unsupported value.
 */
int swe_set_tuning(swe_ctx* ctx, int solver, int seg_rows, int waves, int poles_per_lane);

/* swe_get_tuning -- the current schedule and launch shape (see swe_set_tuning).
 * Errors: REXI_EINVAL for NULL arguments. */
int swe_get_tuning(swe_ctx* ctx, int* solver, int* seg_rows, int* waves, int* poles_per_lane);

/*
 * swe_set_fusion -- launch fusion of the split-precision transforms (contexts
 * created with REXI_PREC_BF16_SPLIT or REXI_PREC_FP16_SPLIT): with enable = 1
 * (the default) the first analysis of every Heun step is fused with the
 * synthesis of its output, and in swe_strang_step the pole sum of the REXI
 * stage with the synthesis of its result; 0 runs the separate launches.  The
 * result bits are the same either way (Section 3.2 transforms; Section 4.4
 * splitting).  swe_get_fusion returns the setting.
 * Errors: REXI_EINVAL (NULL context or pointer, enable not 0 or 1).
 */
int swe_set_fusion(swe_ctx* ctx, int enable);
int swe_get_fusion(swe_ctx* ctx, int* enable);

/*
 * swe_autotune -- times every supported schedule and launch shape of the REXI
 * stage on this problem (reps timed calls each, after one untimed call that
 * also builds a factorization where the schedule needs one) with HIP events
 * on `stream`, and keeps the fastest in the context.  U1 is overwritten with
 * the REXI stage of U0.  *best_ms (may be NULL) receives the mean time of one
 * stage with the chosen shape.  If the fused schedule wins, the cached
 * factorization is released.  Synchronizes the stream.
 * Errors: as rexi_linear_step, REXI_EINVAL for reps outside [1, 1000].
 */
int swe_autotune(swe_ctx* ctx, const double* alpha, const double* beta, int N, double dt,
                 const double* U0, double* U1, int reps, hipStream_t stream, double* best_ms);

#ifdef __cplusplus
}
#endif

#endif /* REXI_SWE_H */
