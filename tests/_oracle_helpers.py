"""Reference scales for the GPU tests, computed from the oracle's pieces only.

term_scales: the largest magnitude among the terms of each component of the
non-linear tendency (Section 3: N_h = -div(h V), N_zeta = -div(zeta V),
N_delta = curl(zeta V) - lap(|V|^2/2)).  For a balanced jet the two terms of
N_delta nearly cancel, so rounding errors are relative to the terms, not to
their difference.

synthesis_term_sums / analysis_term_sums: per output entry, the sum of the
magnitudes of the products a transform adds up (Section 3.2), the quantity a
rounding bound multiplies.  Synthesis: sum over orders (weight 2 for m > 0,
which stand for +-m) of sum_l |f_lm| |Pbar_lm(mu_j)|, per latitude.
Analysis: sum_j w_j |Pbar_lm(mu_j)| |F_m(mu_j)| per (l, m)."""
import numpy as np

from oracle.operator import mode_index, n_modes
from oracle.sht import degree_array, inv_laplacian


def term_scales(g, U):
    L, a = g.L, g.p.a
    h, zeta, delta = U
    hg, zg = g.synthesis(h), g.synthesis(zeta)
    Ug, Vg = g.uv_from_psichi(inv_laplacian(zeta, L, a), inv_laplacian(delta, L, a))
    div_h, _ = g.div_curl(hg * Ug, hg * Vg)
    div_z, curl_z = g.div_curl(zg * Ug, zg * Vg)
    ke = g.analysis((Ug * Ug + Vg * Vg) / (2.0 * (g.sint[:, None] ** 2)))
    l = degree_array(L).astype(np.float64)
    lap = (l * (l + 1.0) / (a * a)) * ke
    return np.array([np.abs(div_h).max(), np.abs(div_z).max(), max(np.abs(curl_z).max(), np.abs(lap).max())])


def synthesis_term_sums(g, spec):
    L = g.L
    T = np.zeros(g.nlat)
    for m in range(L + 1):
        s = mode_index(L, m, m)
        T += (1.0 if m == 0 else 2.0) * (np.abs(spec[s:s + L - m + 1]) @ np.abs(g.P(m)))
    return T


def analysis_term_sums(g, field):
    L = g.L
    F = g._grid_to_fourier(field)
    T = np.zeros(n_modes(L))
    for m in range(L + 1):
        s = mode_index(L, m, m)
        T[s:s + L - m + 1] = np.abs(g.P(m)) @ (g.w * np.abs(F[m]))
    return T


def _rexi_orders(args):
    import os
    os.environ.setdefault("OMP_NUM_THREADS", "1")
    from oracle import linear
    U0, alpha, beta, dt, L, p, orders = args
    return linear.rexi_linear_step(U0, alpha, beta, dt, L, p, orders=orders)


def oracle_rexi_parallel(U0, alpha, beta, dt, L, p, workers=None):
    """oracle.linear.rexi_linear_step over all orders, the orders dealt round-robin
    to a pool of processes (each order's entries are written by one process)."""
    import concurrent.futures as cf
    import os
    workers = workers or min(16, len(os.sched_getaffinity(0)))
    chunks = [list(range(L, -1, -1))[i::workers] for i in range(workers)]
    with cf.ProcessPoolExecutor(max_workers=workers) as ex:
        parts = list(ex.map(_rexi_orders, [(U0, alpha, beta, dt, L, p, c) for c in chunks if c]))
    return sum(parts)


def tendency_error_bound(g, U, u_syn, u_ana):
    """First-order bound, per spectral entry [3, modes], on the error of the
    pseudo-spectral tendency N(U) (Section 3) when every synthesis output carries
    at most u_syn and every analysis output at most u_ana times the sum of the
    magnitudes of the products it adds (the FFTs and pointwise products exact to
    this order).  Built from the oracle's tables:

    * grid errors: h, zeta from sum_m w_m sum_l |x_lm| |Pbar_lm(mu_j)| (w_0 = 1,
      w_m = 2); U, V = (1/a) sum [-psi H + i m chi Pbar], (1/a) sum [i m psi Pbar
      + chi H] with |H_l| counted as |l eps_{l+1} Pbar_{l+1}| + |(l+1) eps_l Pbar_{l-1}|
      (the form a kernel may use);
    * products hU, hV, zeta U, zeta V, KE = (U^2 + V^2)/(2 sin^2): first-order
      propagation of those errors, averaged over longitude for the Fourier
      coefficients' bound (|F_m| <= mean_k |f_jk| for every m);
    * analysis: the propagated Fourier errors plus u_ana times the magnitudes of
      the quadrature terms, through div, curl (weights w_j / (a sin^2), factors m
      and |H|) and l(l+1)/a^2 for the kinetic energy term of N_delta."""
    from oracle.sht import legendre_m

    L, a = g.L, g.p.a
    h, zeta, delta = U
    psi = inv_laplacian(zeta, L, a)
    chi = inv_laplacian(delta, L, a)
    nlat = g.nlat
    s2 = g.sint ** 2
    # per-order tables: Pbar (l = m..L+1) and the two H terms
    tabs = []
    for m in range(L + 1):
        Pe = legendre_m(m, L + 1, g.mu, g.sint)            # [L - m + 2, nlat]
        n = L - m + 1
        hA = np.zeros((n, nlat))
        hB = np.zeros((n, nlat))
        for i in range(n):
            l = m + i
            e1 = np.sqrt(((l + 1) ** 2 - m * m) / (4.0 * (l + 1) ** 2 - 1.0))
            hA[i] = np.abs(l * e1 * Pe[i + 1])
            if i > 0:
                e0 = np.sqrt((l * l - m * m) / (4.0 * l * l - 1.0))
                hB[i] = np.abs((l + 1) * e0 * Pe[i - 1])
        tabs.append((np.abs(Pe[:n]), hA + hB))
    # synthesis term sums per latitude
    Th = np.zeros(nlat)
    Tz = np.zeros(nlat)
    TU = np.zeros(nlat)
    TV = np.zeros(nlat)
    for m in range(L + 1):
        s = mode_index(L, m, m)
        sl = slice(s, s + L - m + 1)
        P, Hs = tabs[m]
        wm = 1.0 if m == 0 else 2.0
        Th += wm * (np.abs(h[sl]) @ P)
        Tz += wm * (np.abs(zeta[sl]) @ P)
        TU += wm * (np.abs(psi[sl]) @ Hs + m * (np.abs(chi[sl]) @ P)) / a
        TV += wm * (m * (np.abs(psi[sl]) @ P) + np.abs(chi[sl]) @ Hs) / a
    hg, zg = g.synthesis(h), g.synthesis(zeta)
    Ug, Vg = g.uv_from_psichi(psi, chi)
    eh, ez, eU, eV = (u_syn * T[:, None] for T in (Th, Tz, TU, TV))
    prods = {"hU": hg * Ug, "hV": hg * Vg, "zU": zg * Ug, "zV": zg * Vg,
             "KE": (Ug * Ug + Vg * Vg) / (2.0 * s2[:, None])}
    perr = {"hU": eh * np.abs(Ug) + np.abs(hg) * eU, "hV": eh * np.abs(Vg) + np.abs(hg) * eV,
            "zU": ez * np.abs(Ug) + np.abs(zg) * eU, "zV": ez * np.abs(Vg) + np.abs(zg) * eV,
            "KE": (np.abs(Ug) * eU + np.abs(Vg) * eV) / s2[:, None]}
    Ebar = {k: v.mean(axis=1) for k, v in perr.items()}                        # per latitude
    Fabs = {k: np.abs(g._grid_to_fourier(v)) for k, v in prods.items()}        # [m, j]
    out = np.zeros((3, n_modes(L)))
    wd = g.w / (a * s2)
    for m in range(L + 1):
        s = mode_index(L, m, m)
        sl = slice(s, s + L - m + 1)
        P, Hs = tabs[m]

        def dc(A, B):
            """bound on a div or curl of the cos-weighted pair (A, B) at order m"""
            prop = P @ (wd * m * Ebar[A]) + Hs @ (wd * Ebar[B])
            rnd = P @ (wd * m * Fabs[A][m]) + Hs @ (wd * Fabs[B][m])
            return prop + u_ana * rnd
        l = np.arange(m, L + 1, dtype=np.float64)
        ke = P @ (g.w * Ebar["KE"]) + u_ana * (P @ (g.w * Fabs["KE"][m]))
        out[0, sl] = dc("hU", "hV")
        out[1, sl] = dc("zU", "zV")
        out[2, sl] = dc("zV", "zU") + l * (l + 1.0) / (a * a) * ke
    return out
