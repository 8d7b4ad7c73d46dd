"""Oracle for the constraints-based attenuation of narrow-band fluctuations
(Sec. 3, Eqs. 3-7, Figs. 3 and 4).

Test infrastructure only (see the package docstring).

The TDDFT spectrum is split as S = S_p + S_n (Eq. 3), with F = F_p + F_n for
the ITCFs (Eq. 4).  S_p comes from a Savitzky-Golay filter: at every sample
the least-squares polynomial of a given degree over a window of samples
around it, evaluated there.  Window and degree are found by a grid search
scored by the corrected Akaike criterion plus two penalties, one on what is
left of the fluctuations' frequencies in the spectrum of dS/dw and one on
the curvature of S_p; a solution must leave the ITCF nearly unchanged:
|F_n / F| small at every tau (Eq. 5) and a small RMS deviation of F_n from
its mean compared with F(beta/2) (Eq. 7).

Readings (the paper gives no formulas for these):
  * near the ends the window is moved inside the grid and the same fit is
    evaluated at the sample (the usual "interp" edge rule);
  * the effective number of parameters k of a filter is the trace of its
    smoother matrix (the sum of the weights of each sample in its own
    filtered value); AICc = n ln(RSS/n) + 2k + 2k(k+1)/(n-k-1);
  * the spectrum of dS/dw is the squared modulus of the mean of the
    central-difference derivative times exp(-2 pi i nu w) over the interior
    samples; the frequency penalty is the mean over the target frequencies of
    (power after filtering) / (power before);
  * the curvature penalty is the sum of squared second differences after
    filtering over the same sum before;
  * the selection minimises AICc / n + lam_f P_freq + lam_c P_curv among the
    filters that meet the residual tolerances; by default lam_f = 100 and
    lam_c = 10, so that leaving a fluctuation's power in place costs more
    than the AICc gains by fitting it (a few nats per sample for ripples of
    a few per cent over noise), and the tolerances are the bounds the paper
    reports for its selected filters (|Fbar_n| / F(beta/2) < 0.4 %,
    sigma_n / F(beta/2) <= 0.0042 %);
  * Eq. 7 prints the same symbol for the bound and the variable of its
    integral and calls sigma_n a normalised root-mean-square deviation: it is
    read as sigma_n = [(1/beta) int_0^beta (F_n - Fbar_n)^2 dtau]^{1/2}, the
    RMS over [0, beta], with Fbar_n the mean of F_n there; integrals are the
    composite trapezoid on the tau grid.
"""
from __future__ import annotations

import numpy as np


def _window_start(i, n, w):
    return min(max(i - w // 2, 0), n - w)


def sg_filter(y, w, p):
    """Savitzky-Golay filter of degree p and odd window w: each output is the
    degree-p least-squares polynomial over the window around it evaluated at
    that sample (np.polyfit per sample)."""
    y = np.asarray(y, dtype=np.float64)
    n = len(y)
    if w % 2 != 1 or w <= p or w > n:
        raise ValueError("window must be odd, above the degree and at most n")
    out = np.empty(n)
    for i in range(n):
        s = _window_start(i, n, w)
        x = np.arange(s, s + w, dtype=np.float64) - i
        coef = np.polyfit(x, y[s:s + w], p)
        out[i] = coef[-1]  # the polynomial at x = 0
    return out


def sg_hat_diag(n, w, p):
    """Weight of sample i in its own filtered value: the leverage of sample i
    in the least-squares fit over its window, i.e. the squared norm of row
    i - s of an orthonormal basis Q of the polynomials on the window (QR of
    the Vandermonde matrix, abscissae scaled to [-1, 1] so that Q is
    accurate at degree 8; the projection Q Q^T does not depend on scaling)."""
    h = np.empty(n)
    for i in range(n):
        s = _window_start(i, n, w)
        x = (np.arange(s, s + w, dtype=np.float64) - (s + 0.5 * (w - 1))) / max(0.5 * (w - 1), 1.0)
        Q, _ = np.linalg.qr(np.vander(x, p + 1, increasing=True))
        h[i] = float(Q[i - s] @ Q[i - s])
    return h


def derivative_psd(S, omegas, nus):
    """Power of the central-difference dS/dw at each frequency nu (cycles per
    unit of w)."""
    S = np.asarray(S, dtype=np.float64)
    w = np.asarray(omegas, dtype=np.float64)
    D = (S[2:] - S[:-2]) / (w[2:] - w[:-2])
    wi = w[1:-1]
    out = np.empty(len(nus))
    for k, nu in enumerate(nus):
        z = np.sum(D * np.exp(-2j * np.pi * nu * wi)) / len(D)
        out[k] = abs(z) ** 2
    return out


def aicc(rss, n, k):
    """Corrected Akaike criterion of a fit with k parameters to n samples."""
    if n - k - 1 <= 0:
        return np.inf
    return n * np.log(rss / n) + 2 * k + 2 * k * (k + 1) / (n - k - 1)


def sg_scores(S, Sp, hdiag, omegas, nus):
    """(RSS, k, AICc, P_freq, P_curv) of one filtered spectrum Sp."""
    S = np.asarray(S, dtype=np.float64)
    Sp = np.asarray(Sp, dtype=np.float64)
    n = len(S)
    rss = float(np.sum((Sp - S) ** 2))
    k = float(np.sum(hdiag))
    if len(nus):
        pf = float(np.mean(derivative_psd(Sp, omegas, nus) / derivative_psd(S, omegas, nus)))
    else:
        pf = 0.0
    c0 = float(np.sum(np.diff(S, 2) ** 2))
    cp = float(np.sum(np.diff(Sp, 2) ** 2))
    pc = cp / c0 if c0 > 0 else np.nan
    return np.array([rss, k, aicc(rss, n, k), pf, pc])


def residual_itcf(F_ref, F_p, taus, beta):
    """(max |F_n / F_ref|, Fbar_n / F_ref(beta/2), sigma_n / F_ref(beta/2)) of
    F_n = F_ref - F_p (Eqs. 5 and 7).  A grid that ends at beta/2 is first
    extended to [0, beta] by F(tau) = F(beta - tau)."""
    Fr = np.asarray(F_ref, dtype=np.float64)
    Fn = Fr - np.asarray(F_p, dtype=np.float64)
    t = np.asarray(taus, dtype=np.float64)
    tol = 1e-12 * beta
    if t[0] != 0.0:
        raise ValueError("tau grid must start at 0")
    mid = np.nonzero(np.abs(t - 0.5 * beta) <= tol)[0]
    if len(mid) == 0:
        raise ValueError("tau grid must hold beta/2")
    f_half = Fr[mid[-1]]
    eps_max = float(np.max(np.abs(Fn / Fr)))
    if abs(t[-1] - 0.5 * beta) <= tol:
        t = np.concatenate([t, beta - t[-2::-1]])
        Fn = np.concatenate([Fn, Fn[-2::-1]])
    elif abs(t[-1] - beta) > tol:
        raise ValueError("tau grid must end at beta/2 or beta")
    mean = np.trapezoid(Fn, t) / beta
    # Eq. 7 as the root-mean-square deviation over [0, beta]: the square
    # root of the mean of (F_n - Fbar_n)^2, so that sigma_n / F(beta/2) does
    # not depend on the unit of tau
    sigma = np.sqrt(np.trapezoid((Fn - mean) ** 2, t) / beta)
    return np.array([eps_max, mean / f_half, sigma / f_half])


def sg_select(scores, resid, n_w, lam_f=100.0, lam_c=10.0, mean_tol=4e-3, sigma_tol=4.2e-5):
    """Index of the filter with the smallest AICc/n + lam_f P_freq + lam_c P_curv
    among those meeting the residual tolerances, or -1."""
    best, jb = -1, np.inf
    for f, o in enumerate(np.asarray(scores, dtype=np.float64)):
        J = o[2] / n_w + lam_f * o[3] + lam_c * o[4]
        if not np.isfinite(J):
            continue
        if resid is not None:
            r = resid[f]
            if not (abs(r[1]) <= mean_tol and r[2] <= sigma_tol):
                continue
        if J < jb:
            best, jb = f, J
    return best
