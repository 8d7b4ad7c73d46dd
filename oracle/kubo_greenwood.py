"""Oracle for the Kubo-Greenwood route of the eta test and the attenuation
(Sec. A.3, with Eqs. 8, A-1 and A-2), and for the Kubo-Greenwood
conductivity of the states that the route starts from.

Test infrastructure only (see the package docstring).

Starting from a conductivity sigma(w) in the optical limit: the dielectric
function is eps = 1 + 4 pi i sigma / w (Eq. A-2), the scaled density response
chi* = v(q) chi = 1/eps - 1 (Eq. A-1 with v = 4 pi / q^2), and the scaled
structure factor S* = v S follows from Im chi* by the fluctuation-dissipation
theorem, in the normalisation used for S everywhere here
(S = -Im chi / (pi n (1 - e^{-beta w})), the one under which the sum rules
of S hold).  The paper writes chi*_KG as the imaginary part of 1/eps; here
chi* is the complex 1/eps - 1, whose imaginary part that is, so that
eps^{-1} = 1 + chi* holds as printed.  F*, the eta metrics, the attenuation
and the way back (Re chi* by Kramers-Kronig, eps^{-1} = 1 + chi*,
sigma = i w (1 - eps) / (4 pi)) are those of S with v(q) chi in place of
chi, i.e. the dielectric step with q^2 = 4 pi.
"""
from __future__ import annotations

import numpy as np

from oracle.response import dsf, transitions


def chi_star(sigma, omegas):
    """1 / (1 + 4 pi i sigma / w) - 1 on the grid (NaN at w = 0)."""
    s = np.asarray(sigma, dtype=np.complex128)
    w = np.asarray(omegas, dtype=np.float64)
    out = np.full(len(w), np.nan + 0j)
    nz = w != 0.0
    out[nz] = 1.0 / (1.0 + 4j * np.pi * s[nz] / w[nz]) - 1.0
    return out


def kg_dsf(sigma, omegas, beta, density):
    """S*(w) from sigma(w): the FDT applied to chi* (w = 0 by the limit from
    the next grid point, as for S)."""
    return dsf(chi_star(sigma, omegas), omegas, beta, density)


KG_Q2 = 4.0 * np.pi  # q^2 at which 1 + (4 pi / q^2) chi is 1 + chi*


def momentum_elements(kred, millers, B, coef):
    """<m k| p_a |n k> for p = -i grad and every pair of the bands in coef
    (rows are bands, columns the plane waves of millers at k):
    sum_G conj(c_m(G)) (k + G)_a c_n(G).  Returns [3][nb][nb], element
    [a][m][n], a the Cartesian direction."""
    g = (np.asarray(kred, dtype=np.float64)[None, :] + np.asarray(millers)) @ np.asarray(B)
    C = np.asarray(coef)
    return np.stack([C.conj() @ (g[:, a][:, None] * C.T) for a in range(3)])


def kg_conductivity(st, omegas, eta, thr):
    """Kubo-Greenwood conductivity of the states, the trace average over the
    three Cartesian directions, with the delta function of the transitions
    broadened into a Lorentzian of half-width eta (the eta of the route's
    eta test, Sec. A.3):

      sigma(w) = 2 i / (Omega N_k) sum_t W_t / (w - delta_t + i eta),
      W_t = (df_t / delta_t) (1/3) sum_a |<m k| p_a |n k>|^2,

    over the transitions t = (k, n -> m) at q = 0 (delta = e_m - e_n,
    df = f_n - f_m) screened by |df| > thr, the list chi0 uses at q = 0.  The
    factor 2 counts the spins.  Its real part is the familiar
    (2 pi / (3 Omega w)) sum (f_n - f_m) |p_mn|^2 delta(e_m - e_n - w) per
    k-point weight 1/N_k with the delta function broadened, and the
    imaginary part is its Kramers-Kronig partner (each term is analytic in
    the upper half plane).  Terms with delta = 0 have df = 0 and are screened
    out.  Returns complex [n_w]."""
    w = np.asarray(omegas, dtype=np.float64)
    tr = transitions(st, (0, 0, 0), thr)
    out = np.zeros(len(w), dtype=np.complex128)
    for k in range(st.n_k):
        sel = np.nonzero(tr.k == k)[0]
        if len(sel) == 0:
            continue
        P = momentum_elements(st.kred[k], st.millers[k], st.B, st.coef[k])
        n, m = tr.n[sel], tr.m[sel]
        p2 = np.mean(np.abs(P[:, m, n]) ** 2, axis=0)
        d = tr.delta[sel]
        W = tr.df[sel] / d * p2
        out += (W[None, :] / (w[:, None] - d[None, :] + 1j * eta)).sum(axis=1)
    return 2j * out / (st.omega * st.n_k)
