"""Oracle for the Kubo-Greenwood route of the eta test and the attenuation
(Sec. A.3, with Eqs. 8, A-1 and A-2).

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

from oracle.response import dsf


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
