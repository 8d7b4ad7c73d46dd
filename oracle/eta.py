"""Oracle for the eta-convergence test in imaginary time (Sec. 2, Eq. 2, Fig. 2).

Test infrastructure only (see the package docstring).

For an ITCF F(q, tau) on a tau grid the test looks at the minimum F(beta/2),
the area A = int_0^beta F dtau (so that the static response is
chi(q) = -n A), and the same two quantities of the shifted ITCF of Eq. 2,
F~(tau) = F(tau) - F(0), which drops the tau-independent part that the
quasi-elastic and the omega -> 0 parts of S leave in F.  The reference eta is
the largest eta over which the shifted quantities have converged (Sec. 2);
"converged" is read as: within a relative tolerance of their values at the
smallest eta, for every eta up to it.
"""
from __future__ import annotations

import numpy as np


def itcf_metrics(F, taus, beta, density):
    """[F(beta/2), A, F~(beta/2), int F~, chi(q)] of one ITCF on `taus`.

    The grid starts at 0 and ends at beta, or at beta/2 with the rest of
    [0, beta] given by F(tau) = F(beta - tau); it must hold beta/2.  The
    integrals are the composite trapezoid on the grid (the reading used for
    Eq. 1 as well)."""
    F = np.asarray(F, dtype=np.float64)
    t = np.asarray(taus, dtype=np.float64)
    tol = 1e-12 * beta
    if t[0] != 0.0:
        raise ValueError("tau grid must start at 0")
    if abs(t[-1] - beta) <= tol:
        factor = 1.0
    elif abs(t[-1] - 0.5 * beta) <= tol:
        factor = 2.0
    else:
        raise ValueError("tau grid must end at beta or beta/2")
    mid = np.flatnonzero(np.abs(t - 0.5 * beta) <= tol)
    if len(mid) == 0:
        raise ValueError("tau grid must hold beta/2")
    area = 0.0
    for j in range(len(t) - 1):
        area += 0.5 * (t[j + 1] - t[j]) * (F[j] + F[j + 1])
    area *= factor
    f_half, f0 = F[mid[-1]], F[0]
    return np.array([f_half, area, f_half - f0, area - beta * f0, -density * area])


def eta_reference(metrics, etas, tol):
    """Index of the largest eta such that every eta from the smallest one up to
    it has both shifted metrics (columns 2 and 3) within `tol` (relative) of
    their values at the smallest eta."""
    m = np.asarray(metrics, dtype=np.float64)
    etas = np.asarray(etas, dtype=np.float64)
    if np.any(np.diff(etas) <= 0):
        raise ValueError("etas must increase")
    ref = 0
    for i in range(1, len(etas)):
        ok = all(abs(m[i, c] - m[0, c]) <= tol * abs(m[0, c]) for c in (2, 3))
        if not ok:
            break
        ref = i
    return ref
