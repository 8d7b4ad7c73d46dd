"""Oracle for the dielectric properties obtained from S (Sec. 3 and A.2).

Test infrastructure only (see the package docstring).

From S(q, w) on a frequency grid 0 <= w_0 < w_1 < ...: the FDT (Eq. 8, in
the normalisation used for S throughout) gives Im chi = -pi n (1 - e^{-beta w}) S;
the Kramers-Kronig relation of a causal response with Im chi odd in w gives
  Re chi(w) = (2/pi) P int_0^inf w' Im chi(w') / (w'^2 - w^2) dw',
taken here with Im chi linear between grid points and zero past the grid;
then eps^{-1} = 1 + (4 pi / q^2) chi (Eq. A-1) and eps = 1 + (4 pi i / w)
sigma (Eq. A-2).
"""
from __future__ import annotations

import math

import numpy as np


def _pv_linear(x, f, c):
    """P int over the grid x of the piecewise-linear f(w') / (w' - c) dw'.

    On [a, b] with slope s: int [f(c) + s (w' - c)] / (w' - c) dw' =
    f(c) (ln|b - c| - ln|a - c|) + s (b - a), f(c) the interval's line at c;
    the log(0) terms cancel between the two intervals that meet at c (the
    principal value) and are left out."""
    a, b = x[:-1], x[1:]
    s = (f[1:] - f[:-1]) / (b - a)
    fc = f[:-1] + s * (c - a)
    with np.errstate(divide="ignore"):
        lb = np.where(b != c, np.log(np.abs(b - c)), 0.0)
        la = np.where(a != c, np.log(np.abs(a - c)), 0.0)
    return float(np.sum(fc * (lb - la) + s * (b - a)))


def kramers_kronig_re(im_chi, omegas, at=None):
    """Re chi at the grid frequencies (or at the grid indices `at`) from Im
    chi on the same grid."""
    x = np.asarray(omegas, dtype=np.float64)
    f = np.asarray(im_chi, dtype=np.float64)
    idx = range(len(x)) if at is None else at
    return np.array([(_pv_linear(x, f, x[i]) + _pv_linear(x, f, -x[i])) / math.pi for i in idx])


def dielectric(S, omegas, beta, density, q2):
    """(chi, eps^{-1}, sigma) at every grid frequency from S."""
    w = np.asarray(omegas, dtype=np.float64)
    im = -math.pi * density * (-np.expm1(-beta * w)) * np.asarray(S, dtype=np.float64)
    chi = kramers_kronig_re(im, w) + 1j * im
    eps_inv = 1.0 + (4.0 * math.pi / q2) * chi
    eps = 1.0 / eps_inv
    sigma = (eps - 1.0) * w / (4j * math.pi)
    return chi, eps_inv, sigma
