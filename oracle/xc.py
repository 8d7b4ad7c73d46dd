"""Oracle adiabatic LDA kernel f_xc = d^2(n eps_xc)/dn^2.

Test infrastructure only (see the package docstring).

The paper uses an adiabatic (static) GGA kernel (Sec. A.1).  The model here
is its local-density form: Slater exchange plus the Perdew-Wang 1992
parametrisation of the unpolarised correlation energy,
  eps_c(rs) = -2A (1 + a1 rs) ln[1 + 1/(2A (b1 rs^1/2 + b2 rs + b3 rs^3/2 + b4 rs^2))]
with A = 0.031091, a1 = 0.21370, b1..b4 = 7.5957, 3.5876, 1.6382, 0.49294
(Hartree; Phys. Rev. B 45, 13244 (1992), Table I, zeta = 0 column).

The kernel matrix is f_xc(G - G') with
  f_xc(G) = (1/N_r) sum_j f_xc(n(r_j)) exp(-i G.r_j)
on the real-space grid r_j = sum_i (j_i/N_i) a_i, and
  n(r_j) = 2/(N_k Omega) sum_kn f_nk |sum_G c_nk(G) exp(i G.r_j)|^2.
"""
from __future__ import annotations

import math

import numpy as np

PW92_A = 0.031091
PW92_A1 = 0.21370
PW92_B = (7.5957, 3.5876, 1.6382, 0.49294)


def rs_of(n):
    return (3.0 / (4.0 * math.pi * np.asarray(n, dtype=np.float64))) ** (1.0 / 3.0)


def _pw92_terms(rs):
    """eps_c and its first two rs-derivatives."""
    A, a1 = PW92_A, PW92_A1
    b1, b2, b3, b4 = PW92_B
    s = np.sqrt(rs)
    Q = 2 * A * (b1 * s + b2 * rs + b3 * rs * s + b4 * rs * rs)
    Q1 = 2 * A * (0.5 * b1 / s + b2 + 1.5 * b3 * s + 2 * b4 * rs)
    Q2 = 2 * A * (-0.25 * b1 / (rs * s) + 0.75 * b3 / s + 2 * b4)
    L = np.log1p(1.0 / Q)
    D = Q + Q * Q
    L1 = -Q1 / D
    L2 = -Q2 / D + Q1 * Q1 * (1 + 2 * Q) / (D * D)
    g = -2 * A * (1 + a1 * rs)
    e = g * L
    e1 = -2 * A * a1 * L + g * L1
    e2 = -4 * A * a1 * L1 + g * L2
    return e, e1, e2


def exc_pw92(n):
    """eps_xc(n) per electron (Ha): Slater exchange + PW92 correlation."""
    n = np.asarray(n, dtype=np.float64)
    ex = -0.75 * (3.0 * n / math.pi) ** (1.0 / 3.0)
    ec, _, _ = _pw92_terms(rs_of(n))
    return ex + ec


def fxc_alda(n):
    """d^2 (n eps_xc) / dn^2."""
    n = np.asarray(n, dtype=np.float64)
    fx = -(1.0 / 3.0) * (3.0 / math.pi) ** (1.0 / 3.0) * n ** (-2.0 / 3.0)
    rs = rs_of(n)
    _, e1, e2 = _pw92_terms(rs)
    # rs(n) = (3/(4 pi n))^(1/3): d/dn = -(rs/3n) d/drs, which gives
    # d^2(n eps)/dn^2 = (rs^2 eps'' - 2 rs eps') / (9 n).
    fc = (rs * rs * e2 - 2.0 * rs * e1) / (9.0 * n)
    return fx + fc


def density_on_grid(st, grid):
    """n(r_j) on the real-space grid (bohr^-3)."""
    N = np.asarray(grid)
    Nr = int(np.prod(N))
    rho = np.zeros(tuple(N))
    for k in range(st.n_k):
        m = st.millers[k]
        span = m.max(axis=0) - m.min(axis=0) + 1
        if np.any(span > N):
            raise ValueError("real-space grid too small for the wavefunction sphere")
        idx = tuple(np.mod(m, N).T)
        for n_, f in enumerate(st.occ[k]):
            box = np.zeros(tuple(N), dtype=np.complex128)
            box[idx] = st.coef[k][n_]
            u = np.fft.ifftn(box) * Nr
            rho += f * (u.real ** 2 + u.imag ** 2)
    return rho * 2.0 / (st.n_k * st.omega)


def fxc_matrix(st, grid, basis):
    """K_xc[G, G'] = f_xc(G - G')."""
    N = np.asarray(grid)
    Nr = int(np.prod(N))
    fr = fxc_alda(density_on_grid(st, grid))
    fg = np.fft.fftn(fr) / Nr
    d = basis[:, None, :] - basis[None, :, :]
    d = np.mod(d, N)
    return fg[d[..., 0], d[..., 1], d[..., 2]]
