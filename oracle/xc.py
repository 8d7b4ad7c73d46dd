"""Oracle adiabatic LDA kernel f_xc = d^2(n eps_xc)/dn^2.

Test infrastructure only (see the package docstring).

The paper uses an adiabatic (static) GGA kernel (Sec. A.1).  The model here
is its local-density form: Slater exchange plus the Perdew-Wang 1992
parametrisation of the unpolarised correlation energy,
  eps_c(rs) = -2A (1 + a1 rs) ln[1 + 1/(2A (b1 rs^1/2 + b2 rs + b3 rs^3/2 + b4 rs^2))]
with A = 0.031091, a1 = 0.21370, b1..b4 = 7.5957, 3.5876, 1.6382, 0.49294
(Hartree; Phys. Rev. B 45, 13244 (1992), Table I, zeta = 0 column).

The second derivative is taken by evaluating n eps_xc(n) in hyper-dual
arithmetic, which yields it exactly (up to rounding) from the energy formula
itself.

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


class HyperDual:
    """x = a + b e1 + c e2 + d e1 e2 with e1^2 = e2^2 = 0 (hyper-dual numbers,
    Fike and Alonso, AIAA 2011-886): evaluating f at a + e1 + e2 gives f(a),
    f'(a), f'(a) and f''(a) in the four parts, exactly up to rounding (no
    step size).  Components are numpy arrays."""

    __slots__ = ("a", "b", "c", "d")

    def __init__(self, a, b=0.0, c=0.0, d=0.0):
        self.a, self.b, self.c, self.d = a, b, c, d

    @staticmethod
    def _lift(x):
        return x if isinstance(x, HyperDual) else HyperDual(x)

    def _chain(self, f, f1, f2):
        """g(self) for a scalar function g with g = f, g' = f1, g'' = f2 at a."""
        return HyperDual(f, f1 * self.b, f1 * self.c, f1 * self.d + f2 * self.b * self.c)

    def __add__(self, o):
        o = self._lift(o)
        return HyperDual(self.a + o.a, self.b + o.b, self.c + o.c, self.d + o.d)

    __radd__ = __add__

    def __neg__(self):
        return HyperDual(-self.a, -self.b, -self.c, -self.d)

    def __sub__(self, o):
        return self + (-self._lift(o))

    def __rsub__(self, o):
        return self._lift(o) - self

    def __mul__(self, o):
        o = self._lift(o)
        return HyperDual(self.a * o.a, self.a * o.b + self.b * o.a, self.a * o.c + self.c * o.a,
                         self.a * o.d + self.b * o.c + self.c * o.b + self.d * o.a)

    __rmul__ = __mul__

    def recip(self):
        a = self.a
        return self._chain(1.0 / a, -1.0 / a ** 2, 2.0 / a ** 3)

    def __truediv__(self, o):
        return self * self._lift(o).recip()

    def __rtruediv__(self, o):
        return self._lift(o) * self.recip()

    def __pow__(self, p):
        a = self.a
        return self._chain(a ** p, p * a ** (p - 1.0), p * (p - 1.0) * a ** (p - 2.0))

    def log1p(self):
        a = self.a
        return self._chain(np.log1p(a), 1.0 / (1.0 + a), -1.0 / (1.0 + a) ** 2)


def rs_of(n):
    return (3.0 / (4.0 * math.pi * np.asarray(n, dtype=np.float64))) ** (1.0 / 3.0)


def _ex(n):
    """Slater exchange energy per electron, -(3/4)(3 n / pi)^(1/3)."""
    return -0.75 * (3.0 / math.pi) ** (1.0 / 3.0) * n ** (1.0 / 3.0)


def _ec(n):
    """PW92 correlation energy per electron (unpolarised) at density n, with
    rs = (3 / (4 pi n))^(1/3) (works on floats, arrays and HyperDual)."""
    A, a1 = PW92_A, PW92_A1
    b1, b2, b3, b4 = PW92_B
    rs = (3.0 / (4.0 * math.pi)) ** (1.0 / 3.0) * n ** (-1.0 / 3.0)
    den = 2.0 * A * (b1 * rs ** 0.5 + b2 * rs + b3 * rs ** 1.5 + b4 * rs ** 2.0)
    inner = 1.0 / den
    log_term = inner.log1p() if isinstance(inner, HyperDual) else np.log1p(inner)
    return -2.0 * A * (1.0 + a1 * rs) * log_term


def ec_pw92_rs(rs):
    """PW92 correlation energy per electron as a function of rs (Ha)."""
    rs = np.asarray(rs, dtype=np.float64)
    return _ec(3.0 / (4.0 * math.pi * rs ** 3))


def exc_pw92(n):
    """eps_xc(n) per electron (Ha): Slater exchange + PW92 correlation."""
    n = np.asarray(n, dtype=np.float64)
    return _ex(n) + _ec(n)


def fxc_parts(n):
    """(f_x, f_c): the second derivatives d^2(n eps_x)/dn^2 and
    d^2(n eps_c)/dn^2, each read off n eps(n) evaluated at the hyper-dual
    point n + e1 + e2 (no chain rule through rs written by hand)."""
    n = np.asarray(n, dtype=np.float64)
    x = HyperDual(n, np.ones_like(n), np.ones_like(n), np.zeros_like(n))
    return (x * _ex(x)).d, (x * _ec(x)).d


def fxc_alda(n):
    """d^2 (n eps_xc) / dn^2."""
    fx, fc = fxc_parts(n)
    return fx + fc


def fxc_deriv_parts(n, h=1e-30):
    """(d f_x/dn, d f_c/dn), the third derivatives of n eps_x and n eps_c:
    the hyper-dual evaluation of fxc_parts at the complex point n (1 + i h),
    whose imaginary part over h n is the derivative up to O(h^2) with no
    cancellation (the complex-step derivative, Squire and Trapp, SIAM Rev.
    40, 110 (1998)); the second derivative stays exact in the hyper-dual
    parts."""
    n = np.asarray(n, dtype=np.float64)
    z = n * (1.0 + 1j * h)
    x = HyperDual(z, np.ones_like(z), np.ones_like(z), np.zeros_like(z))
    fx, fc = (x * _ex(x)).d, (x * _ec(x)).d
    return fx.imag / (h * n), fc.imag / (h * n)


def fxc_alda_deriv(n):
    """d f_xc / dn = d^3 (n eps_xc) / dn^3 (the ALDA kernel's response to
    the density, needed by its tangent)."""
    dx, dc = fxc_deriv_parts(n)
    return dx + dc


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


def kernel_from_real(fr, grid, basis):
    """M[G, G'] = g(G - G') for a real-space function fr on the grid, with
    g(G) = (1/N_r) sum_j fr(r_j) exp(-i G.r_j)."""
    N = np.asarray(grid)
    Nr = int(np.prod(N))
    fg = np.fft.fftn(fr) / Nr
    d = basis[:, None, :] - basis[None, :, :]
    d = np.mod(d, N)
    return fg[d[..., 0], d[..., 1], d[..., 2]]


def fxc_matrix(st, grid, basis):
    """K_xc[G, G'] = f_xc(G - G')."""
    return kernel_from_real(fxc_alda(density_on_grid(st, grid)), grid, basis)
