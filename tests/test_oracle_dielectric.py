"""Pins of the oracle's dielectric properties from S (Sec. 3, A.2): the
Kramers-Kronig step exact for a piecewise-linear Im chi (triangle, closed
form), a Lorentz oscillator within its discretisation error, the static limit
against the Dyson solve at w = 0 on a cold free-electron gas, and Eq. A-1/A-2
algebra."""
import math

import numpy as np

import oracle
import workloads
from oracle import dielectric as od


def _triangle_re(w):
    """(1/pi) P int_0^2 f(x) [1/(x - w) + 1/(x + w)] dx for the triangle
    f = x on [0, 1], 2 - x on [1, 2], from the antiderivatives
    x + c ln|x - c| and (2 - c) ln|x - c| - x (log(0) terms cancel)."""
    def lg(x, c):
        return math.log(abs(x - c)) if x != c else 0.0

    def pv(c):
        first = (1 + c * lg(1, c)) - (0 + c * lg(0, c))
        second = ((2 - c) * lg(2, c) - 2) - ((2 - c) * lg(1, c) - 1)
        return first + second
    return (pv(w) + pv(-w)) / math.pi


def test_kk_exact_for_piecewise_linear():
    x = np.linspace(0.0, 3.0, 31)
    f = np.where(x <= 1, x, np.maximum(2 - x, 0.0))
    got = od.kramers_kronig_re(f, x)
    ref = np.array([_triangle_re(w) for w in x])
    assert np.max(np.abs(got - ref)) < 1e-13


def test_kk_of_a_lorentz_oscillator():
    """chi = A / (w0^2 - w^2 - i g w) is causal with Im chi odd."""
    A, w0, g = -1.0, 1.0, 0.3
    x = np.linspace(0.0, 400.0, 40001)
    chi = A / (w0 ** 2 - x ** 2 - 1j * g * x)
    at = np.flatnonzero(x <= 3.0)[::10]
    got = od.kramers_kronig_re(chi.imag, x, at=at)
    assert np.max(np.abs(got - chi.real[at])) < 1e-3 * np.max(np.abs(chi.real))


def test_static_limit_matches_the_dyson_solve():
    w = workloads.feg_tiny().with_(ecut_wf=5.0, temperatures=(0.05,) * 3, f_trans_thr=0.0,
                                   eta=0.002, n_omega=3001, omega_max=(6.0,) * 3)
    st = oracle.build_states(w)
    r = oracle.run_q(w, st, 1)
    qc = (np.asarray(r.qred) @ st.B)
    chi, eps_inv, sigma = od.dielectric(r.S, r.omegas, r.beta, r.density, float(qc @ qc))
    chi_static = oracle.run_q(w, st, 1, omegas=[0.0, 1e-9]).chi00[0].real
    assert abs(chi[0].real / chi_static - 1) < 2e-2
    # Eq. A-1 / A-2 consistency: eps = 1 / eps^{-1} and Re sigma = w Im eps / (4 pi)
    eps = 1 / eps_inv
    assert np.allclose(sigma.real, r.omegas * eps.imag / (4 * math.pi), rtol=1e-13, atol=1e-300)
    assert np.allclose(sigma.imag, -r.omegas * (eps.real - 1) / (4 * math.pi), rtol=1e-13,
                       atol=1e-300)
