"""Pins of the Kubo-Greenwood route oracle (Sec. A.3): the loss-function
sum rule of a Drude conductivity, the static limit of S* in closed form,
positivity for a passive conductivity, and the way back from S* to sigma
through the (separately pinned) dielectric oracle at q^2 = 4 pi."""
import numpy as np

import workloads
from oracle import kubo_greenwood as kg


def _drude(w, sigma0, tau):
    return sigma0 / (1.0 - 1j * w * tau)


def test_loss_sum_rule_drude():
    # int_0^inf w Im(1/eps) dw = -(pi/2) w_p^2 with w_p^2 = 4 pi sigma0 / tau
    sigma0, tau = 1.0 / (4 * np.pi) * 5.0, 5.0  # w_p = 1
    w = np.concatenate([np.linspace(1e-6, 20.0, 200001)[:-1], np.geomspace(20.0, 4000.0, 20001)])
    im = kg.chi_star(_drude(w, sigma0, tau), w).imag
    integral = np.trapezoid(w * im, w)
    assert abs(integral / (-0.5 * np.pi) - 1.0) <= 1e-3


def test_static_limit_closed_form():
    sigma0, tau, beta, n = 0.05, 8.0, 30.0, 0.018
    w = np.array([0.0, 1e-5, 2e-5])
    S = kg.kg_dsf(_drude(w, sigma0, tau), w, beta, n)
    assert abs(S[0] * 4 * np.pi ** 2 * sigma0 * n * beta - 1.0) <= 1e-8


def test_positive_for_passive_conductivity():
    w, sig = workloads.kg_conductivity()
    assert np.all(sig.real[1:] > 0)
    S = kg.kg_dsf(sig, w, 30.0, 0.018)
    assert np.all(S > 0)


def test_round_trip_through_dielectric():
    """S* of a Drude conductivity, taken back through Im chi* (FDT), Re chi*
    (Kramers-Kronig), eps^{-1} = 1 + chi* and sigma = i w (1 - eps)/(4 pi),
    returns the conductivity (to the Kramers-Kronig truncation at w_max)."""
    from oracle.dielectric import dielectric
    sigma0, tau, beta, n = 0.4, 5.0, 30.0, 0.018
    w = np.linspace(0.0, 40.0, 4001)
    sig = _drude(w, sigma0, tau)
    S = kg.kg_dsf(sig, w, beta, n)
    chi, eps_inv, sig_back = dielectric(S, w, beta, n, kg.KG_Q2)
    sel = (w >= 0.2) & (w <= 3.0)
    assert np.max(np.abs(sig_back[sel] - sig[sel]) / np.abs(sig[sel])) <= 1e-2
    # eps^{-1} = 1 + chi* as printed
    assert np.allclose(eps_inv, 1.0 + chi, atol=1e-14)
