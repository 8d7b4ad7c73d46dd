"""Pins of the oracle's eta-convergence metrics (Sec. 2, Eq. 2): closed-form
integrals within the trapezoid error bound, the half-grid symmetry, the
reference-eta rule on constructed tables, and the static-response identity
chi(q, 0) = -n int_0^beta F dtau on a cold free-electron gas."""
import math

import numpy as np
import pytest

import oracle
import workloads
from oracle import eta as oeta
from oracle import response


def test_metrics_of_a_cosh_itcf():
    """F = cosh(a (tau - beta/2)) has F(beta/2) = 1, F(0) = cosh(a beta/2) and
    int_0^beta F = 2 sinh(a beta/2) / a; the trapezoid on 65 points must be
    inside its error bound beta h^2 max|F''| / 12."""
    beta, a, n = 3.0, 1.7, 0.05
    taus = np.linspace(0.0, beta, 65)
    F = np.cosh(a * (taus - beta / 2))
    m = oeta.itcf_metrics(F, taus, beta, n)
    exact = 2 * math.sinh(a * beta / 2) / a
    h = taus[1] - taus[0]
    bound = beta * h * h * a * a * math.cosh(a * beta / 2) / 12
    assert m[0] == pytest.approx(1.0, abs=1e-15)
    assert abs(m[1] - exact) <= bound and abs(m[1] - exact) > 0.1 * bound
    assert m[2] == pytest.approx(1.0 - math.cosh(a * beta / 2), rel=1e-15)
    assert m[3] == pytest.approx(m[1] - beta * math.cosh(a * beta / 2), rel=1e-14)
    assert m[4] == pytest.approx(-n * m[1], rel=1e-15)


def test_half_grid_equals_full_grid():
    beta = 2.5
    full = np.linspace(0.0, beta, 81)
    half = full[:41]
    F = 0.3 + np.cosh(0.9 * (full - beta / 2)) ** 2
    mf = oeta.itcf_metrics(F, full, beta, 0.1)
    mh = oeta.itcf_metrics(F[:41], half, beta, 0.1)
    assert np.max(np.abs(mf - mh) / np.abs(mf)) < 1e-14
    with pytest.raises(ValueError):
        oeta.itcf_metrics(F[:50], full[:50], beta, 0.1)


def test_reference_eta_rule():
    etas = [0.1, 0.2, 0.4, 0.8]
    base = np.array([0.5, 1.0, -0.2, -0.7, 0.3])
    m = np.tile(base, (4, 1))
    assert oeta.eta_reference(m, etas, 1e-2) == 3
    m2 = m.copy()
    m2[2, 2] *= 1.02                     # eta 0.4 leaves the 1 % band
    assert oeta.eta_reference(m2, etas, 1e-2) == 1
    assert oeta.eta_reference(m2, etas, 3e-2) == 3
    m3 = m.copy()
    m3[1, 3] *= 0.98
    assert oeta.eta_reference(m3, etas, 1e-2) == 0
    m4 = m.copy()
    m4[3, 0] *= 5.0                      # unshifted metrics do not decide
    assert oeta.eta_reference(m4, etas, 1e-2) == 3


def test_area_metric_is_the_static_response():
    """chi(q) = -n int_0^beta F dtau (Sec. 2) against the static chi_00(q, 0)
    from the Dyson solve at omega = 0 on a cold free-electron gas."""
    w = workloads.feg_tiny().with_(ecut_wf=5.0, temperatures=(0.05,) * 3, f_trans_thr=0.0,
                                   eta=0.002, n_omega=3001, omega_max=(6.0,) * 3)
    st = oracle.build_states(w)
    r = oracle.run_q(w, st, 1)
    taus = np.linspace(0.0, r.beta, 801)
    F = response.itcf(r.S, r.omegas, r.beta, taus)
    m = oeta.itcf_metrics(F, taus, r.beta, r.density)
    chi_static = oracle.run_q(w, st, 1, omegas=[0.0, 1e-9]).chi00[0].real
    assert abs(m[4] / chi_static - 1) < 2e-2
