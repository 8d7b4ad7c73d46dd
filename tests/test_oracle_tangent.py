"""Pins of the oracle's forward-mode tangents of F(q,tau): central finite
differences (h = 1e-5) of the oracle's forward pipeline, a different
computation from the tangent's matrix-level derivation.

The workload is the 4-proton hydrogen box with screening off (every pair
with f_n != f_m kept), so that the transition set cannot change inside the
finite-difference stencil."""
import numpy as np
import pytest

import workloads
from oracle import tangent


def _w():
    w = workloads.h_tiny()
    return w.with_(f_trans_thr=0.0, n_omega=40, qs=w.qs[:1],
                   temperatures=w.temperatures[:1], ecut_chi=w.ecut_chi[:1],
                   omega_max=w.omega_max[:1], n_tau=9)


H = 1e-5


def _fd(w, T, eta, v, dT, deta, dv):
    fp = tangent.itcf_value(w, 0, T + H * dT, eta + H * deta, v + H * dv)
    fm = tangent.itcf_value(w, 0, T - H * dT, eta - H * deta, v - H * dv)
    return (fp - fm) / (2 * H)


@pytest.mark.parametrize("direction", ["T", "eta", "v"])
def test_tangent_matches_central_differences(direction):
    w = _w()
    T, eta = w.temperatures[0], w.eta
    v = np.asarray(w.potential.shell_v)
    rng = np.random.default_rng(11)
    dT = 1.0 if direction == "T" else 0.0
    deta = 1.0 if direction == "eta" else 0.0
    dv = rng.standard_normal(len(v)) * np.abs(v) if direction == "v" else np.zeros(len(v))
    F, dF, _ = tangent.itcf_tangent(w, 0, T, eta, dT, deta, dv)
    F0 = tangent.itcf_value(w, 0, T, eta, v)
    np.testing.assert_allclose(F, F0, rtol=1e-12, atol=0)
    fd = _fd(w, T, eta, v, dT, deta, dv)
    err = np.max(np.abs(dF - fd)) / np.max(np.abs(fd))
    assert np.max(np.abs(fd)) > 1e-3 * np.max(np.abs(F))   # a real dependence
    assert err < 1e-6, err


def test_tangent_is_linear_in_the_direction():
    """dF(a d1 + b d2) = a dF(d1) + b dF(d2) (one shared base point)."""
    w = _w()
    T, eta = w.temperatures[0], w.eta
    v = np.asarray(w.potential.shell_v)
    d1 = (0.3, -0.2, np.array([0.01, 0.0, -0.02]))
    d2 = (-0.1, 0.5, np.array([0.0, 0.03, 0.01]))
    _, g1, _ = tangent.itcf_tangent(w, 0, T, eta, *d1)
    _, g2, _ = tangent.itcf_tangent(w, 0, T, eta, *d2)
    _, g3, _ = tangent.itcf_tangent(w, 0, T, eta, 2 * d1[0] - d2[0], 2 * d1[1] - d2[1],
                                    2 * d1[2] - d2[2])
    np.testing.assert_allclose(g3, 2 * g1 - g2, rtol=1e-9, atol=1e-12 * np.max(np.abs(g1)))


def _w_alda():
    return _w().with_(xc="alda", dens_grid=(12, 12, 12))


@pytest.mark.parametrize("direction", ["T", "v"])
def test_alda_tangent_matches_central_differences(direction):
    """With the ALDA kernel the density of the states moves with T (through
    the occupations) and with v (through orbitals and occupations), and K
    with it: the tangent's dK = [f_xc'(n) dn](G - G') against central
    differences of the forward pipeline, which rebuilds n and K."""
    w = _w_alda()
    T, eta = w.temperatures[0], w.eta
    v = np.asarray(w.potential.shell_v)
    rng = np.random.default_rng(13)
    dT = 1.0 if direction == "T" else 0.0
    dv = rng.standard_normal(len(v)) * np.abs(v) if direction == "v" else np.zeros(len(v))
    F, dF, _ = tangent.itcf_tangent(w, 0, T, eta, dT, 0.0, dv)
    F0 = tangent.itcf_value(w, 0, T, eta, v)
    np.testing.assert_allclose(F, F0, rtol=1e-12, atol=0)
    fd = _fd(w, T, eta, v, dT, 0.0, dv)
    err = np.max(np.abs(dF - fd)) / np.max(np.abs(fd))
    assert err < 1e-6, err
    # the kernel's share of the tangent is not negligible: the RPA tangent
    # along the same direction differs
    _, dF_rpa, _ = tangent.itcf_tangent(_w(), 0, T, eta, dT, 0.0, dv)
    assert np.max(np.abs(dF - dF_rpa)) > 1e-3 * np.max(np.abs(dF))
