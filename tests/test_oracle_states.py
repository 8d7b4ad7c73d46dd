"""Oracle pins for the lattice, the model Hamiltonian and the occupations."""
import math

import numpy as np
import pytest
from scipy import integrate, special

import oracle
import workloads
from oracle import lindhard, states
from oracle.lattice import gsphere, kq_map, mp_kpoints, reciprocal


def test_reciprocal_and_mp_grid():
    w = workloads.fcc_c2()
    A = np.array(w.cell)
    B = reciprocal(A)
    assert np.allclose(A @ B.T, 2 * math.pi * np.eye(3), atol=1e-13)
    red, idx = mp_kpoints((4, 4, 4))
    keys = {tuple(np.round(r * 8).astype(int)) for r in red}
    assert all(tuple(-k for k in key) in keys for key in keys)      # k -> -k closed
    assert len(keys) == 64


@pytest.mark.parametrize("qj", [(0, 4, 4), (16, 0, 0), (3, -5, 17)])
def test_kq_map_is_exact(qj):
    N = (16, 16, 16)
    red, _ = mp_kpoints(N)
    kp, gs = kq_map(N, qj)
    lhs = red + np.asarray(qj) / np.asarray(N)
    rhs = red[kp] + gs
    assert np.max(np.abs(lhs - rhs)) < 1e-14
    assert np.all(np.abs(red[kp]) < 0.5)


def test_gsphere_is_complete():
    B = reciprocal(workloads.fcc_c2().cell)
    k = np.array([0.1, -0.2, 0.3])
    m = gsphere(B, k, 5.0)
    r = np.arange(-8, 9)
    allm = np.array(np.meshgrid(r, r, r, indexing="ij")).reshape(3, -1).T
    p = (k + allm) @ B
    ref = {tuple(x) for x, e in zip(allm, 0.5 * np.sum(p * p, 1)) if e <= 5.0}
    assert {tuple(x) for x in m} == ref


def test_mu_bisection_against_brentq():
    w = workloads.fcc_small()
    st = oracle.build_states(w)
    e = np.concatenate(st.eps)
    from scipy.optimize import brentq
    g = lambda mu: 2 / st.n_k * special.expit(-(e - mu) / st.T).sum() - w.n_electrons
    ref = brentq(g, e.min() - 1, e.max() + 1, xtol=1e-15, rtol=1e-15)
    assert abs(st.mu - ref) < 1e-13
    count = 2 / st.n_k * sum(o.sum() for o in st.occ)
    assert abs(count - w.n_electrons) < 1e-12


def test_fermi_function_is_overflow_safe():
    x = np.array([-1e4, -50, -1, 0, 1, 50, 1e4])
    f = states.fermi(x)
    assert np.all(np.isfinite(f))
    assert np.allclose(f, special.expit(-x), rtol=1e-15, atol=0)


def _gap_at(w, k_red, shell_v):
    A = np.array(w.cell)
    B = reciprocal(A)
    omega = abs(np.linalg.det(A))
    m = gsphere(B, k_red, 6.0)
    H = states.hamiltonian(k_red, m, B, w.potential, omega)
    return np.linalg.eigvalsh(H)


def test_nearly_free_electron_gap_is_two_v():
    """One Fourier component V_G of size 1e-3: at k = G/2 the two degenerate
    plane waves k and k - G split by 2|V_G| (first order; second order is
    O(V^2 / E))."""
    a = 7.6
    pot = workloads.Potential(shell_unit=2 * math.pi / a, shell_n2=(4,), shell_v=(1e-3,))
    w = workloads.fcc_c2().with_(potential=pot)
    B = reciprocal(w.cell)
    # G = (2pi/a)(2,0,0) = b2 + b3 ; k = G/2 in reduced coordinates
    e = _gap_at(w, np.array([0.0, 0.5, 0.5]), 1e-3)
    assert abs((e[1] - e[0]) - 2e-3) < 2e-5


def test_structure_factor_extinction():
    """Two identical ions at 0 and (a/2)(1,1,1) in a cubic cell: S(G) = 0 for
    odd h+k+l, so the zone-boundary gap at G = (2pi/a)(1,0,0) closes, while a
    one-ion cell with the same form factor opens it by 2|2 v|."""
    a = 6.0
    cell = ((a, 0, 0), (0, a, 0), (0, 0, a))
    base = workloads.feg_c1().with_(cell=cell)
    two = workloads.Potential(positions=((0, 0, 0), (a / 2, a / 2, a / 2)),
                              shell_unit=2 * math.pi / a, shell_n2=(1,), shell_v=(1e-3,))
    one = workloads.Potential(positions=((0, 0, 0),), shell_unit=2 * math.pi / a,
                              shell_n2=(1,), shell_v=(2e-3,))
    k = np.array([0.5, 0.0, 0.0])
    e2 = _gap_at(base.with_(potential=two), k, 1e-3)
    e1 = _gap_at(base.with_(potential=one), k, 2e-3)
    assert e2[1] - e2[0] < 1e-5
    assert abs((e1[1] - e1[0]) - 4e-3) < 1e-4


def test_gaussian_coulomb_form_factor_by_radial_quadrature():
    """v(G) = -4 pi Z e^{-sigma^2 G^2/2} / (Omega G^2) is the cell Fourier
    transform of -Z erf(r / (sqrt2 sigma)) / r (Coulomb part removed
    analytically, the short-range rest integrated numerically)."""
    w = workloads.h_tiny()
    pot = w.potential
    omega = w.cell[0][0] ** 3
    B = reciprocal(w.cell)
    for m in [(1, 0, 0), (2, 1, 0), (3, 2, 2)]:
        single = workloads.Potential(positions=((0.0, 0.0, 0.0),), gauss=True,
                                     sigma=pot.sigma, z_ion=1.0)
        vg = states.potential_fourier(single, B, omega, [m])[0].real
        G = np.linalg.norm(np.asarray(m) @ B)
        s = pot.sigma
        short = lambda r: special.erfc(r / (math.sqrt(2) * s)) * math.sin(G * r) / G * 4 * math.pi
        val, _ = integrate.quad(short, 0, 20 * s, limit=200, epsabs=1e-14)
        ref = (-4 * math.pi / G ** 2 + val) / omega
        assert abs(vg - ref) < 1e-10 * abs(ref)


def test_structure_factor_sign_convention():
    """V(G) = v(G) sum_I exp(-i G.R_I): shifting every ion by R multiplies
    V(G) by exp(-i G.R) (the Hamiltonian of the shifted crystal is the
    translate of the original)."""
    w = workloads.h_tiny()
    pot = w.potential
    B = reciprocal(w.cell)
    L = w.cell[0][0]
    shift = np.array([0.3, -0.7, 1.1])
    moved = workloads.Potential(positions=tuple(tuple(np.asarray(p) + shift) for p in pot.positions),
                                shell_unit=pot.shell_unit, shell_n2=pot.shell_n2,
                                shell_v=pot.shell_v, gauss=True, sigma=pot.sigma)
    m = np.array([[1, 0, 0], [1, 2, -1]])
    v0 = states.potential_fourier(pot, B, L ** 3, m)
    v1 = states.potential_fourier(moved, B, L ** 3, m)
    assert np.allclose(v1, v0 * np.exp(-1j * (m @ B) @ shift), rtol=1e-13, atol=0)


def test_band_truncation_check():
    w = workloads.h_tiny().with_(n_bands=20)
    with pytest.raises(ValueError):
        oracle.build_states(w)


def test_snap_band_count():
    e = np.array([0.0, 1.0, 1.0, 1.0, 2.0, 2.0 + 1e-9, 3.0])
    assert states.snap_band_count(e, 2) == 4
    assert states.snap_band_count(e, 5) == 6
    assert states.snap_band_count(e, 1) == 1
    assert states.snap_band_count(e, 0) == 7
