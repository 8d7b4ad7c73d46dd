"""Oracle pins for the Kubo-Greenwood conductivity of the states (Sec. A.3's
starting point): the momentum matrix elements against the effective-mass sum
rule, whose left side comes from eigenvalues at displaced k alone; the
large-frequency moment of sigma against the band curvatures; free electrons;
the reflection symmetry sigma(-w) = conj(sigma(w))."""
import math

import numpy as np
import pytest

import oracle
import workloads
from oracle import kubo_greenwood as kg
from oracle.lattice import gsphere
from oracle.states import hamiltonian


def _bands(w, kred, millers, B, omega):
    e, V = np.linalg.eigh(hamiltonian(kred, millers, B, w.potential, omega))
    return e, V.T


def _curvatures(w, kred, millers, B, omega, h):
    """d^2 e_n / dk_a^2 at fixed plane-wave set (sorted eigenvalues,
    Cartesian a): central differences at steps h and 2h combined by
    Richardson extrapolation, which cancels the h^2 error term."""
    e0, _ = _bands(w, kred, millers, B, omega)
    Binv = np.linalg.inv(B)
    out = []
    for a in range(3):
        c = []
        for step in (h, 2 * h):
            dk = step * Binv[a]  # reduced displacement along Cartesian a
            ep, _ = _bands(w, kred + dk, millers, B, omega)
            em, _ = _bands(w, kred - dk, millers, B, omega)
            c.append((ep - 2 * e0 + em) / step ** 2)
        out.append((4 * c[0] - c[1]) / 3)
    return e0, np.array(out)


def test_momentum_elements_satisfy_effective_mass_sum_rule():
    """For H(k) = 1/2|k+G|^2 + V on a fixed plane-wave set, d^2H/dk_a^2 = 1,
    so every non-degenerate band obeys
      d^2 e_n/dk_a^2 = 1 + 2 sum_{m != n} |<m|p_a|n>|^2 / (e_n - e_m),
    summed over the complete set of that basis.  A dropped k, a wrong sign of
    k + G, a conjugate on the wrong side or a missing factor fails it."""
    w = workloads.fcc_small()
    st = oracle.build_states(w)
    B, omega = st.B, st.omega
    kred = np.array([0.11, 0.23, 0.37])
    millers = gsphere(B, kred, 5.0)
    e, C = _bands(w, kred, millers, B, omega)
    P = kg.momentum_elements(kred, millers, B, C)
    _, curv = _curvatures(w, kred, millers, B, omega, 5e-4)
    nb = len(e)
    gaps = np.minimum(np.r_[np.inf, np.diff(e)], np.r_[np.diff(e), np.inf])
    checked = 0
    for n in range(min(nb, 30)):
        if gaps[n] < 0.05:
            continue
        de = e[n] - e
        de[n] = np.inf
        for a in range(3):
            rhs = 1.0 + 2.0 * np.sum(np.abs(P[a, :, n]) ** 2 / de)
            assert abs(curv[a, n] - rhs) < 2e-6 * max(1.0, abs(rhs)), (n, a, curv[a, n], rhs)
        checked += 1
    assert checked >= 10
    # diagonal elements are the group velocities de/dk (Hellmann-Feynman)
    Binv = np.linalg.inv(B)
    h = 1e-5
    for a in range(3):
        ep, _ = _bands(w, kred + h * Binv[a], millers, B, omega)
        em, _ = _bands(w, kred - h * Binv[a], millers, B, omega)
        v = (ep - em) / (2 * h)
        for n in range(min(nb, 30)):
            if gaps[n] >= 0.05:
                assert abs(P[a, n, n].real - v[n]) < 1e-6 and abs(P[a, n, n].imag) < 1e-12


def test_conductivity_moment_equals_band_curvature_sum():
    """At large w, -i w sigma(w) -> 2/(Omega N_k) sum_t W_t, and with every
    band of the basis kept and no screening the effective-mass sum rule turns
    that into 2/(Omega N_k) sum_k sum_n f_n (1 - (1/3) lap_k e_n): the
    conductivity's prefactor, its factor 2 for spin, the trace average and
    the weights against eigenvalue curvatures alone."""
    w = workloads.fcc_small().with_(kgrid=(2, 2, 2), n_bands=10 ** 6, f_trunc=2.0, ecut_wf=5.0)
    st = oracle.build_states(w)
    assert len(st.eps[0]) == len(st.millers[0])  # complete basis
    big = 1.0e6
    s = kg.kg_conductivity(st, np.array([big]), w.eta, 0.0)[0]
    moment = (-1j * big * s).real
    rhs = 0.0
    for k in range(st.n_k):
        e0, curv = _curvatures(w, st.kred[k], st.millers[k], st.B, st.omega, 5e-4)
        assert np.allclose(e0, st.eps[k], atol=1e-10)
        rhs += np.sum(st.occ[k] * (1.0 - curv.mean(axis=0)))
    rhs *= 2.0 / (st.omega * st.n_k)
    assert abs(rhs) > 1e-3
    assert abs(moment - rhs) < 5e-5 * abs(rhs), (moment, rhs)


def test_free_electrons_have_no_interband_conductivity():
    """Plane waves are momentum eigenstates: p is diagonal, so no transition
    between different bands carries weight."""
    w = workloads.feg_tiny()
    st = oracle.build_states(w)
    s = kg.kg_conductivity(st, np.linspace(0.0, 3.0, 31), w.eta, w.f_trans_thr)
    assert np.max(np.abs(s)) < 1e-14


def test_conductivity_reflection_symmetry_and_positive_real_part():
    w = workloads.h_tiny()
    st = oracle.build_states(w)
    om = np.linspace(0.05, 4.0, 40)
    sp = kg.kg_conductivity(st, om, w.eta, w.f_trans_thr)
    sm = kg.kg_conductivity(st, -om, w.eta, w.f_trans_thr)
    assert np.max(np.abs(sm - sp.conj())) < 1e-14 * np.max(np.abs(sp))
    assert np.all(sp.real > 0)
