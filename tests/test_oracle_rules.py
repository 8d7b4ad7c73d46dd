"""Oracle pins from sum rules, symmetries and brute force (P4-P10, P14, P15)."""
import math

import numpy as np
import pytest

import oracle
import workloads
from oracle import response
from oracle.lattice import kq_map, response_basis


def _qc(st, r):
    return r.qred @ st.B


def _fsum_transitions(st, r):
    n = r.density
    s = np.sum(r.tr.df * np.abs(r.P[:, r.iG0]) ** 2 * r.tr.delta)
    qc = _qc(st, r)
    return s / (n * st.n_k * st.omega) / (0.5 * qc @ qc)


def _cold_feg():
    return workloads.feg_tiny().with_(ecut_wf=5.0, temperatures=(0.05,) * 3,
                                      f_trans_thr=0.0)


@pytest.mark.parametrize("iq", [0, 1, 2])
def test_p4_fsum_on_transitions_free_electrons(iq):
    """Complete band set, occupations negligible at the sphere edge:
    1/(n N_k Omega) sum_t df |rho_t(0)|^2 Delta_t = q^2/2 to rounding."""
    w = _cold_feg()
    st = oracle.build_states(w)
    r = oracle.run_q(w, st, iq, omegas=[0.0, 0.1])
    assert abs(_fsum_transitions(st, r) - 1.0) < 1e-12


def test_p4_fsum_on_transitions_crystal():
    """EPM crystal, every band of the plane-wave basis kept: the f-sum holds
    up to the weight of occupied states that the q-shift pushes outside the
    k+q basis sphere."""
    w = workloads.fcc_small().with_(n_bands=0, ecut_wf=10.0)
    st = oracle.build_states(w)
    r = oracle.run_q(w, st, 0, omegas=[0.0, 0.1])
    assert abs(_fsum_transitions(st, r) - 1.0) < 1e-6


def _states_and_pm(w, iq):
    st = oracle.build_states(w).with_temperature(w.temperatures[iq])
    om = w.omega_grid(iq)[1:]
    pos = oracle.run_q(w, st, iq, omegas=om)
    neg = oracle.run_q(w, st, iq, omegas=-om)
    return st, om, pos, neg


@pytest.mark.parametrize("name,iq", [("fcc_small", 0), ("fcc_small", 1), ("h_tiny", 1)])
def test_p7_p8_detailed_balance_from_negative_frequencies(name, iq):
    """S(q,-w) computed from chi(q,-w) equals exp(-beta w) S(q,w), and the
    two-sided Laplace transform of the directly computed S is symmetric
    about beta/2 (Sec. 2, Eq. 1)."""
    w = workloads.get(name)
    st, om, pos, neg = _states_and_pm(w, iq)
    beta = pos.beta
    sp, sn = pos.S, neg.S
    assert np.max(np.abs(sn - np.exp(-beta * om) * sp)) <= 1e-10 * np.max(sp)
    # two-sided grid [-w_max, w_max] with the w = 0 limit from the w1 point
    s0 = -pos.chi00[0].imag / (math.pi * pos.density * beta * om[0])
    grid = np.concatenate([-om[::-1], [0.0], om])
    S = np.concatenate([sn[::-1], [s0], sp])
    c = response.trapezoid_weights(grid)
    taus = np.linspace(0, beta, 33)
    F = np.array([np.sum(c * S * np.exp(-t * grid)) for t in taus])
    assert np.max(np.abs(F - F[::-1])) <= 1e-10 * np.max(F)


@pytest.mark.parametrize("name,iq", [("fcc_small", 1), ("h_tiny", 0)])
def test_p9_hermitian_parts_and_reciprocity(name, iq):
    """chi0 = H_R + i H_A with H_A negative semi-definite for w > 0, and
    chi0(q,-w) = chi0(q,w)^H (time-reversal closure of the transition set)."""
    w = workloads.get(name)
    st, om, pos, neg = _states_and_pm(w, iq)
    scale = np.max(np.abs(pos.chi0))
    for i in range(0, len(om), 7):
        c = pos.chi0[i]
        HA = (c - c.conj().T) / 2j
        ev = np.linalg.eigvalsh(HA)
        assert ev.max() <= 1e-13 * scale
        assert np.max(np.abs(neg.chi0[i] - c.conj().T)) <= 1e-13 * scale


def test_p10_noninteracting_itcf_closed_form():
    """K = 0 and eta -> 0: F0(q,tau) = 2/(n N_k Omega) sum_t f_n (1 - f_m)
    |rho_t(0)|^2 exp(-tau Delta_t), against the chi0 -> S -> F pipeline."""
    w = workloads.feg_tiny()
    st = oracle.build_states(w)
    iq = 1
    eta = 5e-4
    qj = w.qs[iq]
    qred = np.asarray(qj) / np.asarray(w.kgrid)
    basis, iG0 = response_basis(st.B, qred, w.ecut_chi[iq])
    tr = response.transitions(st, qj, w.f_trans_thr)
    P = response.pair_densities(st, tr, qj, basis)[:, [iG0]]
    om = np.linspace(0.0, 4.0, 24001)
    c00 = np.concatenate([response.chi0(tr, P, om[i:i + 2000], eta, st.n_k, st.omega)[:, 0, 0]
                          for i in range(0, len(om), 2000)])
    n = w.n_electrons / st.omega
    beta = 1.0 / w.temperatures[iq]
    S = response.dsf(c00, om, beta, n)
    taus = np.linspace(0, beta, 9)
    F = response.itcf(S, om, beta, taus)
    fn = np.array([st.occ[k][i] for k, i in zip(tr.k, tr.n)])
    fm = np.array([st.occ[k][i] for k, i in zip(tr.kp, tr.m)])
    wgt = fn * (1 - fm) * np.abs(P[:, 0]) ** 2 * 2 / (n * st.n_k * st.omega)
    F0 = np.array([np.sum(wgt * np.exp(-t * tr.delta)) for t in taus])
    assert np.max(np.abs(F - F0) / F0) < 1e-2


def test_p5_p6_sum_rules_on_S():
    """f-sum on S and the static-response identity chi(q,0) = -n int F dtau."""
    w = _cold_feg().with_(eta=0.002, n_omega=3001, omega_max=(6.0,) * 3)
    st = oracle.build_states(w)
    r = oracle.run_q(w, st, 1)
    om, S, beta = r.omegas, r.S, r.beta
    c = response.trapezoid_weights(om)
    fsum = np.sum(c * om * (-np.expm1(-beta * om)) * S)
    qc = _qc(st, r)
    assert abs(fsum / (0.5 * qc @ qc) - 1) < 2e-2
    taus = np.linspace(0, beta, 801)
    F = response.itcf(S, om, beta, taus)
    area = np.sum(response.trapezoid_weights(taus) * F)
    chi_static = oracle.run_q(w, st, 1, omegas=[0.0, 1e-9]).chi00[0].real
    assert abs(-r.density * area / chi_static - 1) < 2e-2


def test_p15_gauge_and_permutation_invariance():
    w = workloads.fcc_small()
    st = oracle.build_states(w)
    rng = np.random.default_rng(7)
    r = oracle.run_q(w, st, 0, omegas=w.omega_grid(0)[::8])
    coef2 = [c * np.exp(2j * math.pi * rng.random(len(c)))[:, None] for c in st.coef]
    st2 = oracle.States(st.cell, st.B, st.omega, st.kgrid, st.kred, st.millers,
                        st.eps, coef2, st.occ, st.mu, st.T, st.n_electrons)
    r2 = oracle.run_q(w, st2, 0, omegas=r.omegas)
    scale = np.max(np.abs(r.chi0))
    assert np.max(np.abs(r2.chi0 - r.chi0)) <= 1e-12 * scale
    assert not np.allclose(r2.P, r.P)
    perm = rng.permutation(len(r.tr))
    tr = r.tr
    trp = response.Transitions(tr.k[perm], tr.kp[perm], tr.n[perm], tr.m[perm],
                               tr.delta[perm], tr.df[perm])
    c3 = response.chi0(trp, r.P[perm], r.omegas, w.eta, st.n_k, st.omega)
    assert np.max(np.abs(c3 - r.chi0)) <= 1e-12 * scale
