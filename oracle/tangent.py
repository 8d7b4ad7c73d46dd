"""Oracle forward-mode tangents of F(q,tau) with respect to the temperature
T, the broadening eta and the tabulated shell values v(G_s) of the local
potential.

Test infrastructure only (see the package docstring).

This is forward mode at the level of matrices and full eigensystems; the
library's adjoint is reverse mode at the level of transitions, so the two
are different algorithms.  For a direction (dT, deta, dv):

  Hamiltonian   dH_GG' = sum_s dv_s [G - G' on shell s] S(G - G'),
                S(G) = sum_I exp(-i G.R_I) the structure factor.
  eigenpairs    full diagonalisation of H(k) (all N_pw states):
                d eps_n = <n|dH|n>,
                d psi_n = sum_{m != n} psi_m <m|dH|n> / (eps_n - eps_m),
                pairs closer than the multiplet tolerance left out (F is
                invariant under rotations inside a kept multiplet).
  occupations   f = 1/(1 + e^x), x = (eps - mu)/T, N_e fixed:
                dx = (d eps - d mu)/T - (eps - mu) dT/T^2, df = -f(1-f) dx,
                d mu from sum_j f_j(1-f_j) dx_j = 0.
  transitions   d Delta_t = d eps_m(k') - d eps_n(k),  d df_t = df_n(k) - df_m(k')
                (the transition set of the base point is held fixed).
  pair dens.    rho is sesquilinear in (c_n, c_m):
                d rho = rho(dc_n, c_m) + rho(c_n, dc_m)
                      = [rho(c + dc) - rho(c - dc)] / 2  (polarisation).
  weights       w_t = df_t / D_t, D_t = w - Delta_t + i eta:
                dw_t = d df_t / D_t + df_t (d Delta_t - i d eta) / D_t^2.
  chi0          d chi0 = pref sum_t [dw_t rho rho^H + w_t (d rho rho^H + rho d rho^H)].
  kernel        RPA: K = v(q + G) delta_GG' has no tangent.  ALDA: K adds
                f_xc(n)(G - G') with n the density of the states on the
                real-space grid; n is linear in f and sesquilinear in c, so
                dn = n(f = df) + [n(c + dc) - n(c - dc)] / 2 at fixed f,
                and dK_xc is the same transform of f_xc'(n) dn.
  Dyson         chi = A^{-1} chi0, A = 1 - chi0 K:
                d chi = A^{-1} [d chi0 (1 + K chi) + chi0 dK chi].
  DSF           S = -Im chi_00 g(beta, w), beta = 1/T (w = 0 from the next
                point, as in the forward path).
  ITCF          F(tau_j) = sum_i c_i S_i (e^{-tau_j w_i} + e^{-(beta - tau_j) w_i})
                with tau_j = x_j beta: the tau grid is a fixed fraction of beta.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

from .lattice import reciprocal, volume, mp_kpoints, gsphere, response_basis
from .states import (DEGEN_TOL, States, fermi, find_mu, hamiltonian,
                     potential_fourier, snap_band_count)
from .response import pair_densities, transitions, trapezoid_weights
from .xc import density_on_grid, fxc_alda, fxc_alda_deriv, kernel_from_real


def with_shell_values(w, v):
    """Workload w with the tabulated shell values replaced by v."""
    pot = dataclasses.replace(w.potential, shell_v=tuple(float(x) for x in v))
    return w.with_(potential=pot)


def shell_matrix(pot, B, omega, millers, s):
    """dH/dv_s on a plane-wave basis: [G - G' on shell s] S(G - G')."""
    unit = dataclasses.replace(pot, shell_v=tuple(1.0 if j == s else 0.0
                                                  for j in range(len(pot.shell_v))),
                               gauss=False)
    d = millers[:, None, :] - millers[None, :, :]
    return potential_fourier(unit, B, omega, d.reshape(-1, 3)).reshape(len(millers), -1)


def states_and_tangents(w, T, dT, dv):
    """Kept eigenpairs, occupations and their tangents along (dT, dv)."""
    cell = np.asarray(w.cell, dtype=np.float64)
    B = reciprocal(cell)
    omega = volume(cell)
    kred, _ = mp_kpoints(w.kgrid)
    millers, eps, coef, deps, dcoef = [], [], [], [], []
    for k in kred:
        m = gsphere(B, k, w.ecut_wf)
        H = hamiltonian(k, m, B, w.potential, omega)
        e, V = np.linalg.eigh(H)
        nb = snap_band_count(e, w.n_bands)
        dH = np.zeros_like(H)
        for s, d in enumerate(dv):
            if d != 0.0:
                dH += d * shell_matrix(w.potential, B, omega, m, s)
        Hm = V.conj().T @ dH @ V[:, :nb]                    # <m|dH|n>, all m
        gap = e[:nb][None, :] - e[:, None]                   # eps_n - eps_m
        inv = np.where(np.abs(gap) > DEGEN_TOL, 1.0 / np.where(gap == 0, 1.0, gap), 0.0)
        millers.append(m)
        eps.append(e[:nb].copy())
        coef.append(np.ascontiguousarray(V[:, :nb].T))
        deps.append(np.real(np.diag(Hm[:nb, :nb])).copy())
        dcoef.append(np.ascontiguousarray((V @ (Hm * inv)).T))
    n_k = len(kred)
    mu = find_mu(eps, T, w.n_electrons, n_k)
    occ = [fermi((e - mu) / T) for e in eps]
    wgt = [o * (1 - o) for o in occ]
    # sum_j wgt_j [(d eps_j - d mu)/T - (eps_j - mu) dT/T^2] = 0
    sw = sum(float(np.sum(x)) for x in wgt)
    dmu = (sum(float(np.sum(x * de)) for x, de in zip(wgt, deps)) -
           dT / T * sum(float(np.sum(x * (e - mu))) for x, e in zip(wgt, eps))) / sw
    docc = [-x * ((de - dmu) / T - (e - mu) * dT / T ** 2)
            for x, de, e in zip(wgt, deps, eps)]
    st = States(cell, B, omega, tuple(w.kgrid), kred, millers, eps, coef, occ,
                mu, T, w.n_electrons)
    return st, deps, dcoef, docc


def _with_coef(st, coef):
    return dataclasses.replace(st, coef=coef)


def itcf_tangent(w, iq, T, eta, dT=0.0, deta=0.0, dv=None, omegas=None):
    """F(q_iq, tau) and its directional derivative along (dT, deta, dv).

    States are built at T with the workload's shell values; tau runs over
    the workload's grid scaled to beta = 1/T.  RPA or ALDA kernel.
    Returns (F, dF, taus).
    """
    if w.xc not in ("rpa", "alda"):
        raise ValueError(f"no tangent for the kernel {w.xc!r}")
    dv = np.zeros(len(w.potential.shell_v)) if dv is None else np.asarray(dv, float)
    st, deps, dcoef, docc = states_and_tangents(w, T, dT, dv)
    qj = tuple(w.qs[iq])
    beta = 1.0 / T
    dbeta = -dT / T ** 2
    qred = np.asarray(qj, dtype=np.float64) / np.asarray(w.kgrid)
    basis, iG0 = response_basis(st.B, qred, w.ecut_chi[iq])
    tr = transitions(st, qj, w.f_trans_thr)
    P = pair_densities(st, tr, qj, basis)
    plus = [c + d for c, d in zip(st.coef, dcoef)]
    minus = [c - d for c, d in zip(st.coef, dcoef)]
    dP = 0.5 * (pair_densities(_with_coef(st, plus), tr, qj, basis) -
                pair_densities(_with_coef(st, minus), tr, qj, basis))
    d_delta = np.array([deps[kp][m] - deps[k][n]
                        for k, n, kp, m in zip(tr.k, tr.n, tr.kp, tr.m)])
    d_df = np.array([docc[k][n] - docc[kp][m]
                     for k, n, kp, m in zip(tr.k, tr.n, tr.kp, tr.m)])
    om = w.omega_grid(iq) if omegas is None else np.asarray(omegas, dtype=np.float64)
    x = w.tau_grid(iq) / w.tau_grid(iq)[-1] * (0.5 if w.tau_half else 1.0)
    taus = x * beta
    pref = 2.0 / (st.n_k * st.omega)
    p = (qred + basis) @ st.B
    K = np.diag(4 * math.pi / np.einsum("ij,ij->i", p, p)).astype(np.complex128)
    dK = np.zeros_like(K)
    if w.xc == "alda":
        grid = w.dens_grid
        nr = density_on_grid(st, grid)
        dn = (density_on_grid(dataclasses.replace(st, occ=docc), grid) +
              0.5 * (density_on_grid(_with_coef(st, plus), grid) -
                     density_on_grid(_with_coef(st, minus), grid)))
        K = K + kernel_from_real(fxc_alda(nr), grid, basis)
        dK = kernel_from_real(fxc_alda_deriv(nr) * dn, grid, basis)
    I = np.eye(len(basis))
    n = w.n_electrons / st.omega
    chi00 = np.empty(len(om), complex)
    dchi00 = np.empty(len(om), complex)
    Pc, dPc = P.conj(), dP.conj()
    for i, wv in enumerate(om):
        D = wv - tr.delta + 1j * eta
        wt = tr.df / D
        dwt = d_df / D + tr.df * (d_delta - 1j * deta) / D ** 2
        c0 = pref * ((P * wt[:, None]).T @ Pc)
        dc0 = pref * ((P * dwt[:, None]).T @ Pc +
                      (dP * wt[:, None]).T @ Pc + (P * wt[:, None]).T @ dPc)
        A = I - c0 @ K
        chi = np.linalg.solve(A, c0)
        chi00[i] = chi[iG0, iG0]
        dchi00[i] = np.linalg.solve(A, dc0 @ (I + K @ chi) + c0 @ dK @ chi)[iG0, iG0]
    S = np.empty(len(om))
    dS = np.empty(len(om))
    for i, wv in enumerate(om):
        j, wg = (i, wv) if wv != 0.0 else (i + 1, om[i + 1])
        if wv != 0.0:
            e = math.exp(-beta * wv)
            g = 1.0 / (math.pi * n * (1 - e))
            dg = -wv * e / (math.pi * n * (1 - e) ** 2) * dbeta
        else:
            g = 1.0 / (math.pi * n * beta * wg)
            dg = -g / beta * dbeta
        S[i] = -chi00[j].imag * g
        dS[i] = -dchi00[j].imag * g - chi00[j].imag * dg
    c = trapezoid_weights(om)
    F = np.empty(len(taus))
    dF = np.empty(len(taus))
    for j, (xj, t) in enumerate(zip(x, taus)):
        k1 = np.exp(-t * om)
        k2 = np.exp(-(beta - t) * om)
        F[j] = np.sum(c * S * (k1 + k2))
        dk = (-xj * om * k1 - (1 - xj) * om * k2) * dbeta
        dF[j] = np.sum(c * dS * (k1 + k2)) + np.sum(c * S * dk)
    return F, dF, taus


def itcf_value(w, iq, T, eta, v=None, omegas=None):
    """F(q_iq, tau) from the oracle's forward pipeline at (T, eta, v), tau
    on the workload's grid scaled to beta = 1/T (used for finite
    differences of the forward path)."""
    from .states import build_states
    from .pipeline import run_q
    ww = w if v is None else with_shell_values(w, v)
    ww = ww.with_(temperatures=tuple(T for _ in ww.temperatures), eta=eta)
    st = build_states(ww, T=T, check_trunc=False)
    return run_q(ww, st, iq, omegas=omegas, keep=False).F
