"""Oracle response functions: transitions, pair densities, chi0, Dyson, S, F.

Test infrastructure only (see the package docstring).

Definitions (Hartree units, spin-unpolarised, cell volume Omega, N_k points):

  transitions  T(q) = {(k, n, m) : |f_nk - f_m,k+q| > thr}, with
               Delta_t = eps_m,k+q - eps_nk and df_t = f_nk - f_m,k+q.
  pair density rho_t(G) = <n k| exp(-i(q+G).r) |m k+q>
                        = sum_G1 c*_nk(G1) c_m,k'(G1 + G + G_s),  k+q = k'+G_s.
  chi0         chi0_GG'(q,w) = 2/(N_k Omega) sum_t df_t / (w - Delta_t + i eta)
                               rho_t(G) rho_t(G')*                 (Adler-Wiser)
  Dyson        chi = chi0 + chi0 K chi,  K_GG' = 4 pi/|q+G|^2 delta_GG' + f_xc(G-G')
  DSF          S(q,w) = -Im chi_00(q,w) / (pi n (1 - exp(-beta w)))   (Eq. 8)
  ITCF         F(q,tau) = int dw S(q,w) exp(-tau w) over the real line (Eq. 1)
               with S(q,-w) = exp(-beta w) S(q,w) (detailed balance, Sec. 2).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from .lattice import kq_map


@dataclass
class Transitions:
    k: np.ndarray        # (T,) k index
    kp: np.ndarray       # (T,) index of k' with k+q = k' + G_s
    n: np.ndarray        # (T,) band at k
    m: np.ndarray        # (T,) band at k'
    delta: np.ndarray    # (T,) eps_m(k') - eps_n(k)
    df: np.ndarray       # (T,) f_n(k) - f_m(k')

    def __len__(self):
        return len(self.k)


def transitions(st, qj, thr):
    """Screened transition list, k-major then n then m."""
    kp, _ = kq_map(st.kgrid, qj)
    ks, kps, ns, ms, dl, dfs = [], [], [], [], [], []
    for k in range(st.n_k):
        j = kp[k]
        df = st.occ[k][:, None] - st.occ[j][None, :]
        n, m = np.nonzero(np.abs(df) > thr)
        ks.append(np.full(len(n), k)); kps.append(np.full(len(n), j))
        ns.append(n); ms.append(m)
        dl.append(st.eps[j][m] - st.eps[k][n])
        dfs.append(df[n, m])
    cat = lambda x, dt: np.concatenate(x).astype(dt)
    return Transitions(cat(ks, np.int64), cat(kps, np.int64), cat(ns, np.int64),
                       cat(ms, np.int64), cat(dl, np.float64), cat(dfs, np.float64))


def _miller_key(m):
    m = np.asarray(m, dtype=np.int64) + 512
    return (m[..., 0] * 1024 + m[..., 1]) * 1024 + m[..., 2]


def pair_densities(st, tr, qj, basis):
    """P[t, G] = rho_t(G) by the direct sum over G1 (FP64)."""
    kp_of, gs = kq_map(st.kgrid, qj)
    P = np.zeros((len(tr), len(basis)), dtype=np.complex128)
    starts = np.searchsorted(tr.k, np.arange(st.n_k + 1))
    for k in range(st.n_k):
        lo, hi = starts[k], starts[k + 1]
        if lo == hi:
            continue
        j = kp_of[k]
        keys_j = _miller_key(st.millers[j])
        order = np.argsort(keys_j)
        sorted_keys = keys_j[order]
        Ck = st.coef[k].conj()                          # (nb_k, npw_k)
        Cj = st.coef[j]                                 # (nb_j, npw_j)
        for g, G in enumerate(basis):
            tgt = _miller_key(st.millers[k] + G + gs[k])
            pos = np.searchsorted(sorted_keys, tgt)
            pos = np.minimum(pos, len(sorted_keys) - 1)
            found = sorted_keys[pos] == tgt
            idx = order[pos]
            Cg = np.where(found[None, :], Cj[:, idx], 0.0)  # (nb_j, npw_k)
            M = Ck @ Cg.T                                    # (nb_k, nb_j)
            P[lo:hi, g] = M[tr.n[lo:hi], tr.m[lo:hi]]
    return P


def weights(tr, w, eta):
    """df_t / (w - Delta_t + i eta) for one frequency (FP64)."""
    return tr.df / (w - tr.delta + 1j * eta)


def chi0(tr, P, omegas, eta, n_k, omega_cell, chunk_bytes=1 << 28):
    """chi0[w, G, G'] = 2/(N_k Omega) sum_t w_t(w) P[t,G] conj(P[t,G']).

    The sum over t is one matrix product per chunk of transitions:
    W[w, t] @ X[t, (G,G')] with X[t] = rho_t rho_t^H.
    """
    pref = 2.0 / (n_k * omega_cell)
    nG = P.shape[1]
    om = np.asarray(omegas, dtype=np.float64)
    out = np.zeros((len(om), nG * nG), dtype=np.complex128)
    step = max(1, int(chunk_bytes // (16 * nG * nG)))
    for lo in range(0, len(tr), step):
        hi = min(lo + step, len(tr))
        Pt = P[lo:hi]
        X = (Pt[:, :, None] * Pt.conj()[:, None, :]).reshape(hi - lo, nG * nG)
        W = tr.df[None, lo:hi] / (om[:, None] - tr.delta[None, lo:hi] + 1j * eta)
        out += W @ X
    return pref * out.reshape(len(om), nG, nG)


def coulomb(B, qred, basis):
    """v(q+G) = 4 pi / |q+G|^2."""
    p = (np.asarray(qred) + basis) @ B
    return 4.0 * math.pi / np.einsum("ij,ij->i", p, p)


def dyson(chi0_w, K, iG0):
    """chi_00 for each frequency: solve (1 - chi0 K) x = chi0 e_00, take x_00."""
    nG = chi0_w.shape[1]
    I = np.eye(nG)
    out = np.empty(len(chi0_w), dtype=np.complex128)
    for i, c in enumerate(chi0_w):
        x = np.linalg.solve(I - c @ K, c[:, iG0])
        out[i] = x[iG0]
    return out


def dsf(chi_00, omegas, beta, n):
    """Fluctuation-dissipation theorem, Eq. (8), in the normalisation
    S = -Im chi / (pi n (1 - e^{-beta w})).

    Eq. (8) as printed carries no 1/pi; with it, F(q,0) is the static
    structure factor, -dF/dtau at 0 is q^2/2 (f-sum) and the ITCF area is
    -chi(q,0)/n (Sec. 2), which the printed form does not satisfy.
    At w = 0 exactly the w -> 0 limit is taken from the next grid point:
    S(0) = -Im chi(w1) / (pi n beta w1).
    """
    chi_00 = np.asarray(chi_00)
    omegas = np.asarray(omegas, dtype=np.float64)
    S = np.empty(len(omegas))
    for i, w in enumerate(omegas):
        if w != 0.0:
            S[i] = -chi_00[i].imag / (math.pi * n * (-math.expm1(-beta * w)))
        else:
            if i + 1 >= len(omegas) or omegas[i + 1] <= 0.0:
                raise ValueError("w = 0 needs a positive neighbour")
            w1 = omegas[i + 1]
            S[i] = -chi_00[i + 1].imag / (math.pi * n * beta * w1)
    return S


def trapezoid_weights(omegas):
    x = np.asarray(omegas, dtype=np.float64)
    c = np.zeros(len(x))
    h = np.diff(x)
    c[:-1] += 0.5 * h
    c[1:] += 0.5 * h
    return c


def itcf(S, omegas, beta, taus):
    """Eq. (1) on the w >= 0 grid, negative w by detailed balance:
    F(tau) = sum_j c_j S_j (exp(-tau w_j) + exp(-(beta - tau) w_j)),
    c_j the composite-trapezoid weights of the grid.
    """
    c = trapezoid_weights(omegas)
    w = np.asarray(omegas, dtype=np.float64)
    F = np.empty(len(taus))
    for i, t in enumerate(taus):
        F[i] = float(np.sum(c * S * (np.exp(-t * w) + np.exp(-(beta - t) * w))))
    return F
