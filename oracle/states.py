"""Oracle Kohn-Sham states for a local (non-self-consistent) model potential.

Test infrastructure only (see the package docstring).

Plane-wave Hamiltonian H_GG'(k) = 1/2 |k+G|^2 delta_GG' + V(G - G') on the
sphere 1/2 |k+G|^2 <= E_wf, dense Hermitian eigensolve, Fermi-Dirac
occupations at temperature T with the chemical potential fixed by the
electron count (2/N_k) sum_kn f_nk = N_e (spin-unpolarised).  The paper's
states come from self-consistent DFT (Sec. A.1); the model here is the
non-self-consistent local-potential reading of the configurations.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List

import numpy as np

from .lattice import reciprocal, volume, mp_kpoints, gsphere

# Eigenvalues closer than this (Ha) are one multiplet; the kept band count is
# moved up to the end of a multiplet so that the kept subspace is unique.
DEGEN_TOL = 1e-6


def potential_fourier(pot, B, omega, m):
    """V(G) for Miller triples m (N,3): v(|G|) * sum_I exp(-i G.R_I), V(0)=0."""
    m = np.atleast_2d(np.asarray(m))
    G = m @ np.asarray(B)
    g2 = np.einsum("ij,ij->i", G, G)
    v = np.zeros(len(m), dtype=np.float64)
    matched = np.zeros(len(m), dtype=bool)
    for n2, val in zip(pot.shell_n2, pot.shell_v):
        s2 = pot.shell_unit ** 2 * n2
        hit = np.abs(g2 - s2) <= 1e-9 * s2
        v[hit] = val
        matched |= hit
    if pot.gauss:
        free = (~matched) & (g2 > 0)
        v[free] = (-4.0 * math.pi * pot.z_ion *
                   np.exp(-0.5 * pot.sigma ** 2 * g2[free]) / (omega * g2[free]))
    v[g2 == 0] = 0.0
    R = np.asarray(pot.positions, dtype=np.float64)
    sfac = np.exp(-1j * (G @ R.T)).sum(axis=1)
    return v * sfac


def hamiltonian(kred, millers, B, pot, omega):
    """Dense H(k) on the given plane-wave basis."""
    p = (np.asarray(kred) + millers) @ B
    H = np.zeros((len(millers), len(millers)), dtype=np.complex128)
    if not pot.is_free:
        d = millers[:, None, :] - millers[None, :, :]
        H = potential_fourier(pot, B, omega, d.reshape(-1, 3)).reshape(H.shape)
    H[np.diag_indices_from(H)] += 0.5 * np.einsum("ij,ij->i", p, p)
    return H


def fermi(x):
    """1 / (1 + exp(x)), evaluated without overflow."""
    x = np.asarray(x, dtype=np.float64)
    out = np.empty_like(x)
    pos = x > 0
    e = np.exp(-x[pos])
    out[pos] = e / (1.0 + e)
    out[~pos] = 1.0 / (1.0 + np.exp(x[~pos]))
    return out


def electron_count(eps_all, mu, T, n_k):
    return 2.0 / n_k * float(np.sum(fermi((eps_all - mu) / T)))


def find_mu(eps_list, T, n_electrons, n_k):
    """Chemical potential by bisection on (2/N_k) sum f = N_e.

    Bisection runs until the bracket cannot shrink in FP64.
    """
    e = np.concatenate([np.asarray(x) for x in eps_list])
    if 2.0 * len(e) / n_k <= n_electrons:
        raise ValueError("too few bands for the electron count")
    lo, hi = float(e.min()) - 50.0 * T, float(e.max()) + 50.0 * T
    for _ in range(2000):
        mid = 0.5 * (lo + hi)
        if mid <= lo or mid >= hi:
            break
        if electron_count(e, mid, T, n_k) < n_electrons:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def snap_band_count(eps, n_bands):
    """Smallest count >= n_bands that does not split a multiplet (0 = all)."""
    n = len(eps)
    if n_bands <= 0 or n_bands >= n:
        return n
    nb = n_bands
    while nb < n and eps[nb] - eps[nb - 1] < DEGEN_TOL:
        nb += 1
    return nb


@dataclass
class States:
    cell: np.ndarray
    B: np.ndarray
    omega: float
    kgrid: tuple
    kred: np.ndarray                 # (N_k, 3)
    millers: List[np.ndarray]        # per k: (N_pw_k, 3)
    eps: List[np.ndarray]            # per k: (nb_k,)
    coef: List[np.ndarray]           # per k: (nb_k, N_pw_k), row n = band n
    occ: List[np.ndarray]            # per k: (nb_k,)
    mu: float
    T: float
    n_electrons: float

    @property
    def n_k(self):
        return len(self.kred)

    def with_temperature(self, T):
        """Same orbitals, occupations and mu at another temperature."""
        mu = find_mu(self.eps, T, self.n_electrons, self.n_k)
        occ = [fermi((e - mu) / T) for e in self.eps]
        return States(self.cell, self.B, self.omega, self.kgrid, self.kred,
                      self.millers, self.eps, self.coef, occ, mu, T,
                      self.n_electrons)


def build_states(w, T=None, check_trunc=True):
    """Eigenstates and occupations for workload ``w`` at temperature T."""
    T = w.temperatures[0] if T is None else T
    cell = np.asarray(w.cell, dtype=np.float64)
    B = reciprocal(cell)
    omega = volume(cell)
    kred, _ = mp_kpoints(w.kgrid)
    millers, eps, coef = [], [], []
    for k in kred:
        m = gsphere(B, k, w.ecut_wf)
        H = hamiltonian(k, m, B, w.potential, omega)
        e, V = np.linalg.eigh(H)
        nb = snap_band_count(e, w.n_bands)
        millers.append(m)
        eps.append(e[:nb].copy())
        coef.append(np.ascontiguousarray(V[:, :nb].T))
    st = States(cell, B, omega, tuple(w.kgrid), kred, millers, eps, coef,
                [], 0.0, T, w.n_electrons)
    st = st.with_temperature(T)
    if check_trunc:
        top = max(float(o[-1]) for o in st.occ)
        if top >= w.f_trunc:
            raise ValueError(f"band set too small: top occupation {top:.3e}")
    return st
