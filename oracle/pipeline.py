"""Oracle driver: one workload through states -> chi0 -> Dyson -> S -> F.

Test infrastructure only (see the package docstring).
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Optional

import numpy as np

from .lattice import response_basis
from .response import (transitions, pair_densities, chi0 as chi0_fn, coulomb,
                       dyson, dsf, itcf, Transitions)
from .states import States, build_states
from .xc import fxc_matrix


@dataclass
class QResult:
    qj: tuple
    qred: np.ndarray
    basis: np.ndarray
    iG0: int
    tr: Transitions
    P: np.ndarray
    omegas: np.ndarray
    chi0: np.ndarray           # (N_w, N_G, N_G)
    K: np.ndarray              # (N_G, N_G)
    chi00: np.ndarray          # (N_w,)
    S: np.ndarray              # (N_w,)
    taus: np.ndarray
    F: np.ndarray              # (N_tau,)
    beta: float
    density: float


def run_q(w, st: States, iq: int, omegas=None, keep=True) -> QResult:
    """Full path for q index iq of workload w on states st (at the q's T)."""
    qj = tuple(w.qs[iq])
    T = w.temperatures[iq]
    if abs(st.T - T) > 0.0:
        st = st.with_temperature(T)
    beta = 1.0 / T
    qred = np.asarray(qj, dtype=np.float64) / np.asarray(w.kgrid)
    basis, iG0 = response_basis(st.B, qred, w.ecut_chi[iq])
    tr = transitions(st, qj, w.f_trans_thr)
    P = pair_densities(st, tr, qj, basis)
    om = w.omega_grid(iq) if omegas is None else np.asarray(omegas)
    c0 = chi0_fn(tr, P, om, w.eta, st.n_k, st.omega)
    K = np.diag(coulomb(st.B, qred, basis)).astype(np.complex128)
    if w.xc == "alda":
        K = K + fxc_matrix(st, w.dens_grid, basis)
    elif w.xc != "rpa":
        raise ValueError(w.xc)
    c00 = dyson(c0, K, iG0)
    n = w.n_electrons / st.omega
    S = dsf(c00, om, beta, n)
    taus = w.tau_grid(iq)
    F = itcf(S, om, beta, taus)
    return QResult(qj, qred, basis, iG0, tr, P if keep else None, om,
                   c0 if keep else None, K, c00, S, taus, F, beta, n)


def run_workload(w, states: Optional[States] = None):
    st = build_states(w, T=w.temperatures[0]) if states is None else states
    return st, [run_q(w, st, iq) for iq in range(len(w.qs))]
