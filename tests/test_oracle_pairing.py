"""Time-reversal pairing of transitions, checked on the oracle's plain sum.

For a real local potential without spin-orbit coupling the orbitals at -k
are the complex conjugates of those at k (up to a gauge), and a
Monkhorst-Pack grid is closed under k -> -k.  The transition (k, n -> k+q, m)
and its partner (-k-q, m -> -k, n) then carry the same rho rho^H (summed over
degenerate multiplets), opposite Delta and opposite df, so the Adler-Wiser
sum over the full screened set equals the sum over one transition per pair
with the weight df [1/(w - Delta + i eta) - 1/(w + Delta + i eta)].  The
library's paired lists keep the transitions of every k whose partner index
is larger, and n < m where k is its own partner; this test applies that rule
to the oracle's full list, independently of the library.
"""
import numpy as np
import pytest

import oracle
import pairing_rule
import workloads
from oracle import response
from oracle.lattice import response_basis


def _partner(kgrid, qj):
    return pairing_rule.partner(kgrid, qj)


def _keep(tr, kt):
    return pairing_rule.keep(tr.k, tr.n, tr.m, kt)


@pytest.mark.parametrize("name,iq", [("fcc_small", 0), ("fcc_small", 1), ("h_tiny", 0),
                                     ("h_tiny", 1), ("feg_tiny", 1)])
def test_paired_sum_equals_full_sum(name, iq):
    w = workloads.get(name)
    st = oracle.build_states(w).with_temperature(w.temperatures[iq])
    qj = w.qs[iq]
    qred = np.asarray(qj, dtype=np.float64) / np.asarray(w.kgrid)
    basis, _ = response_basis(st.B, qred, w.ecut_chi[iq])
    tr = response.transitions(st, qj, w.f_trans_thr)
    P = response.pair_densities(st, tr, qj, basis)
    om = w.omega_grid(iq)[::10]
    full = response.chi0(tr, P, om, w.eta, st.n_k, st.omega)

    kt = _partner(w.kgrid, qj)
    keep = _keep(tr, kt)
    # every transition is kept or is the partner of a kept one
    kept = set(zip(tr.k[keep], tr.n[keep], tr.m[keep]))
    k_of = {k: kt[k] for k in range(st.n_k)}
    dropped = list(zip(tr.k[~keep], tr.n[~keep], tr.m[~keep]))
    n_self = 0
    for k, n, m in dropped:
        if n == m and k_of[k] == k:
            n_self += 1   # own partner with n = m: df is zero up to rounding
            continue
        assert (k_of[k], m, n) in kept
    assert int(keep.sum()) * 2 + n_self == len(tr.k)

    d, f, Pk = tr.delta[keep], tr.df[keep], P[keep]
    W = f[None, :] * (1.0 / (om[:, None] - d[None, :] + 1j * w.eta)
                      - 1.0 / (om[:, None] + d[None, :] + 1j * w.eta))
    X = (Pk[:, :, None] * Pk.conj()[:, None, :]).reshape(len(d), -1)
    paired = (2.0 / (st.n_k * st.omega)) * (W @ X).reshape(full.shape)
    err = np.max(np.abs(paired - full)) / np.max(np.abs(full))
    print(f"{name} q{iq}: {len(tr.k)} -> {int(keep.sum())} transitions, rel diff {err:.1e}")
    assert err < 1e-11


def test_partner_map_is_an_involution():
    for kgrid, qj in (((4, 4, 4), (0, 1, 1)), ((2, 2, 2), (2, 0, 0)), ((16, 16, 16), (4, 0, 0)),
                      ((3, 5, 4), (1, 2, 3))):
        kt = _partner(kgrid, qj)
        assert np.array_equal(kt[kt], np.arange(len(kt)))
