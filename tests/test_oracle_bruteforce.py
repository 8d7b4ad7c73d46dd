"""P14: explicit-loop evaluation of every step on a tiny crystal against the
vectorised oracle, plus quadrature checks of the DSF/ITCF steps."""
import cmath
import math

import numpy as np
import pytest
from scipy import integrate

import oracle
import workloads
from oracle import response, states
from oracle.lattice import kq_map, response_basis


def _tiny():
    return workloads.fcc_small().with_(kgrid=(2, 2, 2), ecut_wf=2.0, n_bands=8,
                                       qs=((0, 1, 1),), temperatures=(workloads.ev(8.0),),
                                       ecut_chi=(0.9,), n_omega=6, omega_max=(1.5,),
                                       f_trunc=1.0, xc="rpa")


def _solve_loops(A, b):
    """Gaussian elimination with partial pivoting, written out."""
    n = len(b)
    M = [[complex(A[i][j]) for j in range(n)] + [complex(b[i])] for i in range(n)]
    for c in range(n):
        p = max(range(c, n), key=lambda r: abs(M[r][c]))
        M[c], M[p] = M[p], M[c]
        for r in range(c + 1, n):
            f = M[r][c] / M[c][c]
            for j in range(c, n + 1):
                M[r][j] -= f * M[c][j]
    x = [0j] * n
    for r in range(n - 1, -1, -1):
        s = M[r][n] - sum(M[r][j] * x[j] for j in range(r + 1, n))
        x[r] = s / M[r][r]
    return x


def test_p14_bruteforce_tiny_crystal():
    w = _tiny()
    st = oracle.build_states(w)
    iq = 0
    r = oracle.run_q(w, st, iq)
    assert len(r.basis) <= 7 and max(len(e) for e in st.eps) <= 9
    # Hamiltonian element by element
    k = 3
    m = st.millers[k]
    p = (st.kred[k] + m) @ st.B
    H = np.zeros((len(m), len(m)), dtype=complex)
    for i in range(len(m)):
        for j in range(len(m)):
            G = (m[i] - m[j]) @ st.B
            g2 = float(G @ G)
            v = 0.0
            for n2, val in zip(w.potential.shell_n2, w.potential.shell_v):
                if g2 > 0 and abs(g2 - (w.potential.shell_unit ** 2) * n2) < 1e-9 * g2:
                    v = val
            sf = sum(cmath.exp(-1j * float(G @ np.asarray(R))) for R in w.potential.positions)
            H[i, j] = v * sf + (0.5 * float(p[i] @ p[i]) if i == j else 0.0)
    Hv = states.hamiltonian(st.kred[k], m, st.B, w.potential, st.omega)
    assert np.max(np.abs(H - Hv)) < 1e-15
    # transitions, pair densities, chi0 by explicit loops
    kp, gs = kq_map(w.kgrid, w.qs[iq])
    rows = []
    for kk in range(st.n_k):
        j = kp[kk]
        for n in range(len(st.eps[kk])):
            for mm in range(len(st.eps[j])):
                df = st.occ[kk][n] - st.occ[j][mm]
                if abs(df) > w.f_trans_thr:
                    rows.append((kk, j, n, mm, st.eps[j][mm] - st.eps[kk][n], df))
    assert len(rows) == len(r.tr)
    lookup = [{tuple(x): i for i, x in enumerate(st.millers[j])} for j in range(st.n_k)]
    P = np.zeros((len(rows), len(r.basis)), dtype=complex)
    for t, (kk, j, n, mm, _, _) in enumerate(rows):
        for g, G in enumerate(r.basis):
            s = 0j
            for i1, G1 in enumerate(st.millers[kk]):
                idx = lookup[j].get(tuple(G1 + G + gs[kk]))
                if idx is not None:
                    s += st.coef[kk][n][i1].conjugate() * st.coef[j][mm][idx]
            P[t, g] = s
    assert np.max(np.abs(P - r.P)) < 1e-14
    nG = len(r.basis)
    pref = 2 / (st.n_k * st.omega)
    for wi, om in enumerate(r.omegas):
        C = np.zeros((nG, nG), dtype=complex)
        for a in range(nG):
            for b in range(nG):
                s = 0j
                for t, (_, _, _, _, dl, df) in enumerate(rows):
                    s += df / (om - dl + 1j * w.eta) * P[t, a] * P[t, b].conjugate()
                C[a, b] = pref * s
        assert np.max(np.abs(C - r.chi0[wi])) < 1e-13 * np.max(np.abs(C))
        # Dyson by elimination
        A = np.eye(nG) - C @ r.K
        x = _solve_loops(A, C[:, r.iG0])
        assert abs(x[r.iG0] - r.chi00[wi]) < 1e-12 * abs(r.chi00[wi])
    # DSF and ITCF by loops
    S = []
    for wi, om in enumerate(r.omegas):
        if om == 0:
            S.append(-r.chi00[wi + 1].imag / (math.pi * r.density * r.beta * r.omegas[wi + 1]))
        else:
            S.append(-r.chi00[wi].imag / (math.pi * r.density * (1 - math.exp(-r.beta * om))))
    assert np.allclose(S, r.S, rtol=1e-13, atol=0)
    for ti, tau in enumerate(r.taus):
        F = 0.0
        for j in range(len(S) - 1):
            h = r.omegas[j + 1] - r.omegas[j]
            g = lambda i: S[i] * (math.exp(-tau * r.omegas[i]) + math.exp(-(r.beta - tau) * r.omegas[i]))
            F += 0.5 * h * (g(j) + g(j + 1))
        assert abs(F - r.F[ti]) < 1e-13 * abs(F)


def test_itcf_quadrature_converges_to_integral():
    """Trapezoid ITCF of a smooth S(w) against adaptive quadrature."""
    beta = 3.0
    S = lambda x: x * x * math.exp(-2 * (x - 1.5) ** 2)
    om = np.linspace(0, 8, 4001)
    Sv = np.array([S(x) for x in om])
    taus = np.linspace(0, beta, 7)
    F = response.itcf(Sv, om, beta, taus)
    for t, f in zip(taus, F):
        ref, _ = integrate.quad(lambda x: S(x) * (math.exp(-t * x) + math.exp(-(beta - t) * x)), 0, 8)
        assert abs(f - ref) < 1e-6 * ref


def test_dsf_zero_frequency_limit():
    """-Im chi(w)/(pi n (1-e^{-beta w})) -> -Im chi'(0)/(pi n beta) as w -> 0."""
    n, beta = 0.01, 4.0
    om = np.array([0.0, 1e-3, 2e-3])
    chi = -1j * 0.7 * om                    # Im chi linear in w
    chi[0] = 0
    S = response.dsf(chi, om, beta, n)
    lim = 0.7 / (math.pi * n * beta)
    assert abs(S[0] - lim) < 1e-15 * lim
    assert abs(S[1] - lim) < 1e-2 * lim
