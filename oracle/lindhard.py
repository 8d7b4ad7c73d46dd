"""Free-electron-gas closed forms used to pin the oracle.

Test infrastructure only (see the package docstring).

  * k-sampled finite-T Lindhard function: the Adler-Wiser sum written
    directly over plane waves (no eigensolver, no pair-density sums).
  * continuum finite-T Lindhard function (spin-summed, per volume):
      chi0(q,z) = 1/(2 pi^2 q) int_0^inf dk k f(k^2/2)
                  [Log(z - q^2/2 + kq) - Log(z - q^2/2 - kq)
                   - Log(z + q^2/2 + kq) + Log(z + q^2/2 - kq)],  z = w + i eta
    and its eta -> 0 imaginary part
      Im chi0 = -T/(2 pi q) ln[(1 + e^{(mu - a^2/2)/T}) / (1 + e^{(mu - b^2/2)/T})],
      a = w/q - q/2, b = w/q + q/2.
  * continuum chemical potential from n = sqrt(2)/pi^2 T^{3/2} F_{1/2}(mu/T).
"""
from __future__ import annotations

import itertools
import math

import numpy as np
from scipy import integrate, optimize


def _fd(e, mu, T):
    x = (e - mu) / T
    return np.where(x > 0, np.exp(-np.clip(x, 0, None)) / (1 + np.exp(-np.clip(x, 0, None))),
                    1.0 / (1.0 + np.exp(np.clip(x, None, 0))))


def pw_sets(cell, kgrid, ecut, n_bands, degen_tol=1e-6):
    """Kept plane waves per MP k-point: lowest n_bands energies, with the cut
    moved up past any degenerate multiplet (0 = all).  Independent of the
    oracle's lattice and eigensolver code."""
    A = np.asarray(cell, dtype=np.float64)
    B = 2 * math.pi * np.linalg.inv(A).T
    N = np.asarray(kgrid)
    out = []
    gmax = int(math.ceil(math.sqrt(2 * ecut) * np.max(np.linalg.norm(A, axis=1))
                         / (2 * math.pi))) + 2
    rng = range(-gmax, gmax + 1)
    allm = np.array(list(itertools.product(rng, rng, rng)))
    for r in itertools.product(range(N[0]), range(N[1]), range(N[2])):
        kr = (2 * np.asarray(r) + 1 - N) / (2.0 * N)
        p = (kr + allm) @ B
        e = 0.5 * np.sum(p * p, axis=1)
        sel = e <= ecut
        m, e = allm[sel], e[sel]
        o = np.argsort(e, kind="stable")
        m, e = m[o], e[o]
        nb = len(e) if n_bands <= 0 else min(n_bands, len(e))
        while nb < len(e) and e[nb] - e[nb - 1] < degen_tol:
            nb += 1
        out.append((kr, m[:nb], e[:nb]))
    return B, out


def ksampled_mu(sets, T, n_electrons, n_k):
    e = np.concatenate([s[2] for s in sets])
    g = lambda mu: 2.0 / n_k * float(np.sum(_fd(e, mu, T))) - n_electrons
    return optimize.brentq(g, e.min() - 60 * T, e.max() + 60 * T, xtol=1e-15,
                           rtol=1e-15, maxiter=500)


def ksampled_chi0(cell, kgrid, ecut, n_bands, qj, Gm, omegas, eta, T,
                  n_electrons, thr):
    """chi0_GG(q, w) for V = 0, written over plane waves p = k + G1:
    2/(N_k Omega) sum_k sum_{p kept at k, p+q+G kept at k+q, |df|>thr}
      [f(p^2/2) - f(|p+q+G|^2/2)] / (w + p^2/2 - |p+q+G|^2/2 + i eta).
    """
    A = np.asarray(cell, dtype=np.float64)
    omega_cell = abs(np.linalg.det(A))
    N = np.asarray(kgrid)
    B, sets = pw_sets(cell, kgrid, ecut, n_bands)
    n_k = len(sets)
    mu = ksampled_mu(sets, T, n_electrons, n_k)
    qred = np.asarray(qj) / N
    out = np.zeros(len(omegas), dtype=np.complex128)
    for ki, (kr, m, e) in enumerate(sets):
        # the k-point reached by k+q, found by its reduced coordinate
        krq = kr + qred
        target = None
        for kr2, m2, e2 in sets:
            d = krq - kr2
            if np.allclose(d, np.rint(d), atol=1e-12):
                target = (np.rint(d).astype(int), m2)
                break
        gs, m2 = target
        kept2 = {tuple(x) for x in m2}
        for G1, e1 in zip(m, e):
            # k + q + G1 + G = k2 + gs + G1 + G: Miller index G1 + G + gs at k2
            dest = tuple(G1 + np.asarray(Gm) + gs)
            if dest not in kept2:
                continue
            pp = (kr + G1 + qred + np.asarray(Gm)) @ B
            e2v = 0.5 * float(pp @ pp)
            df = float(_fd(e1, mu, T) - _fd(e2v, mu, T))
            if abs(df) <= thr:
                continue
            out += df / (np.asarray(omegas) + e1 - e2v + 1j * eta)
    return out * 2.0 / (n_k * omega_cell), mu


def fermi_half(eta_red):
    """F_{1/2}(x) = int_0^inf t^{1/2} / (1 + e^{t - x}) dt."""
    f = lambda t: math.sqrt(t) / (1.0 + math.exp(min(t - eta_red, 700.0)))
    hi = max(eta_red, 0.0) + 60.0
    v, _ = integrate.quad(f, 0.0, hi, limit=400, epsabs=1e-14, epsrel=1e-13)
    return v


def continuum_mu(n, T):
    g = lambda mu: math.sqrt(2) / math.pi ** 2 * T ** 1.5 * fermi_half(mu / T) - n
    return optimize.brentq(g, -50 * T, 50 * T + 10.0, xtol=1e-15, rtol=1e-14)


def continuum_chi0(q, w, eta, T, mu):
    """Continuum Lindhard function at z = w + i eta by quadrature over k."""
    z = w + 1j * eta
    h = 0.5 * q * q

    def integrand(k, part):
        f = 1.0 / (1.0 + math.exp(min((0.5 * k * k - mu) / T, 700.0)))
        L = (np.log(z - h + k * q) - np.log(z - h - k * q)
             - np.log(z + h + k * q) + np.log(z + h - k * q))
        return k * f * (L.real if part == 0 else L.imag)

    kmax = math.sqrt(2 * (max(mu, 0.0) + 60 * T))
    # breakpoints where a log argument's real part changes sign
    pts = sorted({abs(x) for x in ((w - h) / q, (w + h) / q) if 0 < abs(x) < kmax})
    re, _ = integrate.quad(integrand, 0, kmax, args=(0,), points=pts or None,
                           limit=800, epsabs=1e-13, epsrel=1e-11)
    im, _ = integrate.quad(integrand, 0, kmax, args=(1,), points=pts or None,
                           limit=800, epsabs=1e-13, epsrel=1e-11)
    return (re + 1j * im) / (2 * math.pi ** 2 * q)


def continuum_im_chi0(q, w, T, mu):
    """eta -> 0 imaginary part, closed form."""
    a = w / q - q / 2
    b = w / q + q / 2
    la = np.logaddexp(0.0, (mu - 0.5 * a * a) / T)
    lb = np.logaddexp(0.0, (mu - 0.5 * b * b) / T)
    return -T / (2 * math.pi * q) * (la - lb)


def fermi_energy(n):
    """E_F = (3 pi^2 n)^(2/3) / 2 for the spin-unpolarised electron gas."""
    return 0.5 * (3.0 * math.pi ** 2 * n) ** (2.0 / 3.0)


def mp_free_chi0(cell, kgrid, ecut, qj, omegas, eta, T, n_electrons, chunk=1 << 18):
    """chi0_00(q, w) of the free-electron gas on a Monkhorst-Pack grid with
    every plane wave of energy <= ecut at every k (no band count), written
    over the momenta p = k + G of all grid points and plane waves at once:
      2/(N_k Omega) sum_p [f(p^2/2) - f(|p+q|^2/2)] / (w + p^2/2 - |p+q|^2/2 + i eta),
    mu from the same momenta at N_e electrons.  q = sum_i qj_i / N_i b_i.
    Returns (chi0 [n_w], mu).  The same sum as ksampled_chi0 with n_bands = 0
    and no screening, vectorised so that fine grids stay affordable."""
    A = np.asarray(cell, dtype=np.float64)
    omega_cell = abs(np.linalg.det(A))
    B = 2 * math.pi * np.linalg.inv(A).T
    N = np.asarray(kgrid)
    gmax = int(math.ceil(math.sqrt(2 * ecut) * np.max(np.linalg.norm(A, axis=1))
                         / (2 * math.pi))) + 2
    rng = np.arange(-gmax, gmax + 1)
    G = np.array(np.meshgrid(rng, rng, rng, indexing="ij")).reshape(3, -1).T
    axes = [(2 * np.arange(n) + 1 - n) / (2.0 * n) for n in N]
    K = np.array(np.meshgrid(*axes, indexing="ij")).reshape(3, -1).T
    ps, es = [], []
    for kr in K:
        p = (kr + G) @ B
        e = 0.5 * np.sum(p * p, axis=1)
        sel = e <= ecut
        ps.append(p[sel])
        es.append(e[sel])
    p = np.concatenate(ps)
    e = np.concatenate(es)
    n_k = len(K)
    g = lambda mu: 2.0 / n_k * float(np.sum(_fd(e, mu, T))) - n_electrons
    mu = optimize.brentq(g, e.min() - 60 * T, e.max() + 60 * T, xtol=1e-15, rtol=1e-15,
                         maxiter=500)
    q = (np.asarray(qj, dtype=np.float64) / N) @ B
    om = np.asarray(omegas, dtype=np.float64)
    out = np.zeros(len(om), dtype=np.complex128)
    for lo in range(0, len(e), chunk):
        e1 = e[lo:lo + chunk]
        pq = p[lo:lo + chunk] + q
        e2 = 0.5 * np.sum(pq * pq, axis=1)
        df = _fd(e1, mu, T) - _fd(e2, mu, T)
        out += (df[None, :] / (om[:, None] + (e1 - e2)[None, :] + 1j * eta)).sum(axis=1)
    return out * 2.0 / (n_k * omega_cell), mu
