"""Seeded synthetic workloads for the chi0 -> S(q,w) -> F(q,tau) path.

This module is shared by the FP64 CPU oracle and by the HIP path.  It holds
only problem *definitions* (cells, grids, cutoffs, temperatures, potential
form-factor tables) and the seeded random draws that some of them need
(ion positions, q-vectors, per-q temperatures).  It contains none of the
arithmetic of the method itself: no Hamiltonian, no occupations, no pair
densities, no response functions.

All quantities are in Hartree atomic units unless a name says otherwise.

Workloads (the paper's systems are the model for their shapes):
  feg_c1     free-electron gas at the density of the paper's hydrogen box
             (14 protons in L = 6.641174 A, Sec. A.1), theta = T/T_F = 1.
  fcc_c2     Al-like fcc local empirical pseudopotential crystal (a = 4.05 A,
             Sec. 4.2 / A.1), q along [100] near 1 A^-1 (Sec. 4.2).
  h16_c3     warm-dense-hydrogen-like supercell, 16 protons at seeded random
             positions, rho = 0.08 g/cc, T = 4 eV (Sec. 4.1 / A.1).
  fcc_c4     fcc_c2 crystal, 32 seeded q-vectors with per-q temperature.
  h16_c5     h16_c3 system, 4 q-vectors, imaginary-time grid on [0, beta/2].
Small variants (``*_small``/``*_tiny``) keep every feature at sizes the
oracle finishes in seconds.
"""
from __future__ import annotations

import dataclasses
import math
from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

# CODATA 2018 conversion factors.
BOHR_PER_ANGSTROM = 1.0 / 0.529177210903
HARTREE_EV = 27.211386245988
AMU_GRAM = 1.66053906660e-24
HYDROGEN_AMU = 1.00794
CM3_PER_BOHR3 = (0.529177210903e-8) ** 3

# The paper's hydrogen box: 14 protons in a cube of side 6.641174 Angstrom
# (Sec. A.1).  Its electron density fixes rs for the free-electron workload.
PAPER_H_PROTONS = 14
PAPER_H_BOX_ANGSTROM = 6.641174


def ev(x: float) -> float:
    """Electron-volts to Hartree."""
    return x / HARTREE_EV


def paper_h_density() -> float:
    """Electron density (bohr^-3) of the paper's 14-proton box."""
    L = PAPER_H_BOX_ANGSTROM * BOHR_PER_ANGSTROM
    return PAPER_H_PROTONS / L ** 3


@dataclass(frozen=True)
class Potential:
    """Local pseudopotential: V(G) = v(|G|) * sum_I exp(-i G.R_I), V(0) = 0.

    v on the listed shells |G|^2 = shell_unit^2 * n2 is taken from shell_v.
    Off the listed shells v is 0, or, when ``gauss`` is set, the
    Gaussian-regularised Coulomb form factor
    -4 pi Z exp(-sigma^2 G^2 / 2) / (Omega G^2).
    """
    positions: Tuple[Tuple[float, float, float], ...] = ((0.0, 0.0, 0.0),)
    shell_unit: float = 1.0
    shell_n2: Tuple[int, ...] = ()
    shell_v: Tuple[float, ...] = ()
    gauss: bool = False
    z_ion: float = 1.0
    sigma: float = 0.5

    @property
    def is_free(self) -> bool:
        return (not self.gauss) and all(v == 0.0 for v in self.shell_v)


@dataclass(frozen=True)
class Workload:
    name: str
    cell: Tuple[Tuple[float, float, float], ...]      # rows a1, a2, a3 (bohr)
    kgrid: Tuple[int, int, int]                        # Monkhorst-Pack sizes
    ecut_wf: float                                     # 1/2 |k+G|^2 <= ecut_wf
    n_bands: int                                       # bands kept (snapped up; 0 = all)
    n_electrons: float                                 # electrons per cell
    potential: Potential
    qs: Tuple[Tuple[int, int, int], ...]               # q = sum_i qj_i/N_i b_i
    temperatures: Tuple[float, ...]                    # per q (Ha)
    ecut_chi: Tuple[float, ...]                        # per q: 1/2|q+G|^2 <= E
    n_omega: int
    omega_max: Tuple[float, ...]                       # per q
    eta: float
    xc: str                                            # "rpa" | "alda"
    dens_grid: Tuple[int, int, int] = (0, 0, 0)        # ALDA real-space grid
    n_tau: int = 65
    tau_half: bool = False                             # tau on [0, beta/2]
    f_trans_thr: float = 1e-8                          # |f_n - f_m| > thr
    f_trunc: float = 1e-5                              # last band must be below
    precisions: Tuple[str, ...] = ("fp64",)
    seed: int = 0

    @property
    def n_k(self) -> int:
        return int(np.prod(self.kgrid))

    def omega_grid(self, iq: int) -> np.ndarray:
        """Inclusive uniform grid on [0, omega_max(q)]."""
        return np.linspace(0.0, self.omega_max[iq], self.n_omega)

    def tau_grid(self, iq: int) -> np.ndarray:
        beta = 1.0 / self.temperatures[iq]
        top = 0.5 * beta if self.tau_half else beta
        return np.linspace(0.0, top, self.n_tau)

    def with_(self, **kw) -> "Workload":
        return dataclasses.replace(self, **kw)


def _cubic(a: float):
    return ((a, 0.0, 0.0), (0.0, a, 0.0), (0.0, 0.0, a))


def _fcc(a: float):
    h = 0.5 * a
    return ((0.0, h, h), (h, 0.0, h), (h, h, 0.0))


def feg_c1() -> Workload:
    """Free-electron gas, sc a=7 bohr, rs-matched to the paper's H box, theta=1.

    8^3 MP grid, plane waves up to 10 Ha, 56 bands kept (the lowest-lying
    band set whose top occupation is below 1e-5, the paper's band-count
    practice of Sec. 4.2), response basis 1/2|q+G|^2 <= 2 Ha, q = (2pi/a) x,
    200 frequencies on [0, 2] Ha, eta = 0.01 Ha, RPA.
    """
    a = 7.0
    n = paper_h_density()
    T = 0.5 * (3.0 * math.pi ** 2 * n) ** (2.0 / 3.0)      # theta = 1
    return Workload(
        name="feg_c1", cell=_cubic(a), kgrid=(8, 8, 8), ecut_wf=10.0,
        n_bands=56, n_electrons=n * a ** 3, potential=Potential(),
        qs=((8, 0, 0),), temperatures=(T,), ecut_chi=(2.0,), n_omega=200,
        omega_max=(2.0,), eta=0.01, xc="rpa", precisions=("fp64",), seed=1)


def fcc_c2() -> Workload:
    """Al-like fcc crystal, a = 7.6 bohr, Z_v = 3, three-shell local EPM.

    V(G) = -0.08, +0.03, +0.01 Ha on the (111), (200), (220) shells.  16^3 MP
    grid, E_wf = 20 Ha, 200 bands, T = 1 eV, response basis E_chi = 8.5 Ha,
    q = (2pi/a)(j/8, 0, 0) for j = 4, 5, 6, 500 frequencies on [0, 2] Ha,
    eta = 0.5 eV, ALDA kernel on a 20^3 real-space grid.
    """
    a = 7.6
    pot = Potential(positions=((0.0, 0.0, 0.0),), shell_unit=2 * math.pi / a,
                    shell_n2=(3, 4, 8), shell_v=(-0.08, 0.03, 0.01))
    qs = tuple((0, j, j) for j in (4, 5, 6))
    return Workload(
        name="fcc_c2", cell=_fcc(a), kgrid=(16, 16, 16), ecut_wf=20.0,
        n_bands=200, n_electrons=3.0, potential=pot, qs=qs,
        temperatures=(ev(1.0),) * 3, ecut_chi=(8.5,) * 3, n_omega=500,
        omega_max=(2.0,) * 3, eta=ev(0.5), xc="alda", dens_grid=(20, 20, 20),
        precisions=("fp64", "fp32", "bf16x3"), seed=2)


def fcc_small() -> Workload:
    """fcc_c2 shrunk so the oracle runs in seconds: 4^3 k, 40 bands, 3 q."""
    c2 = fcc_c2()
    qs = ((0, 1, 1), (1, 2, 0), (0, 2, 2))   # (2pi/a)(1/2,0,0) on the 4^3 grid is (0,1,1)
    return c2.with_(name="fcc_small", kgrid=(4, 4, 4), ecut_wf=8.0, n_bands=40,
                    qs=qs, temperatures=(ev(1.0), ev(4.0), ev(2.0)),
                    ecut_chi=(3.0,) * 3, n_omega=96, omega_max=(2.0,) * 3,
                    dens_grid=(16, 16, 16), seed=3)


def h_box_side(n_protons: int) -> float:
    """Cube side (bohr) holding n protons at the paper's hydrogen density."""
    return (n_protons / paper_h_density()) ** (1.0 / 3.0)


def _random_positions(seed: int, n: int, L: float):
    rng = np.random.default_rng(seed)
    return tuple(tuple(float(x) for x in row) for row in rng.uniform(0.0, L, (n, 3)))


def h16_c3(seed: int = 3) -> Workload:
    """16 protons, seeded uniform positions, rho = 0.08 g/cc, T = 4 eV.

    Gaussian-regularised Coulomb pseudopotential (sigma = 0.5 bohr), 4^3 MP,
    E_wf = 15 Ha, 800 bands, response basis E_chi = 2 Ha, q = 2pi/L x,
    1000 frequencies on [0, 5] Ha, eta = 0.5 eV, RPA.  The form factor on the
    three lowest shells (2pi/L){1, sqrt2, sqrt3} is tabulated so that it can
    be differentiated.
    """
    L = h_box_side(16)
    pot = _h_potential(seed, 16, L)
    return Workload(
        name="h16_c3", cell=_cubic(L), kgrid=(4, 4, 4), ecut_wf=15.0,
        n_bands=800, n_electrons=16.0, potential=pot, qs=((4, 0, 0),),
        temperatures=(ev(4.0),), ecut_chi=(2.0,), n_omega=1000,
        omega_max=(5.0,), eta=ev(0.5), xc="rpa",
        precisions=("bf16x3",), seed=seed)


def _h_potential(seed: int, n: int, L: float) -> Potential:
    g1 = 2 * math.pi / L
    sig = 0.5
    omega = L ** 3
    shells = (1, 2, 3)
    # Tabulated values equal the analytic form factor on those shells; they
    # are separate inputs so that a gradient with respect to them exists.
    vals = tuple(-4 * math.pi * math.exp(-0.5 * sig ** 2 * g1 ** 2 * s) /
                 (omega * g1 ** 2 * s) for s in shells)
    return Potential(positions=_random_positions(seed, n, L), shell_unit=g1,
                     shell_n2=shells, shell_v=vals, gauss=True, z_ion=1.0,
                     sigma=sig)


def h_tiny(seed: int = 5) -> Workload:
    """4 protons at the same density: every C3 feature at oracle-second size."""
    L = h_box_side(4)
    return Workload(
        name="h_tiny", cell=_cubic(L), kgrid=(2, 2, 2), ecut_wf=4.0,
        n_bands=64, n_electrons=4.0, potential=_h_potential(seed, 4, L),
        qs=((2, 0, 0), (1, 1, 0)), temperatures=(ev(4.0),) * 2,
        ecut_chi=(1.5,) * 2, n_omega=120, omega_max=(3.0,) * 2, eta=ev(0.5),
        xc="rpa", precisions=("fp64", "fp32", "bf16x3"), seed=seed)


def h16_c5(seed: int = 3) -> Workload:
    """h16_c3 with 4 q and 64 imaginary times on [0, beta/2]."""
    c3 = h16_c3(seed)
    qs = ((4, 0, 0), (0, 4, 0), (0, 0, 4), (2, 2, 0))
    return c3.with_(name="h16_c5", qs=qs, temperatures=c3.temperatures * 4,
                    ecut_chi=c3.ecut_chi * 4, omega_max=c3.omega_max * 4,
                    n_tau=64, tau_half=True)


def fcc_c4(seed: int = 4, n_q: int = 32, kgrid=(16, 16, 16), qmax: float = 4.0,
           ecut_floor: float = 8.5) -> Workload:
    """fcc_c2 crystal with n_q seeded q-vectors and per-q temperature.

    |q| ~ U[0.5, 4] bohr^-1 along a normalised random integer direction in
    {-2..2}^3 (not 0), snapped to the k-grid difference lattice and re-drawn
    when it lands on a reciprocal-lattice vector; T ~ U{1, 2, 4, 8} eV;
    E_chi(q) = max(8.5, (|q| + 0.5)^2 / 2); 800 frequencies on
    [0, min(max(2, q^2/2 + 2q), 11)] Ha.
    """
    c2 = fcc_c2()
    rng = np.random.default_rng(seed)
    A = np.array(c2.cell)
    B = 2 * math.pi * np.linalg.inv(A).T
    N = np.array(kgrid)
    qs, Ts, ecs, wms = [], [], [], []
    while len(qs) < n_q:
        mag = rng.uniform(0.5, qmax)
        d = rng.integers(-2, 3, size=3)
        T_ev = float(rng.choice([1.0, 2.0, 4.0, 8.0]))
        if not d.any():
            continue
        qc = mag * d / np.linalg.norm(d)
        red = A @ qc / (2 * math.pi)
        qj = np.rint(red * N).astype(int)
        if np.all(qj % N == 0):
            continue
        qn = float(np.linalg.norm((qj / N) @ B))
        qs.append(tuple(int(x) for x in qj))
        Ts.append(ev(T_ev))
        ecs.append(max(ecut_floor, 0.5 * (qn + 0.5) ** 2))
        wms.append(min(max(2.0, 0.5 * qn * qn + 2 * qn), 11.0))
    return c2.with_(name="fcc_c4", kgrid=tuple(kgrid), qs=tuple(qs),
                    temperatures=tuple(Ts), ecut_chi=tuple(ecs), n_omega=800,
                    omega_max=tuple(wms), seed=seed)


def fcc_c4_small(seed: int = 4) -> Workload:
    """fcc_c4 at oracle size: 6 ragged q (|q| <= 1.6) on a 4^3 grid, 40 bands."""
    w = fcc_c4(seed=seed, n_q=6, kgrid=(4, 4, 4), qmax=1.6, ecut_floor=3.0)
    return w.with_(name="fcc_c4_small", ecut_wf=8.0, n_bands=40, n_omega=64,
                   dens_grid=(16, 16, 16))


def feg_tiny() -> Workload:
    """Free-electron gas at brute-force size: 2^3 k, every plane wave a band."""
    c1 = feg_c1()
    return c1.with_(name="feg_tiny", kgrid=(2, 2, 2), ecut_wf=1.5, n_bands=0,
                    qs=((2, 0, 0), (1, 0, 0), (1, 1, 0)),
                    temperatures=c1.temperatures * 3, ecut_chi=(1.2,) * 3,
                    n_omega=40, omega_max=(2.0,) * 3, f_trunc=1.0)


REGISTRY = {
    "feg_c1": feg_c1, "fcc_c2": fcc_c2, "h16_c3": h16_c3, "fcc_c4": fcc_c4,
    "h16_c5": h16_c5, "fcc_small": fcc_small, "h_tiny": h_tiny,
    "fcc_c4_small": fcc_c4_small, "feg_tiny": feg_tiny,
}


def get(name: str) -> Workload:
    return REGISTRY[name]()


def rippled_spectrum(seed: int = 11, n_w: int = 500, omega_max: float = 2.0,
                     ripple_periods=(0.06, 0.11), ripple_amp: float = 0.03):
    """A seeded stand-in for a TDDFT S(q, w) with finite-k-grid ringing (the
    shape of Sec. 3, Fig. 3): a smooth positive spectrum (two Gaussian peaks
    on the w >= 0 grid, atomic units) plus quasi-periodic ripples of the given
    periods in w, slowly modulated, plus 1e-4 white noise.  Returns
    (omega [n_w], S [n_w], ripple frequencies 1/period)."""
    rng = np.random.default_rng(seed)
    w = np.linspace(0.0, omega_max, n_w)
    c1, c2 = omega_max * (0.25 + 0.05 * rng.random()), omega_max * (0.55 + 0.05 * rng.random())
    s1, s2 = omega_max * 0.08, omega_max * 0.15
    smooth = np.exp(-0.5 * ((w - c1) / s1) ** 2) + 0.5 * np.exp(-0.5 * ((w - c2) / s2) ** 2)
    ripple = np.zeros_like(w)
    for p in ripple_periods:
        phase = 2.0 * np.pi * rng.random()
        env = 1.0 + 0.3 * np.sin(2.0 * np.pi * w / omega_max + phase)
        ripple += ripple_amp * env * np.sin(2.0 * np.pi * w / p + phase)
    S = smooth * (1.0 + ripple) + 1e-4 * rng.standard_normal(n_w)
    return w, S, np.array([1.0 / p for p in ripple_periods])


def kg_conductivity(seed: int = 13, n_w: int = 500, omega_max: float = 2.0,
                    ripple_period: float = 0.05, ripple_amp: float = 0.03):
    """A seeded stand-in for a Kubo-Greenwood conductivity sigma(w) of a warm
    metal with finite-k-grid ringing (Sec. A.3): a Drude term
    sigma_D / (1 - i w tau) plus two bound-bound oscillators
    (f / 4 pi) (-i w) / (w0^2 - w^2 - i w gamma), its real part rippled with
    the given period (atomic units, w >= 0 grid).  Returns (omega [n_w],
    sigma [n_w] complex128)."""
    rng = np.random.default_rng(seed)
    w = np.linspace(0.0, omega_max, n_w)
    tau = 8.0 + 4.0 * rng.random()
    sig = (0.05 + 0.02 * rng.random()) / (1.0 - 1j * w * tau)
    for w0, g in ((0.6 * omega_max, 0.05), (0.8 * omega_max, 0.08)):
        f = 0.02 + 0.02 * rng.random()
        sig = sig + (f / (4.0 * np.pi)) * (-1j * w) / (w0 ** 2 - w ** 2 - 1j * w * g)
    phase = 2.0 * np.pi * rng.random()
    sig = sig.real * (1.0 + ripple_amp * np.sin(2.0 * np.pi * w / ripple_period + phase)) \
        + 1j * sig.imag
    return w, sig.astype(np.complex128)
