"""Units and workload definitions against numbers printed in the paper (P12)."""
import json
import math
import os

import numpy as np

import workloads
from oracle.lindhard import fermi_energy

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_units.json")))


def test_fermi_temperature_of_paper_box():
    # Sec. A.1: T = 4.8 eV is the Fermi temperature of 14 protons in L = 6.641174 A.
    box = GOLD["hydrogen_box"]
    L = box["box_angstrom"] * workloads.BOHR_PER_ANGSTROM
    n = box["n_protons"] / L ** 3
    ef_ev = fermi_energy(n) * workloads.HARTREE_EV
    assert abs(ef_ev - box["fermi_temperature_ev"]) < 0.01
    assert abs(n - workloads.paper_h_density()) < 1e-15


def test_q_is_smallest_box_wavenumber():
    # Sec. 2 / Fig. 1: q = 0.946 1/A equals 2 pi / L of the same box.
    L = GOLD["hydrogen_box"]["box_angstrom"]
    assert abs(2 * math.pi / L - GOLD["hydrogen_q"]["q_inv_angstrom"]) < 5e-4


def test_box_density_in_g_per_cc():
    box = GOLD["hydrogen_box"]
    mass = box["n_protons"] * workloads.HYDROGEN_AMU * workloads.AMU_GRAM
    vol = (box["box_angstrom"] * 1e-8) ** 3
    assert abs(mass / vol - GOLD["hydrogen_density"]["rho_g_cc"]) < 5e-4


def test_feg_theta_one():
    w = workloads.feg_c1()
    n = w.n_electrons / 7.0 ** 3
    assert abs(w.temperatures[0] / fermi_energy(n) - 1.0) < 1e-14


def test_h_supercell_density():
    w = workloads.h16_c3()
    L = w.cell[0][0]
    assert abs(16 / L ** 3 - workloads.paper_h_density()) < 1e-15
    assert len(w.potential.positions) == 16
    assert all(0 <= x < L for p in w.potential.positions for x in p)


def test_fcc_q_values_bracket_one_inverse_angstrom():
    # Sec. 4.2 studies q = 1.0 1/A along [100]; the three q bracket it.
    w = workloads.fcc_c2()
    A = np.array(w.cell)
    B = 2 * math.pi * np.linalg.inv(A).T
    qs = [np.linalg.norm((np.array(qj) / 16) @ B) * workloads.BOHR_PER_ANGSTROM for qj in w.qs]
    for qj in w.qs:
        qc = (np.array(qj) / 16) @ B
        assert abs(qc[1]) < 1e-12 and abs(qc[2]) < 1e-12      # along [100]
    assert qs[0] < 1.0 < qs[2]


def test_c4_draws_are_ragged_and_off_lattice():
    w = workloads.fcc_c4()
    assert len(w.qs) == 32
    N = np.array(w.kgrid)
    assert all(np.any(np.array(q) % N != 0) for q in w.qs)
    assert set(round(t * workloads.HARTREE_EV, 6) for t in w.temperatures) <= {1.0, 2.0, 4.0, 8.0}
    assert len(set(w.temperatures)) >= 3
