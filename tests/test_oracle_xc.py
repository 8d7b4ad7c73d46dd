"""Oracle pins for the ALDA kernel and the real-space density (P11)."""
import math

import numpy as np
import pytest

import oracle
import workloads
from oracle import xc
from oracle.lattice import response_basis


@pytest.mark.parametrize("n", [1e-4, 7.0826e-3, 0.027, 0.5])
def test_p11_exchange_kernel_uniform(n):
    """Slater exchange: f_x = -pi / k_F^2."""
    kf = (3 * math.pi ** 2 * n) ** (1 / 3)
    fx = -(1 / 3) * (3 / math.pi) ** (1 / 3) * n ** (-2 / 3)
    assert abs(fx + math.pi / kf ** 2) < 1e-14 * math.pi / kf ** 2
    # full kernel minus its correlation part equals f_x
    rs = xc.rs_of(n)
    _, e1, e2 = xc._pw92_terms(rs)
    fc = (rs * rs * e2 - 2 * rs * e1) / (9 * n)
    assert abs(xc.fxc_alda(n) - fc + math.pi / kf ** 2) < 1e-12 * math.pi / kf ** 2


@pytest.mark.parametrize("n", [1e-3, 7.0826e-3, 0.03, 0.3])
def test_fxc_is_second_derivative_of_energy_density(n):
    h = 1e-3 * n
    e = lambda x: x * xc.exc_pw92(x)
    fd = (e(n + h) - 2 * e(n) + e(n - h)) / h ** 2
    # 4th-order stencil for a tighter check
    fd4 = (-e(n + 2 * h) + 16 * e(n + h) - 30 * e(n) + 16 * e(n - h) - e(n - 2 * h)) / (12 * h * h)
    assert abs(fd4 - xc.fxc_alda(n)) < 1e-6 * abs(xc.fxc_alda(n))


def test_pw92_correlation_reference_values():
    """PW92 reproduces the Ceperley-Alder electron-gas correlation energies
    it was fitted to (about -0.0598 Ha at rs = 1 and -0.0448 Ha at rs = 2)
    and the high-density form 0.0311 ln rs - 0.047."""
    ec = lambda rs: xc._pw92_terms(np.array(rs))[0]
    assert abs(ec(1.0) + 0.0598) < 1e-3
    assert abs(ec(2.0) + 0.0448) < 1e-3
    rs = 1e-4
    assert abs(ec(rs) - (0.031091 * math.log(rs) - 0.047)) < 2e-3


def test_density_is_uniform_for_free_electrons():
    w = workloads.feg_tiny().with_(dens_grid=(16, 16, 16))
    st = oracle.build_states(w)
    rho = xc.density_on_grid(st, w.dens_grid)
    n = w.n_electrons / st.omega
    assert np.max(np.abs(rho - n)) < 1e-13 * n


def test_density_integrates_to_electron_count():
    w = workloads.fcc_small()
    st = oracle.build_states(w)
    rho = xc.density_on_grid(st, w.dens_grid)
    total = rho.mean() * st.omega
    assert abs(total - w.n_electrons) < 1e-12 * w.n_electrons
    assert rho.min() > 0


def test_fxc_matrix_free_electrons_is_diagonal():
    w = workloads.feg_tiny().with_(dens_grid=(16, 16, 16))
    st = oracle.build_states(w)
    qred = np.asarray(w.qs[0]) / np.asarray(w.kgrid)
    basis, _ = response_basis(st.B, qred, w.ecut_chi[0])
    K = xc.fxc_matrix(st, w.dens_grid, basis)
    n = w.n_electrons / st.omega
    assert np.allclose(K, xc.fxc_alda(n) * np.eye(len(basis)), rtol=0, atol=1e-12 * abs(xc.fxc_alda(n)))


def test_fxc_matrix_is_hermitian_and_matches_direct_dft():
    w = workloads.fcc_small()
    st = oracle.build_states(w)
    qred = np.asarray(w.qs[1]) / np.asarray(w.kgrid)
    basis, _ = response_basis(st.B, qred, w.ecut_chi[1])
    K = xc.fxc_matrix(st, w.dens_grid, basis)
    assert np.allclose(K, K.conj().T, atol=1e-14 * np.abs(K).max())
    # one element by a direct real-space sum
    N = np.array(w.dens_grid)
    f = xc.fxc_alda(xc.density_on_grid(st, w.dens_grid))
    j = np.array(np.meshgrid(*[np.arange(x) for x in N], indexing="ij")).reshape(3, -1).T
    d = basis[3] - basis[7]
    direct = np.mean(f.reshape(-1) * np.exp(-2j * math.pi * (j @ (d / N))))
    assert abs(direct - K[3, 7]) < 1e-13 * np.abs(K).max()
