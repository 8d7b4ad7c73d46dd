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
    fx, fc = xc.fxc_parts(n)
    assert abs(fx + math.pi / kf ** 2) < 1e-14 * math.pi / kf ** 2
    assert abs(xc.fxc_alda(n) - fc - fx) <= 1e-15 * abs(xc.fxc_alda(n))


@pytest.mark.parametrize("n", [1e-3, 7.0826e-3, 0.03, 0.3])
def test_fxc_is_second_derivative_of_energy_density(n):
    h = 1e-3 * n
    e = lambda x: x * xc.exc_pw92(x)
    # fourth-order central stencil (truncation of order h^4)
    fd4 = (-e(n + 2 * h) + 16 * e(n + h) - 30 * e(n) + 16 * e(n - h) - e(n - 2 * h)) / (12 * h * h)
    assert abs(fd4 - xc.fxc_alda(n)) < 1e-6 * abs(xc.fxc_alda(n))


def test_hyperdual_arithmetic_against_closed_forms():
    """Derivatives of a function with known ones, through every operation
    the kernel uses (sum, product, quotient, power, log1p)."""
    x0 = np.array([0.3, 1.7, 4.0])
    x = xc.HyperDual(x0, np.ones(3), np.ones(3), np.zeros(3))
    f = (x ** 1.5) * (1.0 / (1.0 + x)).log1p() - 2.0 / x
    g = np.log1p(1.0 / (1.0 + x0))
    g1 = -1.0 / ((1.0 + x0) * (2.0 + x0))
    g2 = (2.0 * x0 + 3.0) / ((1.0 + x0) ** 2 * (2.0 + x0) ** 2)
    p, p1, p2 = x0 ** 1.5, 1.5 * x0 ** 0.5, 0.75 * x0 ** -0.5
    want1 = p1 * g + p * g1 + 2.0 / x0 ** 2
    want2 = p2 * g + 2 * p1 * g1 + p * g2 - 4.0 / x0 ** 3
    assert np.max(np.abs(f.b - want1) / np.abs(want1)) < 1e-13
    assert np.max(np.abs(f.c - want1) / np.abs(want1)) < 1e-13
    assert np.max(np.abs(f.d - want2) / np.abs(want2)) < 1e-13


def test_pw92_high_density_limit():
    """As rs -> 0 the PW92 form reduces to the high-density expansion
    eps_c = c0 ln rs - c1 + O(rs^1/2) with c0 = (1 - ln 2) / pi^2 (the
    random-phase coefficient) and c1 = 0.046644 Ha, which fix A and beta1 of
    the parametrisation; beta2 = 2 A beta1^2 is its own relation between
    them.  A typo in A, beta1 or beta2 fails here."""
    c0 = (1.0 - math.log(2.0)) / math.pi ** 2
    A, (b1, b2, _, _) = xc.PW92_A, xc.PW92_B
    assert abs(A - c0) < 2e-5 * c0
    assert abs(b1 - math.exp(-0.046644 / (2 * A)) / (2 * A)) < 1e-4 * b1
    assert abs(b2 - 2 * A * b1 ** 2) < 1e-4 * b2
    rs, h = 1e-12, 1e-3
    slope = (xc.ec_pw92_rs(rs * math.exp(h)) - xc.ec_pw92_rs(rs * math.exp(-h))) / (2 * h)
    assert abs(slope - c0) < 1e-6
    assert abs(xc.ec_pw92_rs(rs) - (c0 * math.log(rs) - 0.046644)) < 1e-5


def test_pw92_correlation_reference_values():
    """PW92 reproduces the Ceperley-Alder electron-gas correlation energies
    it was fitted to (about -0.0598 Ha at rs = 1 and -0.0448 Ha at rs = 2)."""
    assert abs(xc.ec_pw92_rs(1.0) + 0.0598) < 1e-3
    assert abs(xc.ec_pw92_rs(2.0) + 0.0448) < 1e-3


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


@pytest.mark.parametrize("n", [1e-4, 7.0826e-3, 0.027, 0.5])
def test_p11_exchange_kernel_derivative_closed_form(n):
    """d f_x/dn of Slater exchange: (2/9)(3/pi)^(1/3) n^(-5/3)."""
    dx, _ = xc.fxc_deriv_parts(n)
    ref = (2.0 / 9.0) * (3.0 / math.pi) ** (1.0 / 3.0) * n ** (-5.0 / 3.0)
    assert abs(dx - ref) < 1e-13 * ref


@pytest.mark.parametrize("n", [1e-3, 7.0826e-3, 0.03, 0.3])
def test_fxc_derivative_against_finite_differences(n):
    """The complex-step third derivative against a fourth-order central
    difference of the hyper-dual second derivative."""
    h = 1e-3 * n
    f = xc.fxc_alda
    fd4 = (f(n - 2 * h) - 8 * f(n - h) + 8 * f(n + h) - f(n + 2 * h)) / (12 * h)
    got = xc.fxc_alda_deriv(n)
    assert abs(fd4 - got) < 1e-7 * abs(got)
    _, dc = xc.fxc_deriv_parts(n)
    fc = lambda x: xc.fxc_parts(x)[1]
    fd4c = (fc(n - 2 * h) - 8 * fc(n - h) + 8 * fc(n + h) - fc(n + 2 * h)) / (12 * h)
    assert abs(fd4c - dc) < 1e-6 * abs(dc)
