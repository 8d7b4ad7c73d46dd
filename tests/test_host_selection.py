"""The library's two host-side selection routines against the oracle's, on
seeded random inputs (no GPU involved: both run on the host): the reference
eta of the eta test (Sec. 2) and the filter selection of the attenuation
grid search (Sec. 3), including non-finite scores and empty results."""
import numpy as np
import pytest

from oracle import attenuation as att
from oracle import eta as oeta


@pytest.fixture(scope="module")
def tdx():
    import paper_2510_01875_amd as m
    return m


def test_sg_select_matches_oracle(tdx):
    rng = np.random.default_rng(21)
    for trial in range(300):
        n = int(rng.integers(1, 12))
        sc = np.zeros((n, 5))
        sc[:, 2] = rng.normal(-5000.0, 300.0, n)
        sc[:, 3] = rng.random(n)
        sc[:, 4] = rng.random(n)
        if trial % 5 == 0:
            sc[rng.integers(0, n), 2] = np.inf
        if trial % 7 == 0:
            sc[rng.integers(0, n), 4] = np.nan
        rs = np.abs(rng.normal(0.0, [1.0, 3e-3, 3e-5], (n, 3)))
        lam_f, lam_c = float(rng.choice([0.0, 1.0, 100.0])), float(rng.choice([0.0, 10.0]))
        for resid in (rs, None):
            want = att.sg_select(sc, resid, 500, lam_f, lam_c)
            got = tdx.sg_select(sc, resid, 500, lam_f, lam_c)
            assert got == want, (trial, got, want)


def test_eta_reference_matches_oracle(tdx):
    rng = np.random.default_rng(22)
    for trial in range(300):
        n = int(rng.integers(1, 10))
        etas = np.cumsum(rng.random(n) + 0.01)
        base = rng.normal(1.0, 0.2, 5)
        drift = np.cumsum(np.abs(rng.normal(0.0, 0.01, (n, 5))), axis=0)
        drift[0] = 0.0
        m = base + drift * base
        tol = float(rng.choice([1e-3, 1e-2, 3e-2]))
        assert tdx.eta_reference(m, etas, tol) == oeta.eta_reference(m, etas, tol), trial
