"""The Kubo-Greenwood route on the GPU (Sec. A.3): S* from a conductivity
against the oracle, then the whole route (F*, the eta metrics, the
attenuation of S*, and the way back to eps^{-1} and sigma) against the
oracle's composition of the same steps, on a seeded Drude-Lorentz
conductivity with ringing on 500 frequencies."""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

BETA, DENS = 30.0, 0.018


@pytest.fixture(scope="module")
def tdx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2510_01875_amd as m
    return m


def _dev(x):
    import torch
    return torch.as_tensor(np.ascontiguousarray(x), device="cuda")


def test_kg_dsf_matches_oracle(tdx):
    from oracle import kubo_greenwood as kg
    w, sig = workloads.kg_conductivity(n_w=500)
    ctx = tdx.Context(0)
    S = tdx.kg_dsf(ctx, _dev(sig), _dev(w), BETA, DENS).cpu().numpy()
    ref = kg.kg_dsf(sig, w, BETA, DENS)
    assert np.max(np.abs(S - ref) / np.abs(ref)) <= 1e-12
    ctx.close()


def test_kg_route_matches_oracle(tdx):
    from oracle import attenuation as att
    from oracle import eta as oeta
    from oracle import kubo_greenwood as kg
    from oracle.dielectric import dielectric
    from oracle.response import itcf
    w, sig = workloads.kg_conductivity(n_w=500)
    taus = np.linspace(0.0, 0.5 * BETA, 33)
    ctx = tdx.Context(0)
    wd, td = _dev(w), _dev(taus)
    S = tdx.kg_dsf(ctx, _dev(sig), wd, BETA, DENS)
    S_ref = kg.kg_dsf(sig, w, BETA, DENS)
    # F* and the eta metrics
    F = tdx.itcf(ctx, S, wd, BETA, td)
    F_ref = itcf(S_ref, w, BETA, taus)
    assert np.max(np.abs(F.cpu().numpy() - F_ref) / np.abs(F_ref)) <= 1e-12
    m = tdx.itcf_metrics(ctx, F, td, BETA, DENS).cpu().numpy()[0]
    m_ref = oeta.itcf_metrics(F_ref, taus, BETA, DENS)
    assert np.allclose(m, m_ref, rtol=1e-11, atol=1e-15 * np.max(np.abs(m_ref)))
    # the attenuation of S*: targets at the ripple, degree 2, six windows
    nu = _dev(np.array([20.0]))
    windows, degrees = [11, 17, 23, 29, 35, 41], [2] * 6
    r = tdx.attenuate(ctx, S, wd, BETA, td, windows, degrees, nu)
    sc, rs = [], []
    for win in windows:
        Sp = att.sg_filter(S_ref, win, 2)
        sc.append(att.sg_scores(S_ref, Sp, att.sg_hat_diag(len(w), win, 2), w, [20.0]))
        rs.append(att.residual_itcf(F_ref, itcf(Sp, w, BETA, taus), taus, BETA))
    b = att.sg_select(np.array(sc), np.array(rs), len(w))
    assert r.best[2] == b
    # the way back from the selected (else the unfiltered) S*
    pick = b if b >= 0 else None
    Sp_dev = r.Sp[pick] if pick is not None else S
    Sp_ref = att.sg_filter(S_ref, windows[pick], 2) if pick is not None else S_ref
    chi, eps_inv, sigma = (x.cpu().numpy() for x in tdx.kg_dielectric(ctx, Sp_dev, wd, BETA, DENS))
    chi_r, eps_r, sig_r = dielectric(Sp_ref, w, BETA, DENS, kg.KG_Q2)
    for a, c in ((chi, chi_r), (eps_inv, eps_r), (sigma, sig_r)):
        assert np.max(np.abs(a - c)) <= 1e-10 * np.max(np.abs(c))
    assert np.allclose(eps_inv, 1.0 + chi, atol=1e-14)
    ctx.close()
