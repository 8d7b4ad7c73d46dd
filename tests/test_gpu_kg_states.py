"""The Kubo-Greenwood conductivity of the states on the GPU (Sec. A.3's
starting point) against the oracle, and the whole route from it: sigma for a
set of broadenings -> S* -> F* -> the eta metrics and the reference eta, the
oracle composing the same steps.  At the benchmark crystal's size (16^3 k,
200 bands) the size-independent properties: sigma(-w) = conj(sigma(w)) and
Re sigma > 0."""
import time

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


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


@pytest.mark.parametrize("name", ["fcc_small", "h_tiny"])
def test_conductivity_matches_oracle(tdx, name):
    import oracle
    from oracle import kubo_greenwood as kg
    w = getattr(workloads, name)()
    ctx = tdx.Context(0)
    st = tdx.build_states(ctx, w)
    ost = oracle.build_states(w)
    om = np.linspace(-1.0, 4.0, 301)
    for eta in (w.eta, 4 * w.eta):
        s = tdx.kg_conductivity(ctx, st, _dev(om), eta, w.f_trans_thr).cpu().numpy()
        ref = kg.kg_conductivity(ost, om, eta, w.f_trans_thr)
        err = np.max(np.abs(s - ref)) / np.max(np.abs(ref))
        print(f"{name} eta {eta:.4f}: sigma err {err:.2e}, max |sigma| {np.max(np.abs(ref)):.3e}",
              flush=True)
        assert err <= 1e-10
    ctx.close()


def test_free_electrons_give_zero(tdx):
    w = workloads.feg_tiny()
    ctx = tdx.Context(0)
    st = tdx.build_states(ctx, w)
    s = tdx.kg_conductivity(ctx, st, _dev(np.linspace(0.0, 3.0, 31)), w.eta, w.f_trans_thr)
    assert float(s.abs().max()) < 1e-12
    ctx.close()


def test_eta_test_from_the_conductivity_matches_oracle(tdx):
    """The eta-convergence test in imaginary time started from sigma_KG of
    the states: for 6 broadenings, S*, F*, the metrics and the reference."""
    import oracle
    from oracle import eta as oeta
    from oracle import kubo_greenwood as kg
    from oracle.response import itcf
    w = workloads.fcc_small()
    ctx = tdx.Context(0)
    st = tdx.build_states(ctx, w)
    ost = oracle.build_states(w)
    om = w.omega_grid(0)
    taus = w.tau_grid(0)
    beta, n = 1.0 / w.temperatures[0], w.n_electrons / ost.omega
    etas = w.eta * 2.0 ** np.arange(-2, 4)
    omd, td = _dev(om), _dev(taus)
    tr = tdx.transitions(ctx, st, (0, 0, 0), w.f_trans_thr)
    rows, rows_ref = [], []
    for eta in etas:
        sig = tdx.kg_conductivity(ctx, st, omd, eta, w.f_trans_thr, tr=tr)
        S = tdx.kg_dsf(ctx, sig, omd, st.beta, st.density)
        F = tdx.itcf(ctx, S, omd, st.beta, td)
        rows.append(tdx.itcf_metrics(ctx, F, td, st.beta, st.density).cpu().numpy()[0])
        S_ref = kg.kg_dsf(kg.kg_conductivity(ost, om, eta, w.f_trans_thr), om, beta, n)
        F_ref = itcf(S_ref, om, beta, taus)
        rows_ref.append(oeta.itcf_metrics(F_ref, taus, beta, n))
        err = np.max(np.abs(F.cpu().numpy() - F_ref) / np.abs(F_ref))
        print(f"eta {eta:.4f}: F* err {err:.2e}", flush=True)
        assert err <= 1e-10
    rows, rows_ref = np.array(rows), np.array(rows_ref)
    assert np.allclose(rows, rows_ref, rtol=1e-9, atol=1e-14 * np.max(np.abs(rows_ref)))
    assert tdx.eta_reference(rows, etas) == oeta.eta_reference(rows_ref, etas, 1e-2)
    ctx.close()


def test_errors_and_empty_list(tdx):
    import torch
    w = workloads.h_tiny()
    ctx = tdx.Context(0)
    st = tdx.build_states(ctx, w)
    om = _dev(np.linspace(0.0, 2.0, 11))
    pr = tdx.transitions(ctx, st, (0, 0, 0), w.f_trans_thr, paired=True)
    with pytest.raises(tdx.TdxError):
        tdx.kg_conductivity(ctx, st, om, w.eta, w.f_trans_thr, tr=pr)
    tr = tdx.transitions(ctx, st, (0, 0, 0), w.f_trans_thr)
    small = torch.empty(8, dtype=torch.uint8, device="cuda")
    with pytest.raises(tdx.TdxError):
        tdx.kg_conductivity(ctx, st, om, w.eta, w.f_trans_thr, tr=tr, work=small)
    with pytest.raises(tdx.TdxError):
        tdx.kg_conductivity(ctx, st, om, -1.0, w.f_trans_thr, tr=tr)
    # a screening threshold above every occupation difference: no transitions
    s = tdx.kg_conductivity(ctx, st, om, w.eta, 2.0)
    assert float(s.abs().max()) == 0.0
    ctx.close()


@pytest.mark.timeout(300)
def test_crystal_at_full_size(tdx):
    import torch
    w = workloads.fcc_c2()
    ctx = tdx.Context(0)
    st = tdx.build_states(ctx, w, w.temperatures[0])
    om = w.omega_grid(0)[1:]
    tr = tdx.transitions(ctx, st, (0, 0, 0), w.f_trans_thr)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sp = tdx.kg_conductivity(ctx, st, _dev(om), w.eta, w.f_trans_thr, tr=tr)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    sm = tdx.kg_conductivity(ctx, st, _dev(-om), w.eta, w.f_trans_thr, tr=tr)
    sp, sm = sp.cpu().numpy(), sm.cpu().numpy()
    print(f"fcc_c2: {len(tr)} transitions at q = 0, {len(om)} frequencies, {dt * 1e3:.1f} ms; "
          f"max Re sigma {sp.real.max():.4e}", flush=True)
    assert np.all(np.isfinite(sp))
    assert np.max(np.abs(sm - sp.conj())) <= 1e-12 * np.max(np.abs(sp))
    assert np.all(sp.real > 0)
    ctx.close()
