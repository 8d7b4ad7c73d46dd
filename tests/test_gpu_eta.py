"""The eta-convergence test in imaginary time (Sec. 2, Eq. 2) on the GPU
against the oracle: the metrics kernel on given ITCFs, the reference-eta
rule, and a whole eta scan (chi0 for every eta from one set of pair
densities, Dyson, S, F, metrics) in FP64 (1e-10) and split-BF16 (1e-4)."""
import sys

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def tdx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2510_01875_amd as m
    return m


@pytest.fixture(scope="module")
def ctx(tdx):
    c = tdx.Context(0)
    yield c
    c.close()


def test_metrics_kernel_matches_the_oracle(tdx, ctx):
    import torch
    from oracle import eta as oeta
    rng = np.random.default_rng(3)
    beta, n = 2.7, 0.04
    for npts, end in ((65, beta), (33, beta / 2)):
        taus = np.linspace(0.0, end, npts)
        F = rng.uniform(0.1, 1.0, size=(5, npts))
        got = tdx.itcf_metrics(ctx, torch.as_tensor(F, device="cuda"),
                               torch.as_tensor(taus, device="cuda"), beta, n).cpu().numpy()
        ref = np.array([oeta.itcf_metrics(f, taus, beta, n) for f in F])
        assert np.max(np.abs(got - ref) / np.abs(ref)) < 1e-14
    bad = torch.as_tensor(np.linspace(0.0, 0.9 * beta, 40), device="cuda")
    m = tdx.itcf_metrics(ctx, torch.ones((2, 40), dtype=torch.float64, device="cuda"), bad,
                         beta, n)
    assert torch.isnan(m).all()


def test_reference_rule_matches_the_oracle(tdx):
    from oracle import eta as oeta
    rng = np.random.default_rng(5)
    etas = np.array([0.05, 0.1, 0.2, 0.4, 0.8])
    for _ in range(20):
        m = np.tile(rng.uniform(-1, 1, 5), (5, 1)) * (1 + rng.uniform(-0.02, 0.02, (5, 5)))
        assert tdx.eta_reference(m, etas, 1e-2) == oeta.eta_reference(m, etas, 1e-2)
    with pytest.raises(tdx.TdxError):
        tdx.eta_reference(np.zeros((2, 5)), np.array([0.2, 0.1]), 1e-2)


def test_eta_scan_matches_the_oracle(tdx, ctx):
    import oracle
    from oracle import eta as oeta
    w = workloads.fcc_small()
    etas = w.eta * np.array([0.25, 0.5, 1.0, 2.0, 4.0])
    st = tdx.build_states(ctx, w, w.temperatures[0])
    g = tdx.eta_scan(ctx, w, st, 0, etas, prec="fp64", tol=2e-2)
    ost = oracle.build_states(w)
    ref_m = []
    for i, e in enumerate(etas):
        r = oracle.run_q(w.with_(eta=float(e)), ost, 0, keep=False)
        S, F = g.S[i].cpu().numpy(), g.F[i].cpu().numpy()
        assert np.max(np.abs(S - r.S)) < 1e-10 * np.max(np.abs(r.S))
        assert np.max(np.abs(F - r.F) / np.abs(r.F)) < 1e-10
        ref_m.append(oeta.itcf_metrics(r.F, r.taus, r.beta, r.density))
    ref_m = np.array(ref_m)
    err = np.max(np.abs(g.metrics - ref_m) / np.abs(ref_m))
    ref_i = oeta.eta_reference(ref_m, etas, 2e-2)
    _say(f"  fcc_small q0, {len(etas)} eta: metrics vs oracle {err:.1e}; reference eta "
         f"{etas[g.ref_index]:.4f} (oracle {etas[ref_i]:.4f})")
    for i, e in enumerate(etas):
        _say("   eta %.4f: " % e + "  ".join(f"{v: .5e}" for v in g.metrics[i]))
    assert err < 1e-10
    assert g.ref_index == ref_i
    # split-BF16: the same scan from one persistent launch for all eta
    b = tdx.eta_scan(ctx, w, st, 0, etas, prec="bf16x3", tol=2e-2)
    e16 = np.max(np.abs(b.metrics - g.metrics) / np.abs(g.metrics))
    _say(f"  split-BF16 scan vs FP64: metrics {e16:.1e}, reference index {b.ref_index}")
    assert e16 < 1e-4
