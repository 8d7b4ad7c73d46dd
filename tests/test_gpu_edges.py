"""Edge cases of the response path on the GPU: an empty transition set, a
single frequency off zero, and a transition count smaller than one chunk of
every chi0 kernel (37: a ragged tail in the first and only chunk)."""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


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


@pytest.fixture(scope="module")
def crystal(tdx, ctx):
    import torch
    import oracle
    w = workloads.fcc_small()
    st = tdx.build_states(ctx, w, w.temperatures[0])
    ost = oracle.build_states(w)
    basis, g0 = tdx.response_basis(w.cell, w.kgrid, w.qs[0], w.ecut_chi[0])
    return w, st, ost, basis, g0, torch.from_numpy(basis).cuda()


def test_empty_transition_set_gives_zero_response(tdx, ctx, crystal):
    """|f_n - f_m| <= 1 always, so a threshold of 2 keeps nothing: chi0, chi,
    S and F are exactly zero in every precision."""
    import torch
    _say("empty")
    w, st, _, basis, g0, gb = crystal
    tr = tdx.transitions(ctx, st, w.qs[0], 2.0)
    assert len(tr) == 0
    om = torch.as_tensor(w.omega_grid(0), device="cuda")
    K = tdx.kernel_matrix(ctx, st, w.qs[0], gb, w.xc, w.dens_grid)
    tau = torch.as_tensor(w.tau_grid(0), device="cuda")
    for prec in ("fp64", "fp32", "bf16x3"):
        P = tdx.pair_density(ctx, st, w.qs[0], tr, gb, prec)
        c0 = tdx.chi0(ctx, tr, P, len(basis), prec, om, w.eta, 1.0)
        assert int((c0 != 0).sum()) == 0
        c00 = tdx.dyson(ctx, c0, K, g0)
        S = tdx.dsf(ctx, c00, om, 1.0 / w.temperatures[0], 0.1)
        F = tdx.itcf(ctx, S, om, 1.0 / w.temperatures[0], tau)
        assert int((c00 != 0).sum()) == 0 and int((S != 0).sum()) == 0
        assert int((F != 0).sum()) == 0


def _oracle_chi0(ost, w, n_trans, omegas):
    from oracle.lattice import response_basis
    from oracle.response import Transitions, chi0, pair_densities, transitions
    st = ost.with_temperature(w.temperatures[0])
    qred = np.asarray(w.qs[0], dtype=np.float64) / np.asarray(w.kgrid)
    basis, _ = response_basis(st.B, qred, w.ecut_chi[0])
    tr = transitions(st, w.qs[0], w.f_trans_thr)
    if n_trans is not None:
        tr = Transitions(*(getattr(tr, f)[:n_trans] for f in ("k", "kp", "n", "m", "delta", "df")))
    P = pair_densities(st, tr, w.qs[0], basis)
    return basis, chi0(tr, P, omegas, w.eta, st.n_k, st.omega)


@pytest.mark.parametrize("case", ["single_frequency", "sub_chunk"])
def test_small_cases_match_the_oracle(tdx, ctx, crystal, case):
    import torch
    _say(case)
    w, st, ost, basis, _, gb = crystal
    tr = tdx.transitions(ctx, st, w.qs[0], w.f_trans_thr)
    if case == "single_frequency":
        omegas, nt = np.array([0.37]), None
    else:
        omegas, nt = w.omega_grid(0)[:21], 37
        assert len(tr) > nt
    obasis, ref = _oracle_chi0(ost, w, nt, omegas)
    pos = {tuple(x): i for i, x in enumerate(obasis)}
    p = np.array([pos[tuple(x)] for x in basis])
    ref = ref[:, p][:, :, p]
    om = torch.as_tensor(omegas, device="cuda")
    pref = st.chi0_pref
    for prec, tol in (("fp64", 1e-10), ("fp32", 1e-4), ("bf16x3", 1e-4)):
        P = tdx.pair_density(ctx, st, w.qs[0], tr, gb, prec, n_trans=nt)
        c0 = tdx.chi0(ctx, tr, P, len(basis), prec, om, w.eta, pref, n_trans=nt).cpu().numpy()
        err = np.max(np.abs(c0 - ref)) / np.max(np.abs(ref))
        _say(f"  {prec}: {err:.2e}")
        assert err < tol
