"""HIP path against the FP64 oracle on identical seeded inputs.

Bars: FP64 path 1e-10 relative on S(q,w) (normwise and pointwise where
S > 1e-3 max S) and on F(q,tau) pointwise; FP32 and split-BF16 chi0 at
1e-4.  Integer work (band counts, transition lists) is compared exactly.
Eigenvector phases make pair densities non-unique, so they are compared
only through chi0, which is unique.
"""
import math
import sys

import numpy as np
import pytest

import pairing_rule
import workloads

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-10, "fp32": 1e-4, "bf16x3": 1e-4}


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


_oracle_cache = {}


def oracle_run(name):
    if name not in _oracle_cache:
        import oracle
        w = workloads.get(name)
        st = oracle.build_states(w)
        _oracle_cache[name] = (w, st, [oracle.run_q(w, st, iq) for iq in range(len(w.qs))])
    return _oracle_cache[name]


def _perm(gpu_basis, ora_basis):
    """index into the oracle basis for each GPU basis vector"""
    pos = {tuple(x): i for i, x in enumerate(ora_basis)}
    return np.array([pos[tuple(x)] for x in gpu_basis])


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def s_errors(S, Sref):
    S, Sref = np.asarray(S), np.asarray(Sref)
    norm = np.max(np.abs(S - Sref)) / np.max(np.abs(Sref))
    mask = Sref > 1e-3 * Sref.max()
    point = np.max(np.abs(S[mask] - Sref[mask]) / Sref[mask])
    return norm, point


@pytest.mark.parametrize("name", ["feg_tiny", "fcc_small", "h_tiny"])
def test_states_match_oracle(tdx, ctx, name):
    _say("states", name)
    w, ost, _ = oracle_run(name)
    st = tdx.build_states(ctx, w, w.temperatures[0])
    nb = st.nb.cpu().numpy()
    assert list(nb) == [len(e) for e in ost.eps]
    eps = st.eps.cpu().numpy()
    for k in range(w.n_k):
        assert np.max(np.abs(eps[k, : nb[k]] - ost.eps[k])) < 1e-11
    assert abs(st.mu - ost.mu) < 1e-12
    occ = st.occ.cpu().numpy()
    for k in range(w.n_k):
        assert np.max(np.abs(occ[k, : nb[k]] - ost.occ[k])) < 1e-12


@pytest.mark.parametrize("name", ["feg_tiny", "fcc_small", "h_tiny"])
def test_transitions_match_oracle_exactly(tdx, ctx, name):
    _say("transitions", name)
    w, ost, ores = oracle_run(name)
    st = tdx.build_states(ctx, w, w.temperatures[0])
    for iq, r in enumerate(ores):
        if w.temperatures[iq] != st.temperature:
            tdx.occupations(ctx, st, w.temperatures[iq], w.n_electrons, w.f_trunc)
        tr = tdx.transitions(ctx, st, w.qs[iq], w.f_trans_thr)
        assert len(tr) == len(r.tr)
        n = len(tr)
        assert np.array_equal(tr.k[:n].cpu().numpy(), r.tr.k)
        assert np.array_equal(tr.n[:n].cpu().numpy(), r.tr.n)
        assert np.array_equal(tr.m[:n].cpu().numpy(), r.tr.m)
        assert np.max(np.abs(tr.delta[:n].cpu().numpy() - r.tr.delta)) < 1e-11
        assert np.max(np.abs(tr.df[:n].cpu().numpy() - r.tr.df)) < 1e-12
        off = tr.k_offsets.cpu().numpy()
        assert off[-1] == n and np.all(np.diff(off) >= 0)


@pytest.mark.parametrize("name", ["feg_tiny", "fcc_small", "h_tiny"])
def test_paired_transitions_are_the_oracle_list_filtered(tdx, ctx, name):
    """The paired list is the oracle's full list restricted by the pairing
    rule, in the same order, bit for bit in the integers."""
    _say("paired transitions", name)
    w, ost, ores = oracle_run(name)
    st = tdx.build_states(ctx, w, w.temperatures[0])
    for iq, r in enumerate(ores):
        if w.temperatures[iq] != st.temperature:
            tdx.occupations(ctx, st, w.temperatures[iq], w.n_electrons, w.f_trunc)
        tr = tdx.transitions(ctx, st, w.qs[iq], w.f_trans_thr, paired=True)
        kt = pairing_rule.partner(w.kgrid, w.qs[iq])
        sel = pairing_rule.keep(r.tr.k, r.tr.n, r.tr.m, kt)
        n = len(tr)
        _say(f"  q{iq}: {len(r.tr)} -> {n}")
        assert n == int(sel.sum())
        assert np.array_equal(tr.k[:n].cpu().numpy(), r.tr.k[sel])
        assert np.array_equal(tr.n[:n].cpu().numpy(), r.tr.n[sel])
        assert np.array_equal(tr.m[:n].cpu().numpy(), r.tr.m[sel])
        assert np.max(np.abs(tr.delta[:n].cpu().numpy() - r.tr.delta[sel]), initial=0) < 1e-11
        assert np.max(np.abs(tr.df[:n].cpu().numpy() - r.tr.df[sel]), initial=0) < 1e-12
        off = tr.k_offsets.cpu().numpy()
        assert off[-1] == n and np.all(np.diff(off) >= 0)


@pytest.mark.parametrize("name,prec,paired", [("feg_tiny", "fp64", True),
                                              ("fcc_small", "fp64", True),
                                              ("h_tiny", "fp64", True),
                                              ("fcc_small", "fp64", False),
                                              ("fcc_small", "fp32", True),
                                              ("fcc_small", "bf16x3", True),
                                              ("fcc_small", "bf16x3", False),
                                              ("h_tiny", "fp32", True),
                                              ("h_tiny", "bf16x3", True)])
def test_pipeline_matches_oracle(tdx, ctx, name, prec, paired):
    """The oracle sums over the full screened set; the paired path contracts
    one transition per time-reversal pair with the combined weight."""
    _say("pipeline", name, prec, "paired" if paired else "full")
    w, ost, ores = oracle_run(name)
    st = tdx.build_states(ctx, w, w.temperatures[0])
    tol = TOL[prec]
    for iq, r in enumerate(ores):
        g = tdx.run_q(ctx, w, st, iq, prec=prec, paired=paired)
        p = _perm(g.basis, r.basis)
        ref = r.chi0[:, p][:, :, p]
        c0 = g.chi0.cpu().numpy()
        scale = np.max(np.abs(ref))
        err_c0 = np.max(np.abs(c0 - ref)) / scale
        K = g.K.cpu().numpy()
        err_k = np.max(np.abs(K - r.K[p][:, p])) / np.max(np.abs(r.K))
        norm, point = s_errors(g.S.cpu().numpy(), r.S)
        ferr = np.max(np.abs(g.F.cpu().numpy() - r.F) / r.F)
        _say(f"  q{iq} T={g.n_trans} NG={len(g.basis)} chi0 {err_c0:.2e} K {err_k:.2e} "
             f"S {norm:.2e}/{point:.2e} F {ferr:.2e}")
        assert err_k < 1e-12
        if paired:
            kt = pairing_rule.partner(w.kgrid, w.qs[iq])
            assert g.n_trans == int(pairing_rule.keep(r.tr.k, r.tr.n, r.tr.m, kt).sum())
        else:
            assert g.n_trans == len(r.tr)
        if prec == "fp64":
            assert err_c0 < 1e-12
        assert norm < tol and point < tol
        assert ferr < tol


def test_feg_c1_full_size_against_lindhard(tdx, ctx):
    """Full free-electron workload (8^3 k, 56 bands, 200 w): chi0_00 against
    the plane-wave Lindhard sum, chi_00 against the scalar RPA closed form,
    then S and F through the oracle's FDT and Laplace steps."""
    _say("feg_c1 full")
    import oracle
    from oracle import lindhard
    w = workloads.feg_c1()
    st = tdx.build_states(ctx, w)
    g = tdx.run_q(ctx, w, st, 0, prec="fp64")
    om = g.omega.cpu().numpy()
    ref, mu = lindhard.ksampled_chi0(w.cell, w.kgrid, w.ecut_wf, w.n_bands, w.qs[0], (0, 0, 0),
                                     om, w.eta, w.temperatures[0], w.n_electrons, w.f_trans_thr)
    assert abs(st.mu - mu) < 1e-12
    c0 = g.chi0.cpu().numpy()
    assert np.max(np.abs(c0[:, g.i_g0, g.i_g0] - ref)) < 1e-12 * np.max(np.abs(ref))
    v0 = 4 * math.pi / (2 * math.pi / 7.0) ** 2
    chi = ref / (1 - v0 * ref)
    S = oracle.dsf(chi, om, g.beta, g.density)
    F = oracle.itcf(S, om, g.beta, g.tau.cpu().numpy())
    norm, point = s_errors(g.S.cpu().numpy(), S)
    assert norm < 1e-10 and point < 1e-10
    assert np.max(np.abs(g.F.cpu().numpy() - F) / F) < 1e-10


def test_kernel_from_shared_xc_grid(tdx, ctx):
    """K assembled from one f_xc(G) grid per temperature equals the composed
    call bitwise and the oracle's K; fcc_small has a different temperature
    for each q, so the grid must follow the occupations."""
    _say("kernel from shared xc grid")
    import torch
    w, ost, ores = oracle_run("fcc_small")
    st = tdx.build_states(ctx, w, w.temperatures[0])
    grids = []
    for iq, r in enumerate(ores):
        T = w.temperatures[iq]
        if st.temperature != T:
            tdx.occupations(ctx, st, T, w.n_electrons, w.f_trunc)
        basis, _ = tdx.response_basis(w.cell, w.kgrid, w.qs[iq], w.ecut_chi[iq])
        gb = torch.from_numpy(basis).cuda()
        fx = tdx.xc_kernel_grid(ctx, st, w.dens_grid)
        grids.append(fx)
        for qj in w.qs:   # one grid serves every q at this temperature
            b2, _ = tdx.response_basis(w.cell, w.kgrid, qj, w.ecut_chi[iq])
            g2 = torch.from_numpy(b2).cuda()
            assert torch.equal(tdx.kernel_matrix_from_grid(ctx, st, qj, g2, w.xc, w.dens_grid, fx),
                               tdx.kernel_matrix(ctx, st, qj, g2, w.xc, w.dens_grid))
        K = tdx.kernel_matrix_from_grid(ctx, st, w.qs[iq], gb, w.xc, w.dens_grid, fx).cpu().numpy()
        p = _perm(basis, r.basis)
        assert np.max(np.abs(K - r.K[p][:, p])) < 1e-12 * np.max(np.abs(r.K))
    assert not torch.equal(grids[0], grids[1])
    # RPA needs no grid
    wr = workloads.h_tiny()
    sr = tdx.build_states(ctx, wr)
    basis, _ = tdx.response_basis(wr.cell, wr.kgrid, wr.qs[0], wr.ecut_chi[0])
    gb = torch.from_numpy(basis).cuda()
    assert torch.equal(tdx.kernel_matrix_from_grid(ctx, sr, wr.qs[0], gb, "rpa"),
                       tdx.kernel_matrix(ctx, sr, wr.qs[0], gb, "rpa"))


def test_chi0_is_bitwise_reproducible(tdx, ctx):
    _say("determinism")
    import torch
    w = workloads.fcc_small()
    st = tdx.build_states(ctx, w)
    for prec in ("fp64", "fp32", "bf16x3"):
        a = tdx.run_q(ctx, w, st, 0, prec=prec)
        b = tdx.run_q(ctx, w, st, 0, prec=prec)
        assert torch.equal(a.chi0, b.chi0)
        assert torch.equal(a.S, b.S)


def test_singular_dyson_is_reported(tdx, ctx):
    import torch
    n = 8
    c0 = torch.eye(n, dtype=torch.complex128, device="cuda").repeat(3, 1, 1).contiguous()
    K = torch.eye(n, dtype=torch.complex128, device="cuda")
    with pytest.raises(tdx.TdxError) as e:
        tdx.dyson(ctx, c0, K, 0)
    assert e.value.code == tdx.ERR_NUMERIC


def test_workspace_limit_is_enforced(tdx):
    import torch
    c = tdx.Context(0)
    c.set_workspace_limit(1024)
    w = workloads.fcc_small()
    with pytest.raises(tdx.TdxError) as e:
        tdx.build_states(c, w)
    assert e.value.code == tdx.ERR_ALLOC
    c.close()
