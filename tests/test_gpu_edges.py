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


@pytest.mark.parametrize("variant", [0, 2, None])
def test_whole_last_block_as_tail_rows(tdx, ctx, crystal, variant):
    """A basis of whole 16-row blocks whose last block would make a column
    tile of its own runs that block as 16 tail rows (N_G = 80: five blocks,
    4 + 1 for the 4 x 4 tile of variant 0, 2 + 2 + 1 for the 4 x 2 tile of
    variant 2, so both take the tail rows; the default 2 x 9 tile covers all
    five in one).  chi0 in the
    grid and persistent forms against the oracle on q2 of the crystal."""
    import torch
    w0, st, ost, _, _, _ = crystal
    w = w0.with_(qs=(w0.qs[2],), ecut_chi=(6.0,), temperatures=(w0.temperatures[2],),
                 omega_max=(w0.omega_max[2],))
    basis, _ = tdx.response_basis(w.cell, w.kgrid, w.qs[0], w.ecut_chi[0])
    n_g = len(basis)
    assert n_g == 80
    _say(f"whole last block: N_G {n_g}, variant {variant}")
    omegas = w.omega_grid(0)[::7]
    obasis, ref = _oracle_chi0(ost, w, None, omegas)
    pos = {tuple(x): i for i, x in enumerate(obasis)}
    p = np.array([pos[tuple(x)] for x in basis])
    ref = ref[:, p][:, :, p]
    tdx.occupations(ctx, st, w.temperatures[0], w.n_electrons, w.f_trunc)
    tr = tdx.transitions(ctx, st, w.qs[0], w.f_trans_thr)
    gb = torch.from_numpy(basis).cuda()
    om = torch.as_tensor(omegas, device="cuda")
    v0, sl0 = tdx.chi0_get_config(ctx, n_g)
    if variant is not None:
        tdx.chi0_set_config(ctx, n_g, variant, sl0)
    try:
        P = tdx.pair_density(ctx, st, w.qs[0], tr, gb, "bf16x3")
        c0 = tdx.chi0(ctx, tr, P, n_g, "bf16x3", om, w.eta, st.chi0_pref)
        it = tdx.Chi0Item(tr, P, n_g, om, w.eta, st.chi0_pref)
        plan = tdx.Chi0Plan(ctx, [it], "bf16x3")
        plan.launch()
        torch.cuda.synchronize()
        c1 = it.out.clone()
        plan.close()
    finally:
        tdx.chi0_set_config(ctx, n_g, v0, sl0)
        tdx.occupations(ctx, st, w0.temperatures[0], w0.n_electrons, w0.f_trunc)
    for name, c in (("grid", c0), ("persistent", c1)):
        c = c.cpu().numpy()
        err = np.max(np.abs(c - ref)) / np.max(np.abs(ref))
        _say(f"  {name}: {err:.2e}")
        assert err < 1e-4


def test_slicing_query_matches_the_launch(tdx, ctx, crystal):
    """The host query tdx_chi0_bf16x3_slicing returns the slice length the
    launch takes by itself: fixing the context's slice length to it gives
    bitwise the chi0 of the automatic choice (another length would change
    the rounding order of the FP32 runs and the FP64 slice reduction)."""
    import torch
    w, st, _, basis, _, gb = crystal
    n_g = len(basis)
    tr = tdx.transitions(ctx, st, w.qs[0], w.f_trans_thr)
    om = torch.as_tensor(w.omega_grid(0), device="cuda")
    P = tdx.pair_density(ctx, st, w.qs[0], tr, gb, "bf16x3")
    auto = tdx.chi0(ctx, tr, P, n_g, "bf16x3", om, w.eta, st.chi0_pref)
    v, sl = tdx.chi0_get_config(ctx, n_g)
    v = 9 if v < 0 else v  # the default tile
    n_cu = torch.cuda.get_device_properties(0).multi_processor_count
    length, ns = tdx.chi0_bf16x3_slicing(n_cu, v, len(tr), n_g, om.shape[0], sl)
    _say(f"slicing query: {len(tr)} transitions, N_G {n_g}, {om.shape[0]} frequencies, "
         f"{n_cu} CUs -> {ns} slices of {length}")
    tdx.chi0_set_slice_length(ctx, length)
    try:
        fixed = tdx.chi0(ctx, tr, P, n_g, "bf16x3", om, w.eta, st.chi0_pref)
    finally:
        tdx.chi0_set_slice_length(ctx, 0)
    assert torch.equal(auto, fixed)
