"""Ragged batches in one persistent launch, HIP-graph replay and the tile
autotuner, checked against the single-q path and the FP64 oracle."""
import os
import sys
import tempfile

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


def _prepare(tdx, ctx, w, st, prec, paired=False):
    """Per-q transitions, pair densities and batch items (occupations at each
    q's temperature are taken before its transitions)."""
    import torch
    out = []
    for iq in range(len(w.qs)):
        T = w.temperatures[iq]
        tdx.occupations(ctx, st, T, w.n_electrons, w.f_trunc)
        basis, g0 = tdx.response_basis(w.cell, w.kgrid, w.qs[iq], w.ecut_chi[iq])
        gb = torch.from_numpy(basis).cuda()
        tr = tdx.transitions(ctx, st, w.qs[iq], w.f_trans_thr, paired=paired)
        P = tdx.pair_density(ctx, st, w.qs[iq], tr, gb, prec)
        om = torch.as_tensor(w.omega_grid(iq), device="cuda")
        K = tdx.kernel_matrix(ctx, st, w.qs[iq], gb, w.xc, w.dens_grid)
        item = tdx.Chi0Item(tr, P, len(basis), om, w.eta, st.chi0_pref)
        out.append(dict(iq=iq, basis=basis, g0=g0, gb=gb, tr=tr, P=P, om=om, K=K, item=item))
    return out


@pytest.mark.parametrize("paired", [False, True])
def test_batched_persistent_matches_single_and_oracle(tdx, ctx, paired):
    """Six q with ragged transition counts (T from 1 to 8 eV) in one
    persistent launch: bitwise equal to one launch per q with the same tile
    configuration, and within the split-BF16 bar of the oracle (whose sum is
    over the full list also when the batch contracts paired lists)."""
    import torch
    import oracle
    _say("batched", "paired" if paired else "full")
    w = workloads.fcc_c4_small()
    st = tdx.build_states(ctx, w)
    prep = _prepare(tdx, ctx, w, st, "bf16x3", paired)
    counts = [len(p["tr"]) for p in prep]
    assert max(counts) > 1.5 * min(counts)
    tdx.chi0_batched(ctx, [p["item"] for p in prep], "bf16x3")
    ost = oracle.build_states(w)
    for p in prep:
        single = tdx.chi0(ctx, p["tr"], p["P"], len(p["basis"]), "bf16x3", p["om"], w.eta,
                          st.chi0_pref)
        assert torch.equal(single, p["item"].out)
        r = oracle.run_q(w, ost, p["iq"])
        pos = {tuple(x): i for i, x in enumerate(r.basis)}
        perm = np.array([pos[tuple(x)] for x in p["basis"]])
        ref = r.chi0[:, perm][:, :, perm]
        err = np.max(np.abs(p["item"].out.cpu().numpy() - ref)) / np.max(np.abs(ref))
        _say(f"  q{p['iq']} T={len(p['tr'])} chi0 err {err:.2e}")
        assert err < 1e-4


def test_plan_replays_in_a_hip_graph(tdx, ctx):
    """Pair densities + chi0 plan + Dyson + S + F for every q captured once
    and replayed; each replay, with eager work between replays and the pair
    densities and chi0 cleared before it, equals the eager result."""
    import torch
    _say("graph")
    w = workloads.fcc_c4_small()
    st = tdx.build_states(ctx, w)
    prep = _prepare(tdx, ctx, w, st, "bf16x3")
    plan = tdx.Chi0Plan(ctx, [p["item"] for p in prep], "bf16x3")
    for p in prep:
        n_w, n_g = p["om"].shape[0], len(p["basis"])
        p["work"] = torch.empty(tdx.dyson_work_bytes(n_g, n_w), dtype=torch.uint8, device="cuda")
        p["info"] = torch.empty(n_w, dtype=torch.int32, device="cuda")
        p["chi00"] = torch.empty(n_w, dtype=torch.complex128, device="cuda")
        p["tau"] = torch.as_tensor(w.tau_grid(p["iq"]), device="cuda")
        p["pdw"] = torch.empty(tdx.pair_density_work_bytes(st, len(p["tr"])), dtype=torch.uint8,
                               device="cuda")
    dens = st.density

    def body():
        for p in prep:
            tdx.pair_density_async(ctx, st, w.qs[p["iq"]], p["tr"], p["gb"], p["P"], p["pdw"],
                                   "bf16x3")
        plan.launch()
        outs = []
        for p in prep:
            tdx.dyson_async(ctx, p["item"].out, p["K"], p["g0"], p["chi00"], p["work"], p["info"])
            beta = 1.0 / w.temperatures[p["iq"]]
            S = tdx.dsf(ctx, p["chi00"], p["om"], beta, dens)
            outs.append((S, tdx.itcf(ctx, S, p["om"], beta, p["tau"])))
        return outs

    eager = [(S.clone(), F.clone()) for S, F in body()]
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        body()                          # warm-up on the side stream
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        captured = body()
    for rep in range(3):
        for p in prep:
            p["item"].out.zero_()
            p["chi00"].zero_()
            p["P"].zero_()
        g.replay()
        torch.cuda.synchronize()
        for (S, F), (Se, Fe) in zip(captured, eager):
            assert torch.equal(S, Se) and torch.equal(F, Fe)
        assert all(int(p["info"].abs().max()) == 0 for p in prep)
        junk = torch.randn(1 << 16, device="cuda") @ torch.randn(1 << 16, 8, device="cuda")
        torch.cuda.synchronize()
    plan.close()


def test_autotuner_picks_a_variant_and_round_trips_the_cache(tdx, ctx):
    import torch
    _say("autotune")
    w = workloads.fcc_small()
    st = tdx.build_states(ctx, w)
    p = _prepare(tdx, ctx, w.with_(qs=w.qs[:1], temperatures=w.temperatures[:1]), st,
                 "bf16x3")[0]
    n_g = len(p["basis"])
    v, sl, ms = tdx.autotune_chi0(ctx, p["item"])
    _say(f"  best variant {v} slice 2^{sl} {ms:.3f} ms")
    assert 0 <= v < tdx.chi0_variants("bf16x3") and sl in (18, 20) and ms > 0
    assert tdx.chi0_get_config(ctx, n_g) == (v, sl)
    path = os.path.join(tempfile.mkdtemp(), "tune.json")
    tdx.tune_save(ctx, path)
    c2 = tdx.Context(0)
    tdx.tune_load(c2, path)
    assert tdx.chi0_get_config(c2, n_g) == (v, sl)
    c2.close()
    # a probe truncated below its buffer's row count: the plans the tuner
    # times must read the FP32 rows where the buffer holds them
    nt = len(p["tr"]) // 3
    tdx.autotune_chi0(ctx, p["item"], max_trans=nt)
    P_nt = tdx.pair_density(ctx, st, w.qs[0], p["tr"], p["gb"], "bf16x3", n_trans=nt)
    tdx.chi0_set_config(ctx, n_g, -1, 20)
    a = tdx.Chi0Item(p["tr"], p["P"], n_g, p["om"], w.eta, st.chi0_pref, n_trans=nt,
                     p_rows=len(p["tr"]))
    b = tdx.Chi0Item(p["tr"], P_nt, n_g, p["om"], w.eta, st.chi0_pref, n_trans=nt)
    tdx.chi0_batched(ctx, [a, b], "bf16x3")
    ref_nt = tdx.chi0(ctx, p["tr"], P_nt, n_g, "bf16x3", p["om"], w.eta, st.chi0_pref,
                      n_trans=nt)
    _say(f"  truncated probe: {nt} of {len(p['tr'])} transitions")
    assert torch.equal(a.out, b.out) and torch.equal(a.out, ref_nt)
    err = float((p["item"].out - ref_nt).abs().max() / ref_nt.abs().max())
    assert err < 1e-5, err
    # every variant gives the same chi0 to the split-BF16 bar
    ref = None
    for var in range(tdx.chi0_variants("bf16x3")):
        tdx.chi0_set_config(ctx, n_g, var, 18)
        c = tdx.chi0(ctx, p["tr"], p["P"], n_g, "bf16x3", p["om"], w.eta,
                     st.chi0_pref)
        if ref is None:
            ref = c.clone()
        err = float((c - ref).abs().max() / ref.abs().max())
        _say(f"  variant {var} vs 0: {err:.2e}")
        assert err < 1e-5
    tdx.chi0_set_config(ctx, n_g, -1, 20)


@pytest.mark.parametrize("prec,tol", [("fp32", 1e-5), ("fp64", 1e-12)])
def test_fp_variants_tune_and_match_oracle(tdx, ctx, prec, tol):
    """The FP32 and FP64 tile variants: every one within the precision's bar
    of the oracle (N_G = 119: 8 column blocks in 2 to 4 column tiles, ragged
    last ones among them, and several slices), the autotuner's choice stored
    per precision beside the split-BF16 entry and kept through a save and
    load of the cache."""
    import oracle
    _say("fp variants", prec)
    w = workloads.fcc_small()
    w = w.with_(ecut_chi=(w.ecut_chi[0], 8.0, w.ecut_chi[2]))
    st = tdx.build_states(ctx, w)
    p = _prepare(tdx, ctx, w.with_(qs=w.qs[1:2], temperatures=w.temperatures[1:2],
                                   ecut_chi=w.ecut_chi[1:2], omega_max=w.omega_max[1:2]), st,
                 prec)[0]
    n_g = len(p["basis"])
    assert n_g == 119
    ost = oracle.build_states(w.with_(temperatures=w.temperatures[1:2]))
    r = oracle.run_q(w, ost, 1)
    pos = {tuple(x): i for i, x in enumerate(r.basis)}
    perm = np.array([pos[tuple(x)] for x in p["basis"]])
    ref = r.chi0[:, perm][:, :, perm]
    n_var = tdx.chi0_variants(prec)
    assert n_var >= 4
    tdx.chi0_set_slice_length(ctx, 512)  # several slices at this size
    for var in range(n_var):
        tdx.chi0_set_config(ctx, n_g, var, 20, prec)
        assert tdx.chi0_get_config(ctx, n_g, prec)[0] == var
        c = tdx.chi0(ctx, p["tr"], p["P"], n_g, prec, p["om"], w.eta, st.chi0_pref).cpu().numpy()
        err = np.max(np.abs(c - ref)) / np.max(np.abs(ref))
        _say(f"  {prec} variant {var}: chi0 err {err:.2e}")
        assert err < tol
    tdx.chi0_set_slice_length(ctx, 0)
    tdx.chi0_set_config(ctx, n_g, -1, 20, prec)
    v, _, ms = tdx.autotune_chi0(ctx, p["item"], prec=prec)
    _say(f"  {prec} best variant {v}, {ms:.3f} ms")
    assert 0 <= v < n_var and ms > 0
    assert tdx.chi0_get_config(ctx, n_g, prec)[0] == v
    tdx.chi0_set_config(ctx, n_g, 3, 18, "bf16x3")
    path = os.path.join(tempfile.mkdtemp(), "tune.json")
    tdx.tune_save(ctx, path)
    c2 = tdx.Context(0)
    tdx.tune_load(c2, path)
    assert tdx.chi0_get_config(c2, n_g, prec)[0] == v
    assert tdx.chi0_get_config(c2, n_g, "bf16x3") == (3, 18)
    c2.close()
    tdx.chi0_set_config(ctx, n_g, -1, 20, "bf16x3")
    tdx.chi0_set_config(ctx, n_g, -1, 20, prec)
