"""The benchmarked kernels against the FP64 oracle, element by element.

The benchmark's crystal (fcc_c2: 16^3 k, 200 bands, E_chi = 8.5 Ha, ALDA) is
taken on a 4^3 grid, where the oracle finishes in seconds, with two q:
q0 = (2 pi / a)(1/2, 0, 0) of the benchmark, N_G = 133 (row stride 144: the
tuned split-BF16 tile of the benchmark, 8 waves of 2 frequencies x 9 column
blocks; the FP32/FP64 tiles with three 48-column tiles), and
q = (2 pi / a)(1, 0, 0), N_G = 116 (stride 128: a ragged last column tile).
Each precision runs over the full and the time-reversal paired list, as one
grid launch and as a one-item persistent plan, with the slice length chosen
per call (as the benchmark runs it) and with slices of 2^17 transitions
(several FP32 runs folded into one FP64 partial: 32 for FP32, up to four for
split-BF16).

Bars: chi0 against the oracle's chi0 (relative to its largest element)
1e-12 for FP64, 1e-4 for FP32 and split-BF16; K 1e-12; S normwise and
pointwise (S > 1e-3 max S) and F pointwise at 1e-10 (FP64) and 1e-4; the
transition lists bit-exact in their integers.
"""
import os

import numpy as np
import pytest

import pairing_rule
import workloads

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TUNE = os.path.join(ROOT, "paper_2510_01875_amd", "tune_gfx950.json")
TOL = {"fp64": 1e-10, "fp32": 1e-4, "bf16x3": 1e-4}
CHI0_TOL = {"fp64": 1e-12, "fp32": 1e-4, "bf16x3": 1e-4}
LONG_SLICE = 1 << 17


def _say(*a):
    print(*a, flush=True)


def sample():
    """fcc_c2 on a 4^3 grid, 64 frequencies on its [0, 2] Ha range."""
    w = workloads.fcc_c2()
    return w.with_(name="fcc_c2_k4", kgrid=(4, 4, 4), qs=((0, 1, 1), (0, 2, 2)),
                   temperatures=w.temperatures[:2], ecut_chi=w.ecut_chi[:2],
                   omega_max=w.omega_max[:2], n_omega=64)


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
    tdx.tune_load(c, TUNE)
    yield c
    c.close()


@pytest.fixture(scope="module")
def gpu_states(tdx, ctx):
    w = sample()
    return w, tdx.build_states(ctx, w)


_oracle = {}


def oracle_q(iq):
    if iq not in _oracle:
        import oracle
        w = sample()
        if "states" not in _oracle:
            _oracle["states"] = oracle.build_states(w)
        _say(f"  oracle q{iq} ...")
        _oracle[iq] = oracle.run_q(w, _oracle["states"], iq)
    return _oracle[iq]


def _perm(gpu_basis, ora_basis):
    pos = {tuple(x): i for i, x in enumerate(ora_basis)}
    return np.array([pos[tuple(x)] for x in gpu_basis])


def s_errors(S, Sref):
    norm = np.max(np.abs(S - Sref)) / np.max(np.abs(Sref))
    mask = Sref > 1e-3 * Sref.max()
    return norm, np.max(np.abs(S[mask] - Sref[mask]) / Sref[mask])


@pytest.mark.parametrize("iq", [0, 1])
def test_transitions_bit_exact(tdx, ctx, gpu_states, iq):
    w, st = gpu_states
    r = oracle_q(iq)
    _say(f"transitions q{iq}")
    tr = tdx.transitions(ctx, st, w.qs[iq], w.f_trans_thr)
    n = len(tr)
    assert n == len(r.tr)
    assert np.array_equal(tr.k[:n].cpu().numpy(), r.tr.k)
    assert np.array_equal(tr.n[:n].cpu().numpy(), r.tr.n)
    assert np.array_equal(tr.m[:n].cpu().numpy(), r.tr.m)
    assert np.max(np.abs(tr.delta[:n].cpu().numpy() - r.tr.delta)) < 1e-11
    assert np.max(np.abs(tr.df[:n].cpu().numpy() - r.tr.df)) < 1e-12
    tp = tdx.transitions(ctx, st, w.qs[iq], w.f_trans_thr, paired=True)
    sel = pairing_rule.keep(r.tr.k, r.tr.n, r.tr.m, pairing_rule.partner(w.kgrid, w.qs[iq]))
    npr = len(tp)
    _say(f"  {n} transitions, {npr} paired")
    assert npr == int(sel.sum())
    for a, b in ((tp.k, r.tr.k), (tp.n, r.tr.n), (tp.m, r.tr.m)):
        assert np.array_equal(a[:npr].cpu().numpy(), b[sel])


@pytest.mark.parametrize("iq", [0, 1])
@pytest.mark.parametrize("prec", ["bf16x3", "fp32", "fp64"])
@pytest.mark.parametrize("paired", [True, False])
def test_chi0_K_S_F_match_oracle(tdx, ctx, gpu_states, iq, prec, paired):
    import torch
    w, st = gpu_states
    r = oracle_q(iq)
    qj = w.qs[iq]
    basis, g0 = tdx.response_basis(w.cell, w.kgrid, qj, w.ecut_chi[iq])
    n_g = len(basis)
    _say(f"q{iq} N_G={n_g} {prec} {'paired' if paired else 'full'}")
    if prec == "bf16x3" and n_g == 133:
        # the tile the benchmark runs on this basis size
        assert tdx.chi0_get_config(ctx, n_g) == (9, 20)
    gb = torch.from_numpy(basis).cuda()
    tr = tdx.transitions(ctx, st, qj, w.f_trans_thr, paired=paired)
    P = tdx.pair_density(ctx, st, qj, tr, gb, prec)
    om = torch.as_tensor(w.omega_grid(iq), device="cuda")
    tau = torch.as_tensor(w.tau_grid(iq), device="cuda")
    K = tdx.kernel_matrix(ctx, st, qj, gb, w.xc, w.dens_grid)
    p = _perm(basis, r.basis)
    Kr = r.K[p][:, p]
    assert np.max(np.abs(K.cpu().numpy() - Kr)) < 1e-12 * np.max(np.abs(Kr))
    ref = r.chi0[:, p][:, :, p]
    scale = np.max(np.abs(ref))
    try:
        for slicing in (0, LONG_SLICE):
            tdx.chi0_set_slice_length(ctx, slicing)
            for form in ("grid", "persistent"):
                if form == "grid":
                    c0 = tdx.chi0(ctx, tr, P, n_g, prec, om, w.eta, st.chi0_pref)
                else:
                    item = tdx.Chi0Item(tr, P, n_g, om, w.eta, st.chi0_pref)
                    tdx.chi0_batched(ctx, [item], prec)
                    c0 = item.out
                err = np.max(np.abs(c0.cpu().numpy() - ref)) / scale
                c00 = tdx.dyson(ctx, c0, K, g0)
                S = tdx.dsf(ctx, c00, om, st.beta, st.density).cpu().numpy()
                F = tdx.itcf(ctx, tdx.dsf(ctx, c00, om, st.beta, st.density), om, st.beta,
                             tau).cpu().numpy()
                norm, point = s_errors(S, r.S)
                ferr = np.max(np.abs(F - r.F) / r.F)
                _say(f"  slice {slicing or 'auto'} {form}: chi0 {err:.2e} S {norm:.2e}/"
                     f"{point:.2e} F {ferr:.2e}")
                assert err < CHI0_TOL[prec]
                assert norm < TOL[prec] and point < TOL[prec]
                assert ferr < TOL[prec]
    finally:
        tdx.chi0_set_slice_length(ctx, 0)
