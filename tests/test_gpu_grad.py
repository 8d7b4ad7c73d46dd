"""Reverse mode of F(q,tau) on the GPU.

Each reverse-mode entry point is checked against PyTorch autograd of the
same forward formula written out in plain CPU torch (FP64); the full
gradient in (T, eta, v(G_s)) is checked against the oracle's forward-mode
tangents (a different algorithm) and against central differences
(h = 1e-5) of the GPU forward path.
"""
import math

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


def _w(n_q=1):
    """4-proton box, screening off so that no transition enters or leaves
    the set inside a finite-difference stencil."""
    w = workloads.h_tiny()
    return w.with_(f_trans_thr=0.0, n_omega=40, qs=w.qs[:n_q],
                   temperatures=w.temperatures[:n_q], ecut_chi=w.ecut_chi[:n_q],
                   omega_max=w.omega_max[:n_q], n_tau=9)


def test_itcf_and_dsf_vjp_match_autograd(tdx, ctx):
    import torch
    _say("itcf/dsf vjp")
    g = torch.Generator().manual_seed(1)
    n_w, n_tau = 37, 11
    om = torch.linspace(0.0, 2.5, n_w, dtype=torch.float64)
    beta0 = 6.3
    S = torch.rand(n_w, generator=g, dtype=torch.float64)
    x = torch.linspace(0.0, 1.0, n_tau, dtype=torch.float64)
    Fbar = torch.randn(n_tau, generator=g, dtype=torch.float64)
    # plain torch ITCF
    Sr = S.clone().requires_grad_()
    br = torch.tensor(beta0, dtype=torch.float64, requires_grad=True)
    tr = (x * beta0).clone().requires_grad_()
    h = om[1:] - om[:-1]
    c = torch.zeros(n_w, dtype=torch.float64)
    c[:-1] += 0.5 * h
    c[1:] += 0.5 * h
    F = ((c * Sr)[None, :] * (torch.exp(-tr[:, None] * om[None, :]) +
                              torch.exp(-(br - tr[:, None]) * om[None, :]))).sum(1)
    gS, gb, gt = torch.autograd.grad((F * Fbar).sum(), (Sr, br, tr))
    d = lambda t: t.cuda()
    S_bar, tau_bar, b_bar = tdx.itcf_vjp(ctx, d(S), d(om), beta0, d(x * beta0), d(Fbar))
    torch.cuda.synchronize()
    np.testing.assert_allclose(S_bar.cpu().numpy(), gS.numpy(), rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(tau_bar.cpu().numpy(), gt.numpy(), rtol=1e-11, atol=1e-14)
    np.testing.assert_allclose(float(b_bar[0]), float(gb), rtol=1e-11)
    # plain torch DSF (w = 0 from the next point)
    chi = torch.complex(torch.randn(n_w, generator=g, dtype=torch.float64),
                        -torch.rand(n_w, generator=g, dtype=torch.float64))
    dens = 0.0123
    Sbar = torch.randn(n_w, generator=g, dtype=torch.float64)
    cr = chi.clone().requires_grad_()
    br = torch.tensor(beta0, dtype=torch.float64, requires_grad=True)
    im = cr.imag
    Sv = torch.empty(n_w, dtype=torch.float64)
    parts = [(-im[1] / (math.pi * dens * br * om[1])).reshape(1)]
    parts.append(-im[1:] / (math.pi * dens * (-torch.expm1(-br * om[1:]))))
    Sv = torch.cat(parts)
    gc, gb = torch.autograd.grad((Sv * Sbar).sum(), (cr, br))
    c_bar, b_bar = tdx.dsf_vjp(ctx, d(chi), d(om), beta0, dens, d(Sbar))
    torch.cuda.synchronize()
    np.testing.assert_allclose(c_bar.cpu().numpy(), gc.numpy(), rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(float(b_bar[0]), float(gb), rtol=1e-11)


def test_dyson_vjp_matches_autograd(tdx, ctx):
    import torch
    _say("dyson vjp")
    g = torch.Generator().manual_seed(2)
    n_w, n_g, g0 = 5, 23, 3
    c0 = (torch.randn(n_w, n_g, n_g, generator=g, dtype=torch.float64) +
          1j * torch.randn(n_w, n_g, n_g, generator=g, dtype=torch.float64)) * 0.05
    K = torch.diag(torch.rand(n_g, generator=g, dtype=torch.float64) + 0.5).to(torch.complex128)
    K[0, 1] = K[1, 0] = 0.2           # a non-diagonal entry
    cbar = torch.randn(n_w, generator=g, dtype=torch.float64) + \
        1j * torch.randn(n_w, generator=g, dtype=torch.float64)
    cr = c0.clone().requires_grad_()
    I = torch.eye(n_g, dtype=torch.complex128)
    x = torch.linalg.solve(I - cr @ K, cr[:, :, g0:g0 + 1])[:, g0, 0]
    L = (cbar.conj() * x).real.sum()
    (gc,) = torch.autograd.grad(L, (cr,))
    u, v = tdx.dyson_vjp(ctx, c0.cuda(), K.cuda(), g0, cbar.cuda())
    got = (u[:, :, None] * v.conj()[:, None, :]).cpu()
    err = float((got - gc).abs().max() / gc.abs().max())
    _say(f"  rank-1 cotangent err {err:.2e}")
    assert err < 1e-12


def test_dyson_kernel_vjp_matches_autograd(tdx, ctx):
    """K_bar of chi00 = [(1 - chi0 K)^{-1} chi0]_{g0 g0} with a full complex
    K (the ALDA kernel is not diagonal), accumulated onto a given K_bar."""
    import torch
    _say("dyson kernel vjp")
    g = torch.Generator().manual_seed(5)
    n_w, n_g, g0 = 6, 21, 4
    c0 = (torch.randn(n_w, n_g, n_g, generator=g, dtype=torch.float64) +
          1j * torch.randn(n_w, n_g, n_g, generator=g, dtype=torch.float64)) * 0.05
    K = (torch.randn(n_g, n_g, generator=g, dtype=torch.float64) +
         1j * torch.randn(n_g, n_g, generator=g, dtype=torch.float64)) * 0.1
    K = K + torch.diag(torch.rand(n_g, generator=g, dtype=torch.float64) + 0.5)
    cbar = torch.randn(n_w, generator=g, dtype=torch.float64) + \
        1j * torch.randn(n_w, generator=g, dtype=torch.float64)
    Kr = K.clone().requires_grad_()
    I = torch.eye(n_g, dtype=torch.complex128)
    x = torch.linalg.solve(I - c0 @ Kr, c0[:, :, g0:g0 + 1])[:, g0, 0]
    L = (cbar.conj() * x).real.sum()
    (gK,) = torch.autograd.grad(L, (Kr,))
    base = torch.full((n_g, n_g), 0.25 - 0.5j, dtype=torch.complex128)
    got = tdx.dyson_kernel_vjp(ctx, c0.cuda(), K.cuda(), g0, cbar.cuda(),
                               K_bar=base.clone().cuda()).cpu() - base
    err = float((got - gK).abs().max() / gK.abs().max())
    _say(f"  K cotangent err {err:.2e}")
    assert err < 1e-12


@pytest.mark.parametrize("paired", [False, True])
def test_chi0_vjp_matches_autograd(tdx, ctx, paired):
    """Transitions and FP64 pair densities of the hydrogen box; a ragged
    count (not a multiple of the 64-transition tile) and a frequency count
    that is not a multiple of the 64-frequency block.  The paired list's
    weight is df [1/(w - delta + i eta) - 1/(w + delta + i eta)]."""
    import torch
    _say("chi0 vjp", "paired" if paired else "full")
    w = _w()
    st = tdx.build_states(ctx, w)
    basis, g0 = tdx.response_basis(w.cell, w.kgrid, w.qs[0], w.ecut_chi[0])
    n_g = len(basis)
    gb = torch.from_numpy(basis).cuda()
    tr_full = tdx.transitions(ctx, st, w.qs[0], w.f_trans_thr, paired=paired)
    P_full = tdx.pair_density(ctx, st, w.qs[0], tr_full, gb, "fp64")
    T_all = len(tr_full) - 37          # ragged tail of the last tile
    n_w = 70
    om = torch.linspace(0.0, 3.0, n_w, dtype=torch.float64, device="cuda")
    eta, pref = 0.02, st.chi0_pref
    g = torch.Generator().manual_seed(3)
    u = (torch.randn(n_w, n_g, generator=g, dtype=torch.float64) +
         1j * torch.randn(n_w, n_g, generator=g, dtype=torch.float64))
    v = (torch.randn(n_w, n_g, generator=g, dtype=torch.float64) +
         1j * torch.randn(n_w, n_g, generator=g, dtype=torch.float64))
    w_bar, rho_bar = tdx.chi0_vjp(ctx, tr_full, P_full, n_g, om, eta, pref, u.cuda(), v.cuda(),
                                  want_rho=True, t_end=T_all)
    torch.cuda.synchronize()
    _say(f"  T = {T_all} (T mod 64 = {T_all % 64}), n_g = {n_g}")
    # reference on a subset of transitions (the kernel result is per transition)
    sel = torch.cat([torch.arange(0, T_all, max(1, T_all // 600)),
                     torch.arange(T_all - 40, T_all)])
    P = tdx.pair_density_view(P_full, len(tr_full), n_g, "fp64")[:T_all][sel].cpu()
    df = tr_full.df[:T_all][sel].cpu()
    dl = tr_full.delta[:T_all][sel].cpu()
    dfr, dlr = df.clone().requires_grad_(), dl.clone().requires_grad_()
    er = torch.tensor(eta, dtype=torch.float64, requires_grad=True)
    Pr = P.clone().requires_grad_()
    omc = om.cpu()
    W = dfr[None, :] / (omc[:, None] - dlr[None, :] + 1j * er)            # [w, t]
    if paired:
        W = W - dfr[None, :] / (omc[:, None] + dlr[None, :] + 1j * er)
    # L = Re sum_w sum_GG' conj(u_G conj(v_G')) chi0_GG'
    #   = Re sum_w sum_t pref W (u^H rho_t) conj(v^H rho_t)
    a = u.conj() @ Pr.T                                                     # [w, t]
    b = v.conj() @ Pr.T
    L = (pref * W * a * b.conj()).real.sum()
    g_df, g_dl, g_eta, g_P = torch.autograd.grad(L, (dfr, dlr, er, Pr))
    wb = w_bar[:T_all][sel.cuda()].cpu()
    np.testing.assert_allclose(wb[:, 0].numpy(), g_df.numpy(), rtol=1e-10,
                               atol=1e-10 * float(g_df.abs().max()))
    np.testing.assert_allclose(wb[:, 1].numpy(), g_dl.numpy(), rtol=1e-10,
                               atol=1e-10 * float(g_dl.abs().max()))
    rb = rho_bar[:T_all][sel.cuda()][:, :n_g].cpu()
    err = float((rb - g_P).abs().max() / g_P.abs().max())
    _say(f"  rho_bar err {err:.2e}")
    assert err < 1e-11
    # eta: the kernel's per-transition terms summed over the subset
    np.testing.assert_allclose(float(wb[:, 2].sum()), float(g_eta), rtol=1e-9)
    assert float(rho_bar[:T_all, n_g:].abs().max() if rho_bar.shape[1] > n_g else 0.0) == 0.0
    # the same rows from blocks of the list: pair densities and cotangents
    # recomputed per block agree with the whole-list call, and the orbital
    # cotangents accumulated block by block with the whole-list ones
    n = len(tr_full)
    cb_whole = torch.zeros_like(st.coef)
    wb_all, rb_all = tdx.chi0_vjp(ctx, tr_full, P_full, n_g, om, eta, pref, u.cuda(), v.cuda(),
                                  want_rho=True)
    tdx.pair_density_vjp(ctx, st, w.qs[0], tr_full, gb, rb_all, cb_whole)
    cb_blocks = torch.zeros_like(st.coef)
    cuts = [0, n // 5, n // 5 + 1, n // 2, n]
    for b0, b1 in zip(cuts[:-1], cuts[1:]):
        Pb = tdx.pair_density_range(ctx, st, w.qs[0], tr_full, gb, b0, b1, "fp64")
        assert float((tdx.pair_density_view(Pb, b1 - b0, n_g, "fp64") -
                      tdx.pair_density_view(P_full, n, n_g, "fp64")[b0:b1]).abs().max()) <= \
            1e-13 * float(P_full.view(torch.complex128).abs().max())
        wbb, rbb = tdx.chi0_vjp(ctx, tr_full, Pb, n_g, om, eta, pref, u.cuda(), v.cuda(),
                                want_rho=True, t_begin=b0, t_end=b1)
        assert torch.allclose(wbb, wb_all[b0:b1], rtol=1e-12, atol=1e-12 * float(wb_all.abs().max()))
        tdx.pair_density_vjp(ctx, st, w.qs[0], tr_full, gb, rbb, cb_blocks, t_begin=b0, t_end=b1)
    err = float((cb_blocks - cb_whole).abs().max() / cb_whole.abs().max())
    _say(f"  coef_bar blocks vs whole {err:.2e}")
    assert err < 1e-12


def _loss_weights(n):
    return np.random.default_rng(7).standard_normal(n)


def _gpu_loss(tdx, ctx, w, T, eta, v, c, runner=None):
    import torch
    from paper_2510_01875_amd.grad import itcf_differentiable
    Tt = torch.tensor(T, dtype=torch.float64, requires_grad=True)
    et = torch.tensor(eta, dtype=torch.float64, requires_grad=True)
    vt = torch.tensor(v, dtype=torch.float64, requires_grad=True)
    F = itcf_differentiable(ctx, w, Tt, et, vt, runner=runner)
    L = (F.cpu() * torch.as_tensor(c).reshape(F.shape)).sum()
    return L, (Tt, et, vt)


@pytest.mark.parametrize("form", ["paired", "full", "paired-blocks", "alda"])
def test_gradient_matches_oracle_tangent_and_finite_differences(tdx, ctx, form):
    """The reverse sweep over the time-reversal paired list, over the full
    list, over the paired list in blocks of about 40 transitions (pair
    densities and cotangents recomputed per block), and with the ALDA kernel
    (paired list), whose density moves with T and v."""
    import torch
    from oracle import tangent
    from paper_2510_01875_amd.grad import ChainRunner
    _say("gradient", form)
    w = _w()
    if form == "alda":
        w = w.with_(xc="alda", dens_grid=(12, 12, 12))
    T, eta = w.temperatures[0], w.eta
    v = np.asarray(w.potential.shell_v, dtype=np.float64)
    c = _loss_weights(w.n_tau)
    runner = ChainRunner(ctx, w, paired=form != "full",
                         block_bytes=(40 * 2 * 16 * 64 if form == "paired-blocks" else 8 << 30))
    L, (Tt, et, vt) = _gpu_loss(tdx, ctx, w, T, eta, v, c, runner=runner)
    if form == "paired-blocks":
        q0 = runner.saved["per_q"][0]
        n_t = len(q0["tr"])
        nb = len(runner.blocks(n_t, q0["gb"].shape[0]))
        _say(f"  {nb} blocks of {n_t} paired transitions")
        assert nb >= 3
    gT, ge, gv = torch.autograd.grad(L, (Tt, et, vt))
    grad = np.concatenate([[float(gT), float(ge)], gv.numpy()])
    _say(f"  grad {grad}")
    # oracle forward-mode tangents along two mixed directions
    rng = np.random.default_rng(8)
    for _ in range(2):
        d = rng.standard_normal(2 + len(v)) * np.concatenate([[T, eta], np.abs(v)])
        F0, dF, _ = tangent.itcf_tangent(w, 0, T, eta, d[0], d[1], d[2:])
        ref = float(np.dot(c, dF))
        got = float(np.dot(grad, d))
        _say(f"  direction: adjoint {got:.12e} oracle tangent {ref:.12e}")
        assert abs(got - ref) <= 1e-8 * abs(ref)
        np.testing.assert_allclose(L.item(), float(np.dot(c, F0)), rtol=1e-11)
    # central differences of the GPU forward, one parameter at a time, step
    # 1e-5 relative to the parameter
    base = np.concatenate([[T, eta], v])
    for i in range(len(base)):
        h = 1e-5 * abs(base[i])
        p, m = base.copy(), base.copy()
        p[i] += h
        m[i] -= h
        with torch.no_grad():
            Lp, _ = _gpu_loss(tdx, ctx, w, p[0], p[1], p[2:], c, runner=runner)
            Lm, _ = _gpu_loss(tdx, ctx, w, m[0], m[1], m[2:], c, runner=runner)
        fd = (float(Lp) - float(Lm)) / (2 * h)
        _say(f"  param {i}: adjoint {grad[i]:.10e} central difference {fd:.10e}")
        assert abs(grad[i] - fd) <= 1e-6 * max(abs(fd), 1e-3 * np.max(np.abs(grad)))


def test_gradients_of_several_q_add_up(tdx, ctx):
    """One state build shared by two q: the gradient of F(q1) + F(q2)
    equals the sum of the single-q gradients."""
    import torch
    _say("two q")
    w2 = _w(n_q=2)
    T, eta = w2.temperatures[0], w2.eta
    v = np.asarray(w2.potential.shell_v, dtype=np.float64)
    c = np.concatenate([_loss_weights(w2.n_tau), -0.5 * _loss_weights(w2.n_tau)])
    L, params = _gpu_loss(tdx, ctx, w2, T, eta, v, c)
    g_both = np.concatenate([np.atleast_1d(x.numpy()) for x in torch.autograd.grad(L, params)])
    total = np.zeros_like(g_both)
    for iq, cc in enumerate((c[:w2.n_tau], c[w2.n_tau:])):
        wq = w2.with_(qs=w2.qs[iq:iq + 1], temperatures=w2.temperatures[iq:iq + 1],
                      ecut_chi=w2.ecut_chi[iq:iq + 1], omega_max=w2.omega_max[iq:iq + 1])
        Lq, pq = _gpu_loss(tdx, ctx, wq, T, eta, v, cc)
        total += np.concatenate([np.atleast_1d(x.numpy()) for x in torch.autograd.grad(Lq, pq)])
    _say(f"  both {g_both}\n  sum  {total}")
    np.testing.assert_allclose(g_both, total, rtol=1e-10, atol=1e-12 * np.max(np.abs(total)))
