"""Differentiable F(q,tau) with respect to the temperature, the broadening
and the tabulated shell values of the potential.

Three ``torch.autograd.Function`` steps, each calling the library's
forward kernels and, in ``backward``, its reverse-mode entry points:

  Chi00(T, eta, v)  states -> transitions -> pair densities -> chi0 (FP64)
                    -> Dyson, for every q of a workload (one state build);
                    backward: dyson_vjp -> chi0_vjp -> weights_vjp ->
                    occupations_vjp, pair_density_vjp -> potential_vjp.
                    The transition lists are time-reversal paired (half
                    the transitions) unless paired=False.  Pair densities
                    are not stored for backward: it recomputes them block
                    by block of the transition list (block_bytes of pair
                    densities and their cotangents at a time), so the
                    reverse sweep holds one block, never a whole list.
  DSF(chi00, beta)  S by the fluctuation-dissipation theorem (Eq. 8).
  ITCF(S, beta, tau) F by the two-sided Laplace transform (Eq. 1).

beta = 1/T and tau = x beta are ordinary torch arithmetic, so the explicit
temperature dependence of S and F reaches T through autograd.  One
temperature is used for every q (the states are built once).  The kernel
is RPA, which depends on none of the parameters, or ALDA, whose dependence
on the density adds to backward: dyson_kernel_vjp -> kernel_matrix_vjp per
q, then density_vjp once, feeding the same occupations_vjp and
potential_vjp.
"""
from __future__ import annotations

from typing import Optional

import numpy as np
import torch

from . import (Context, build_states, chi0, chi0_vjp, density_vjp, dsf, dsf_vjp, dyson,
               dyson_kernel_vjp, dyson_vjp, itcf, itcf_vjp, kernel_matrix, kernel_matrix_vjp,
               occupations, occupations_vjp, pair_density, pair_density_range, pair_density_vjp,
               potential_vjp, response_basis, transitions, weights_vjp)


def _with_shell_values(w, v):
    import dataclasses
    pot = dataclasses.replace(w.potential, shell_v=tuple(float(x) for x in v))
    return w.with_(potential=pot)


class ChainRunner:
    """Forward and reverse sweeps of chi_00 for every q of a workload.

    The model is non-self-consistent, so the orbitals depend on the shell
    values v only: a runner called again with the same v keeps its states
    and recomputes the occupations for the new temperature."""

    def __init__(self, ctx: Context, w, paired: bool = True, block_bytes: int = 8 << 30,
                 prec: str = "fp64"):
        if w.xc not in ("rpa", "alda"):
            raise ValueError(f"no gradient for the kernel {w.xc!r}")
        self.ctx = ctx
        self.w = w
        self.paired = paired
        self.block_bytes = int(block_bytes)
        # precision of the forward chi0 (the reverse sweep is FP64 whatever
        # it is; split-BF16 moves the gradient by its ~1e-5 forward error)
        self.prec = prec
        self.saved = None
        self._st, self._st_v = None, None

    def _states(self, w, T, v):
        key = None if v is None else tuple(float(x) for x in v)
        if self._st is not None and self._st_v == key:
            occupations(self.ctx, self._st, T, w.n_electrons, w.f_trunc)
        else:
            self._st = None
            self._st = build_states(self.ctx, w, T)
            self._st_v = key
        return self._st

    def blocks(self, n_trans: int, n_g: int, k_offsets=None):
        """Transition ranges of the reverse sweep: each holds at most
        block_bytes of FP64 pair densities plus their cotangents, and ends
        at a k boundary where one fits (the orbital adjoint's cost per k does
        not depend on how many of the k's transitions a range holds)."""
        ld = (n_g + 15) // 16 * 16
        size = max(64, self.block_bytes // (2 * 16 * ld))
        if k_offsets is None:
            return [(b, min(n_trans, b + size)) for b in range(0, n_trans, size)]
        ko = [int(x) for x in k_offsets]
        out, b = [], 0
        while b < n_trans:
            e = min(n_trans, b + size)
            cut = max((x for x in ko if b < x <= e), default=e)
            e = cut if e < n_trans else e
            out.append((b, e))
            b = e
        return out

    def forward(self, T: float, eta: float, v: Optional[np.ndarray]) -> torch.Tensor:
        w = self.w if v is None else _with_shell_values(self.w, v)
        w = w.with_(temperatures=tuple(T for _ in w.qs), eta=eta)
        ctx = self.ctx
        st = self._states(w, T, v)
        dev = st.eps.device
        pref = st.chi0_pref
        out, per_q = [], []
        for iq, qj in enumerate(w.qs):
            basis, g0 = response_basis(w.cell, w.kgrid, qj, w.ecut_chi[iq])
            gb = torch.from_numpy(basis).to(dev)
            tr = transitions(ctx, st, qj, w.f_trans_thr, paired=self.paired)
            P = pair_density(ctx, st, qj, tr, gb, self.prec)
            om = torch.as_tensor(w.omega_grid(iq), device=dev)
            c0 = chi0(ctx, tr, P, len(basis), self.prec, om, eta, pref)
            del P
            K = kernel_matrix(ctx, st, qj, gb, w.xc, w.dens_grid)
            out.append(dyson(ctx, c0, K, g0))
            per_q.append(dict(qj=tuple(qj), gb=gb, g0=g0, tr=tr, chi0=c0, K=K, omega=om))
        self.saved = dict(w=w, st=st, pref=pref, eta=eta, per_q=per_q)
        return torch.stack(out)

    def backward(self, chi00_bar: torch.Tensor, need_v: bool):
        ctx, sv = self.ctx, self.saved
        st, w = sv["st"], sv["w"]
        dev = st.eps.device
        occ_shape = tuple(st.eps.shape)
        eps_bar = torch.zeros(occ_shape, dtype=torch.float64, device=dev)
        eta_bar = torch.zeros(1, dtype=torch.float64, device=dev)
        coef_bar = torch.zeros_like(st.coef) if need_v else None
        T_bar = 0.0
        alda = w.xc == "alda"
        if alda:
            fxc_bar = torch.zeros(int(np.prod(w.dens_grid)), dtype=torch.float64, device=dev)
        for iq, q in enumerate(sv["per_q"]):
            tr, gb = q["tr"], q["gb"]
            n_g = gb.shape[0]
            u, v = dyson_vjp(ctx, q["chi0"], q["K"], q["g0"], chi00_bar[iq].contiguous())
            if alda:
                K_bar = dyson_kernel_vjp(ctx, q["chi0"], q["K"], q["g0"],
                                         chi00_bar[iq].contiguous())
                kernel_matrix_vjp(ctx, st, gb, w.dens_grid, K_bar, fxc_bar)
                del K_bar
            w_bar = torch.empty((max(len(tr), 1), 3), dtype=torch.float64, device=dev)
            for b0, b1 in self.blocks(len(tr), n_g, tr.k_offsets.cpu().numpy()):
                P = pair_density_range(ctx, st, q["qj"], tr, gb, b0, b1, "fp64")
                _, rho_bar = chi0_vjp(ctx, tr, P, n_g, q["omega"], sv["eta"], sv["pref"], u, v,
                                      want_rho=need_v, t_begin=b0, t_end=b1,
                                      w_out=w_bar[b0:b1])
                del P
                if need_v:
                    pair_density_vjp(ctx, st, q["qj"], tr, gb, rho_bar, coef_bar,
                                     t_begin=b0, t_end=b1)
                del rho_bar
            occ_bar = torch.zeros(occ_shape, dtype=torch.float64, device=dev)
            weights_vjp(ctx, st, q["qj"], tr, w_bar, occ_bar, eps_bar, eta_bar)
            T_bar += float(occupations_vjp(ctx, st, occ_bar, eps_bar)[0])
        if alda:
            occ_bar = torch.zeros(occ_shape, dtype=torch.float64, device=dev)
            density_vjp(ctx, st, w.dens_grid, fxc_bar, occ_bar, coef_bar)
            T_bar += float(occupations_vjp(ctx, st, occ_bar, eps_bar)[0])
        v_bar = potential_vjp(ctx, w, st, eps_bar, coef_bar) if need_v else None
        return T_bar, float(eta_bar[0]), v_bar


class Chi00(torch.autograd.Function):
    """chi_00(q, w) [n_q, n_w] (complex128, device) of (T, eta, v)."""

    @staticmethod
    def forward(fctx, T, eta, v, runner: ChainRunner):
        vv = None if v is None else v.detach().cpu().numpy().astype(np.float64)
        out = runner.forward(float(T), float(eta), vv)
        fctx.runner = runner
        fctx.v_shape = None if v is None else v.shape
        return out

    @staticmethod
    def backward(fctx, g):
        need_v = fctx.v_shape is not None and fctx.needs_input_grad[2]
        T_bar, eta_bar, v_bar = fctx.runner.backward(g.contiguous(), need_v)
        gT = torch.tensor(T_bar, dtype=torch.float64)
        ge = torch.tensor(eta_bar, dtype=torch.float64)
        gv = torch.from_numpy(v_bar) if need_v else None
        return gT, ge, gv, None


class DSF(torch.autograd.Function):
    @staticmethod
    def forward(fctx, chi00, beta, omega, density, ctx):
        fctx.save_for_backward(chi00, omega)
        fctx.beta, fctx.density, fctx.ctx = float(beta), density, ctx
        return dsf(ctx, chi00.contiguous(), omega, float(beta), density)

    @staticmethod
    def backward(fctx, S_bar):
        chi00, omega = fctx.saved_tensors
        c_bar, b_bar = dsf_vjp(fctx.ctx, chi00.contiguous(), omega, fctx.beta, fctx.density,
                               S_bar.contiguous())
        return c_bar, b_bar[0].cpu(), None, None, None


class ITCF(torch.autograd.Function):
    @staticmethod
    def forward(fctx, S, beta, tau, omega, ctx):
        tau_c = tau.detach().contiguous()
        fctx.save_for_backward(S, tau_c, omega)
        fctx.beta, fctx.ctx = float(beta), ctx
        return itcf(ctx, S.contiguous(), omega, float(beta), tau_c)

    @staticmethod
    def backward(fctx, F_bar):
        S, tau, omega = fctx.saved_tensors
        S_bar, tau_bar, b_bar = itcf_vjp(fctx.ctx, S.contiguous(), omega, fctx.beta, tau,
                                         F_bar.contiguous())
        return S_bar, b_bar[0].cpu(), tau_bar, None, None


def tau_fractions(w, iq: int) -> np.ndarray:
    """The workload's tau grid as fractions of beta."""
    t = w.tau_grid(iq)
    return t / t[-1] * (0.5 if w.tau_half else 1.0)


def itcf_differentiable(ctx: Context, w, T: torch.Tensor, eta: torch.Tensor,
                        v: Optional[torch.Tensor] = None,
                        runner: Optional[ChainRunner] = None) -> torch.Tensor:
    """F(q, tau = x beta) [n_q, n_tau] for every q of w, differentiable in
    T, eta and (if given) the shell values v.  T, eta, v: CPU float64.  A
    runner (ChainRunner of w) may be passed to reuse its states and settings."""
    runner = ChainRunner(ctx, w) if runner is None else runner
    chi00 = Chi00.apply(T, eta, v, runner)
    st = runner.saved["st"]
    dens = st.density
    beta = 1.0 / T
    dev = chi00.device
    out = []
    for iq in range(len(w.qs)):
        om = runner.saved["per_q"][iq]["omega"]
        S = DSF.apply(chi00[iq], beta, om, dens, ctx)
        tau = torch.as_tensor(tau_fractions(w, iq), device=dev) * beta.to(dev)
        out.append(ITCF.apply(S, beta, tau, om, ctx))
    return torch.stack(out)
