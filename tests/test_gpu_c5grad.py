"""The gradient workload at full size: the adjoint of F(q, tau) on the
16-proton system with respect to the temperature, the broadening and the
tabulated shell values of the potential, the reverse sweep recomputing the
pair densities block by block.

h16_c5 at the size of its states (64 k, about 6290 plane waves and 860 bands
per k, 304 response vectors, a time-reversal paired list of about 1.6e7
transitions) with its first q, its 64 imaginary times on [0, beta/2] and 21
frequencies on its [0, 5] Ha range (the frequency count only sets the cost
of each forward pass; the gradient is of the same discrete F).  The adjoint
in (T, eta, v_1, v_2, v_3) is checked along one seeded direction against a
central difference (h = 1e-5 relative to each parameter) of the GPU FP64
forward path, whose states are rebuilt for each shell-value step (the
orbitals depend on v).  Peak memory and times are printed.
"""
import time

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


def _workload():
    w = workloads.h16_c5()
    return w.with_(qs=w.qs[:1], temperatures=w.temperatures[:1], ecut_chi=w.ecut_chi[:1],
                   omega_max=w.omega_max[:1], n_omega=21)


@pytest.mark.timeout(900)
def test_h16_c5_gradient_in_T_eta_and_shell_values(tdx):
    import torch
    from paper_2510_01875_amd.grad import ChainRunner, itcf_differentiable
    ctx = tdx.Context(0)
    w = _workload()
    T, eta = w.temperatures[0], w.eta
    v0 = np.array(w.potential.shell_v, dtype=np.float64)
    n_v = len(v0)
    c = np.random.default_rng(11).standard_normal(w.n_tau)
    runner = ChainRunner(ctx, w, paired=True, block_bytes=4 << 30)

    def loss(p, grad):
        Tt = torch.tensor(p[0], dtype=torch.float64, requires_grad=grad)
        et = torch.tensor(p[1], dtype=torch.float64, requires_grad=grad)
        vt = torch.tensor(p[2:], dtype=torch.float64, requires_grad=grad)
        F = itcf_differentiable(ctx, w, Tt, et, vt, runner=runner)
        return (F.cpu() * torch.as_tensor(c).reshape(F.shape)).sum(), (Tt, et, vt)

    base = np.concatenate([[T, eta], v0])
    torch.cuda.reset_peak_memory_stats()
    t0 = time.perf_counter()
    L, params = loss(base, True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    q0 = runner.saved["per_q"][0]
    n_t, n_g = len(q0["tr"]), q0["gb"].shape[0]
    _say(f"forward: {n_t} paired transitions, N_G {n_g}, {n_v} shell values, {t1 - t0:.1f} s, "
         f"peak {torch.cuda.max_memory_allocated() / 2**30:.1f} GiB (torch)")
    torch.cuda.reset_peak_memory_stats()
    gT, ge, gv = torch.autograd.grad(L, params)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    grad = np.concatenate([[float(gT), float(ge)], gv.numpy()])
    nb = len(runner.blocks(n_t, n_g, q0["tr"].k_offsets.cpu().numpy()))
    _say(f"reverse: {nb} blocks of pair densities recomputed, {t2 - t1:.1f} s, peak "
         f"{torch.cuda.max_memory_allocated() / 2**30:.1f} GiB (torch); grad {grad}")
    assert nb >= 10 and np.all(np.isfinite(grad))
    d = np.random.default_rng(12).standard_normal(2 + n_v) * np.abs(base)
    h = 1e-5
    with torch.no_grad():
        Lp, _ = loss(base + h * d, False)
        _say(f"  +h forward done ({time.perf_counter() - t2:.1f} s)")
        Lm, _ = loss(base - h * d, False)
    fd = (float(Lp) - float(Lm)) / (2 * h)
    got = float(np.dot(grad, d))
    _say(f"direction: adjoint {got:.10e} central difference {fd:.10e} "
         f"({time.perf_counter() - t2:.1f} s for the two forward passes)")
    assert abs(got - fd) <= 1e-6 * abs(fd)
    ctx.close()
