"""The split-BF16 pair-density buffer, decoded word by word and compared bit
for bit with the FP64 pair densities of the same transitions rounded the
documented way: x32 = fp32(x), hi = RNE_bf16(x32), lo = RNE_bf16(x32 - hi);
fragment words [t/4][comp][ld][t%4] with comp = hi, lo, word = (re, im) as
bf16 (low half re); then the FP32 rows x32 [T][ld]; rows are padded to a multiple of 32 plus one chunk of 32,
all zero past T.  The crystal with screening at 1e-4 has a transition count
that is not a multiple of 4, which checks the zeroed tail quad; chi0 from that
buffer is checked against the FP64 path on the same transitions."""
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


def _bits16(x32):
    import torch
    return x32.to(torch.bfloat16).view(torch.int16).to(torch.int32) & 0xFFFF


def test_split_bf16_layout_is_bit_exact(tdx):
    import torch
    print("layout", flush=True)
    ctx = tdx.Context(0)
    w = workloads.fcc_small().with_(f_trans_thr=1e-4)
    st = tdx.build_states(ctx, w)
    q = w.qs[0]
    basis, _ = tdx.response_basis(w.cell, w.kgrid, q, w.ecut_chi[0])
    gb = torch.from_numpy(basis).cuda()
    tr = tdx.transitions(ctx, st, q, w.f_trans_thr)
    T, n_g = len(tr), len(basis)
    assert T % 4 != 0
    ld = (n_g + 15) // 16 * 16
    print(f"  T = {T} (T mod 4 = {T % 4}), n_g = {n_g}, ld = {ld}", flush=True)
    P64buf = tdx.pair_density(ctx, st, q, tr, gb, "fp64")
    P64 = tdx.pair_density_view(P64buf, T, n_g, "fp64")
    buf = tdx.pair_density(ctx, st, q, tr, gb, "bf16x3")
    torch.cuda.synchronize()
    T4 = ((T + 31) // 32 + 1) * 32          # rows padded to 32 plus one zero chunk
    assert buf.numel() >= T4 * ld * 16
    words = buf[: T4 * ld * 8].view(torch.int32).view(T4 // 4, 2, ld, 4)
    Rall = buf[T4 * ld * 8: T4 * ld * 16].view(torch.float32).view(T4, ld, 2)
    R = Rall[:T]
    assert int((Rall[T:] != 0).sum()) == 0
    x = torch.zeros((T4, ld), dtype=torch.complex128, device="cuda")
    x[:T, :n_g] = P64
    re32, im32 = x.real.to(torch.float32), x.imag.to(torch.float32)
    assert torch.equal(R[:, :, 0], re32[:T]) and torch.equal(R[:, :, 1], im32[:T])
    rh, ih = re32.to(torch.bfloat16).to(torch.float32), im32.to(torch.bfloat16).to(torch.float32)
    hi = _bits16(re32) | (_bits16(im32) << 16)
    lo = _bits16(re32 - rh) | (_bits16(im32 - ih) << 16)
    for comp, ref in enumerate((hi, lo)):
        # words [T4/4][ld][4] -> rows t = 4 q + j
        got = words[:, comp].permute(0, 2, 1).reshape(T4, ld)
        assert torch.equal(got[:T], ref[:T].to(torch.int32)), f"component {comp}"
        assert int(got[T:].abs().max()) == 0 if T4 > T else True, f"tail of component {comp}"
    om = torch.as_tensor(w.omega_grid(0), device="cuda")
    pref = st.chi0_pref
    c64 = tdx.chi0(ctx, tr, P64buf, n_g, "fp64", om, w.eta, pref)
    c16 = tdx.chi0(ctx, tr, buf, n_g, "bf16x3", om, w.eta, pref)
    err = float((c16 - c64).abs().max() / c64.abs().max())
    print(f"  chi0 split-BF16 vs FP64 on the ragged set: {err:.2e}", flush=True)
    assert err < 1e-4
    ctx.close()
