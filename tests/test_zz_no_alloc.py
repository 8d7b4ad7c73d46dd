"""The no-allocation Dyson entry point (tdx_dyson_noalloc) against tdx_dyson,
called through the C ABI: two calls in a row, the second smaller; a call
whose frequencies need several passes through the fixed scratch; the
singular case; a basis too large for the scratch."""
import ctypes as C

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
def lib(tdx):
    L = C.CDLL(tdx.LIB_PATH)
    L.tdx_dyson_noalloc.restype = C.c_int
    L.tdx_dyson_noalloc.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_int,
                                    C.c_int, C.c_void_p, C.c_void_p]
    L.tdx_dyson_noalloc_max_bytes.restype = C.c_size_t
    L.tdx_last_error.restype = C.c_char_p
    return L


def _noalloc(tdx, lib, ctx, chi0, K, g0, out):
    import torch
    n_w, n_g, _ = chi0.shape
    s = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    return lib.tdx_dyson_noalloc(ctx.handle, C.c_void_p(chi0.data_ptr()),
                                 C.c_void_p(K.data_ptr()), n_g, n_w, g0,
                                 C.c_void_p(out.data_ptr()), s)


def _random_case(n_w, n_g, seed):
    import torch
    g = torch.Generator().manual_seed(seed)
    c0 = (torch.randn(n_w, n_g, n_g, generator=g, dtype=torch.float64) +
          1j * torch.randn(n_w, n_g, n_g, generator=g, dtype=torch.float64)) * (0.3 / n_g)
    K = torch.diag(torch.rand(n_g, generator=g, dtype=torch.float64) + 0.5).to(torch.complex128)
    return c0.cuda(), K.cuda()


def test_noalloc_matches_dyson(tdx, lib):
    import torch
    ctx = tdx.Context(0)
    assert lib.tdx_dyson_noalloc_max_bytes() == 64 << 20
    # a benchmark-shaped chi0 first (fcc_small, ALDA), then a smaller random one
    w = workloads.fcc_small()
    st = tdx.build_states(ctx, w)
    g = tdx.run_q(ctx, w, st, 0, prec="fp64")
    cases = [(g.chi0, g.K, g.i_g0), _random_case(7, 19, 1) + (3,)]
    for chi0, K, g0 in cases:
        n_w, n_g, _ = chi0.shape
        _say(f"noalloc n_w={n_w} n_g={n_g}")
        ref = tdx.dyson(ctx, chi0, K, g0)
        out = torch.full((n_w,), complex("nan"), dtype=torch.complex128, device="cuda")
        assert _noalloc(tdx, lib, ctx, chi0, K, g0, out) == tdx.OK
        torch.cuda.synchronize()
        assert torch.equal(out, ref)
    ctx.close()


def test_noalloc_in_several_passes(tdx, lib):
    """n_g = 640: 6.5 MB per matrix, 10 frequencies per pass, 25 frequencies
    in three passes."""
    import torch
    ctx = tdx.Context(0)
    chi0, K = _random_case(25, 640, 2)
    ref = tdx.dyson(ctx, chi0, K, 5)
    out = torch.zeros(25, dtype=torch.complex128, device="cuda")
    assert _noalloc(tdx, lib, ctx, chi0, K, 5, out) == tdx.OK
    torch.cuda.synchronize()
    assert torch.equal(out, ref)
    ctx.close()


def test_noalloc_reports_singular_and_oversized(tdx, lib):
    import torch
    ctx = tdx.Context(0)
    n = 8
    chi0 = torch.eye(n, dtype=torch.complex128, device="cuda").repeat(3, 1, 1).contiguous()
    K = torch.eye(n, dtype=torch.complex128, device="cuda")
    out = torch.zeros(3, dtype=torch.complex128, device="cuda")
    assert _noalloc(tdx, lib, ctx, chi0, K, 0, out) == tdx.ERR_NUMERIC
    assert b"singular at frequency 0" in lib.tdx_last_error()
    # one 2048 x 2048 matrix (64 MiB) leaves no room for the status words:
    # rejected before any launch (the pointers are never read)
    dummy = torch.zeros(1, dtype=torch.complex128, device="cuda")
    s = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = lib.tdx_dyson_noalloc(ctx.handle, C.c_void_p(dummy.data_ptr()),
                               C.c_void_p(dummy.data_ptr()), 2048, 1, 0,
                               C.c_void_p(dummy.data_ptr()), s)
    assert rc == tdx.ERR_SHAPE and b"scratch" in lib.tdx_last_error()
    ctx.close()
