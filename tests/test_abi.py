"""Host-only checks of the C ABI: the library loads, exports every symbol that
include/tdx.h declares, validates arguments, and its host geometry agrees
with the oracle's.  No kernel is launched."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2510_01875_amd", "libtdx.so")


@pytest.fixture(scope="module")
def tdx():
    if not os.path.exists(LIB):
        from paper_2510_01875_amd import build
        build.build()
    import paper_2510_01875_amd as m
    return m


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "tdx.h")).read()
    return sorted(set(re.findall(r"^\s*(?:int|size_t|const char \*)\s*(tdx_\w+)\(", text, re.M)))


def test_every_declared_symbol_is_exported(tdx):
    lib = C.CDLL(LIB)
    names = declared_symbols()
    assert len(names) >= 17
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(tdx.EXPORTED)


def test_abi_version(tdx):
    assert tdx.abi_version() == 2


def test_null_arguments_are_rejected(tdx):
    lib = C.CDLL(LIB)
    lib.tdx_last_error.restype = C.c_char_p
    assert lib.tdx_create(0, None) == tdx.ERR_INVALID_ARG
    assert b"null" in lib.tdx_last_error()
    assert lib.tdx_states_query(None, None) == tdx.ERR_INVALID_ARG
    assert lib.tdx_transitions(None, None, None, C.c_double(0), None, None, None) == tdx.ERR_INVALID_ARG
    assert lib.tdx_chi0(None, None, C.c_int64(0), None, 1, 0, None, 1, C.c_double(0.1),
                        C.c_double(1.0), None, None) == tdx.ERR_INVALID_ARG
    assert lib.tdx_dyson(None, None, None, 1, 1, 0, None, None) == tdx.ERR_INVALID_ARG
    assert lib.tdx_destroy(None) == tdx.OK


def test_bad_model_is_rejected(tdx):
    w = workloads.fcc_small()
    keep = []
    m = tdx.make_model(w, keep)
    m.ecut_wf = float("nan")
    d = tdx.StatesDims()
    assert tdx._query(C.byref(m), C.byref(d)) == tdx.ERR_INVALID_ARG
    m = tdx.make_model(w.with_(kgrid=(0, 4, 4)), keep)
    assert tdx._query(C.byref(m), C.byref(d)) == tdx.ERR_INVALID_ARG


@pytest.mark.parametrize("name", ["feg_c1", "fcc_c2", "h_tiny", "fcc_small"])
def test_states_query_matches_oracle_spheres(tdx, name):
    from oracle.lattice import gsphere, mp_kpoints, reciprocal
    w = workloads.get(name)
    d = tdx.states_query(w)
    B = reciprocal(w.cell)
    red, _ = mp_kpoints(w.kgrid)
    sel = red if len(red) <= 64 else red[:: max(1, len(red) // 64)]
    npw = [len(gsphere(B, k, w.ecut_wf)) for k in sel]
    assert d.n_k == w.n_k
    assert d.npw_max >= max(npw)
    if len(sel) == len(red):
        assert d.npw_max == max(npw)


@pytest.mark.parametrize("name,iq", [("feg_c1", 0), ("fcc_c2", 0), ("fcc_c2", 2), ("h_tiny", 1),
                                     ("fcc_c4", 5), ("fcc_c4", 17)])
def test_response_basis_matches_oracle(tdx, name, iq):
    from oracle.lattice import reciprocal, response_basis
    w = workloads.get(name)
    g, g0 = tdx.response_basis(w.cell, w.kgrid, w.qs[iq], w.ecut_chi[iq])
    ref, r0 = response_basis(reciprocal(w.cell), np.asarray(w.qs[iq]) / np.asarray(w.kgrid),
                             w.ecut_chi[iq])
    assert {tuple(x) for x in g} == {tuple(x) for x in ref}
    assert len(g) == len(ref)
    assert tuple(g[g0]) == (0, 0, 0) and tuple(ref[r0]) == (0, 0, 0)


@pytest.mark.parametrize("name,iq", [("feg_c1", 0), ("fcc_c2", 1), ("h16_c5", 3), ("fcc_c4", 9)])
def test_momentum_matches_oracle(tdx, name, iq):
    """q and |q|^2 of the library (host) against the oracle's reciprocal
    vectors; feg_c1's q = (2 pi / a) x exactly."""
    from oracle.lattice import reciprocal
    w = workloads.get(name)
    q, q2 = tdx.momentum(w.cell, w.kgrid, w.qs[iq])
    ref = (np.asarray(w.qs[iq]) / np.asarray(w.kgrid)) @ reciprocal(w.cell)
    assert np.max(np.abs(q - ref)) <= 1e-14 * np.max(np.abs(ref))
    assert abs(q2 - ref @ ref) <= 1e-14 * (ref @ ref)
    if name == "feg_c1":
        assert abs(q2 - (2 * np.pi / 7.0) ** 2) <= 1e-14


def test_slice_length_setting_validates(tdx):
    lib = C.CDLL(LIB)
    assert lib.tdx_chi0_set_slice_length(None, C.c_int64(0)) == tdx.ERR_INVALID_ARG


def test_response_basis_rejects_g0_outside(tdx):
    w = workloads.fcc_c2()
    with pytest.raises(tdx.TdxError) as e:
        tdx.response_basis(w.cell, w.kgrid, (0, 160, 160), 0.5)
    assert e.value.code == tdx.ERR_INVALID_ARG


def test_pair_density_bytes(tdx):
    assert tdx.pair_density_bytes(10, 17, "fp64") == 10 * 32 * 16
    assert tdx.pair_density_bytes(10, 17, "fp32") == 10 * 32 * 8
    # split-BF16: rows padded to a multiple of 32 plus one zero chunk of 32
    # (64 rows here) x 32 columns x (8 bytes of fragment words + 8 of FP32 rho)
    assert tdx.pair_density_bytes(10, 17, "bf16x3") == 64 * 32 * 16
    assert tdx.pair_density_bytes(32, 17, "bf16x3") == 64 * 32 * 16
    assert tdx.pair_density_bytes(33, 17, "bf16x3") == 96 * 32 * 16
