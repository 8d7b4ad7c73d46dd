"""Python binding of the tdx HIP library (libtdx.so, gfx950).

Argument marshalling only: every step of the chi0 -> Dyson -> S -> F path
runs in the library's HIP kernels.  PyTorch supplies device memory and the
HIP stream.  Names follow the C ABI in include/tdx.h.

The library is built in-tree by ``paper_2510_01875_amd.build``; importing
this package without it raises immediately (there is no CPU fallback).
"""
from __future__ import annotations

import ctypes as C
import math
import os
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtdx.so")

PREC = {"fp64": 0, "fp32": 1, "bf16x3": 2}
XC = {"rpa": 0, "alda": 1}

OK, ERR_INVALID_ARG, ERR_SHAPE, ERR_ALLOC, ERR_HIP, ERR_NUMERIC, ERR_UNSUPPORTED = 0, -1, -2, -3, -4, -5, -6


class TdxError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"tdx error {code}: {msg}")
        self.code = code


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python paper_2510_01875_amd/build.py` (no CPU fallback exists)")
    return C.CDLL(LIB_PATH)


_lib = _load()

c_int_p = C.POINTER(C.c_int)
c_dbl_p = C.POINTER(C.c_double)


class Model(C.Structure):
    _fields_ = [("cell", C.c_double * 9), ("kgrid", C.c_int * 3), ("ecut_wf", C.c_double),
                ("n_bands", C.c_int), ("n_electrons", C.c_double), ("f_trunc", C.c_double),
                ("n_atoms", C.c_int), ("positions", c_dbl_p), ("shell_unit", C.c_double),
                ("n_shells", C.c_int), ("shell_n2", c_int_p), ("shell_v", c_dbl_p),
                ("gauss", C.c_int), ("z_ion", C.c_double), ("sigma", C.c_double)]


class StatesDims(C.Structure):
    _fields_ = [("n_k", C.c_int), ("npw_max", C.c_int), ("nb_max", C.c_int)]


class StatesC(C.Structure):
    _fields_ = [("n_k", C.c_int), ("npw_max", C.c_int), ("nb_max", C.c_int),
                ("npw", C.c_void_p), ("nb", C.c_void_p), ("miller", C.c_void_p),
                ("eps", C.c_void_p), ("occ", C.c_void_p), ("coef", C.c_void_p),
                ("kgrid", C.c_int * 3), ("mmax", C.c_int * 3), ("cell", C.c_double * 9),
                ("bvec", C.c_double * 9), ("mu", C.c_double), ("temperature", C.c_double),
                ("omega_cell", C.c_double), ("n_electrons", C.c_double), ("beta", C.c_double),
                ("density", C.c_double), ("chi0_pref", C.c_double)]


class TransC(C.Structure):
    _fields_ = [("capacity", C.c_int64), ("k", C.c_void_p), ("n", C.c_void_p),
                ("m", C.c_void_p), ("delta", C.c_void_p), ("df", C.c_void_p),
                ("k_offsets", C.c_void_p), ("paired", C.c_int32)]


def _sig(name, args):
    f = getattr(_lib, name)
    f.argtypes = args
    f.restype = C.c_int
    return f


_lib.tdx_last_error.restype = C.c_char_p
_lib.tdx_last_error.argtypes = []
_lib.tdx_pair_density_bytes.restype = C.c_size_t
_lib.tdx_pair_density_bytes.argtypes = [C.c_int64, C.c_int, C.c_int]
_create = _sig("tdx_create", [C.c_int, C.POINTER(C.c_void_p)])
_destroy = _sig("tdx_destroy", [C.c_void_p])
_set_limit = _sig("tdx_set_workspace_limit", [C.c_void_p, C.c_size_t])
_abi = _sig("tdx_abi_version", [])
_query = _sig("tdx_states_query", [C.POINTER(Model), C.POINTER(StatesDims)])
_build = _sig("tdx_build_states", [C.c_void_p, C.POINTER(Model), C.c_double,
                                   C.POINTER(StatesC), C.c_void_p])
_occ = _sig("tdx_occupations", [C.c_void_p, C.POINTER(StatesC), C.c_double, C.c_double,
                                C.c_double, C.c_void_p])
_basis = _sig("tdx_response_basis", [C.c_double * 9, C.c_int * 3, C.c_int * 3, C.c_double,
                                     c_int_p, C.c_int, c_int_p, c_int_p])
_momentum = _sig("tdx_momentum", [C.c_double * 9, C.c_int * 3, C.c_int * 3, c_dbl_p, c_dbl_p])
_trans = _sig("tdx_transitions", [C.c_void_p, C.POINTER(StatesC), C.c_int * 3, C.c_double,
                                  C.POINTER(TransC), C.POINTER(C.c_int64), C.c_void_p])
_pair = _sig("tdx_pair_density", [C.c_void_p, C.POINTER(StatesC), C.c_int * 3,
                                  C.POINTER(TransC), C.c_int64, C.c_void_p, C.c_int, C.c_int,
                                  C.c_void_p, C.c_void_p])
_pair_range = _sig("tdx_pair_density_range", [C.c_void_p, C.POINTER(StatesC), C.c_int * 3,
                                              C.POINTER(TransC), C.c_int64, C.c_int64,
                                              C.c_void_p, C.c_int, C.c_int, C.c_void_p,
                                              C.c_void_p])
_pair_async = _sig("tdx_pair_density_async", [C.c_void_p, C.POINTER(StatesC), C.c_int * 3,
                                              C.POINTER(TransC), C.c_int64, C.c_int64,
                                              C.c_void_p, C.c_int, C.c_int, C.c_void_p,
                                              C.c_void_p, C.c_size_t, C.c_void_p])
_lib.tdx_pair_density_work_bytes.restype = C.c_size_t
_lib.tdx_pair_density_work_bytes.argtypes = [C.POINTER(StatesC), C.c_int64]
_chi0 = _sig("tdx_chi0", [C.c_void_p, C.POINTER(TransC), C.c_int64, C.c_void_p, C.c_int,
                          C.c_int, C.c_void_p, C.c_int, C.c_double, C.c_double, C.c_void_p,
                          C.c_void_p])
_kmat = _sig("tdx_kernel_matrix", [C.c_void_p, C.POINTER(StatesC), C.c_int * 3, C.c_void_p,
                                   C.c_int, C.c_int, C.c_int * 3, C.c_void_p, C.c_void_p])
_xcgrid = _sig("tdx_xc_kernel_grid", [C.c_void_p, C.POINTER(StatesC), C.c_int * 3, C.c_void_p,
                                      C.c_void_p])
_kmat_g = _sig("tdx_kernel_matrix_from_grid", [C.c_void_p, C.POINTER(StatesC), C.c_int * 3,
                                               C.c_void_p, C.c_int, C.c_int, C.c_int * 3,
                                               C.c_void_p, C.c_void_p, C.c_void_p])
_dyson = _sig("tdx_dyson", [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_int, C.c_int,
                            C.c_void_p, C.c_void_p])
_dsf = _sig("tdx_dsf", [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_double, C.c_double,
                        C.c_void_p, C.c_void_p])
class Chi0ItemC(C.Structure):
    _fields_ = [("tl", C.POINTER(TransC)), ("n_trans", C.c_int64), ("P", C.c_void_p),
                ("n_g", C.c_int), ("omega", C.c_void_p), ("n_w", C.c_int), ("eta", C.c_double),
                ("pref", C.c_double), ("chi0", C.c_void_p), ("p_rows", C.c_int64)]


_plan_create = _sig("tdx_chi0_plan_create", [C.c_void_p, C.POINTER(Chi0ItemC), C.c_int, C.c_int,
                                             C.POINTER(C.c_void_p)])
_plan_launch = _sig("tdx_chi0_plan_launch", [C.c_void_p, C.c_void_p, C.c_void_p])
_plan_destroy = _sig("tdx_chi0_plan_destroy", [C.c_void_p])
_batched = _sig("tdx_chi0_batched", [C.c_void_p, C.POINTER(Chi0ItemC), C.c_int, C.c_int,
                                     C.c_void_p])
_variants = _sig("tdx_chi0_variants", [C.c_int, C.POINTER(C.c_int)])
_set_cfg = _sig("tdx_chi0_set_config", [C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_int])
_set_slice = _sig("tdx_chi0_set_slice_length", [C.c_void_p, C.c_int64])
_bf_slicing = _sig("tdx_chi0_bf16x3_slicing", [C.c_int, C.c_int, C.c_int64, C.c_int, C.c_int,
                                                C.c_int, C.POINTER(C.c_int64),
                                                C.POINTER(C.c_int)])
_get_cfg = _sig("tdx_chi0_get_config", [C.c_void_p, C.c_int, C.c_int, C.POINTER(C.c_int),
                                        C.POINTER(C.c_int)])
_autotune = _sig("tdx_autotune_chi0", [C.c_void_p, C.POINTER(Chi0ItemC), C.c_int, C.c_int64,
                                       C.POINTER(C.c_int), C.POINTER(C.c_int),
                                       C.POINTER(C.c_double)])
_tune_save = _sig("tdx_tune_save", [C.c_void_p, C.c_char_p])
_tune_load = _sig("tdx_tune_load", [C.c_void_p, C.c_char_p])
_lib.tdx_dyson_work_bytes.restype = C.c_size_t
_lib.tdx_dyson_work_bytes.argtypes = [C.c_int, C.c_int]
_dyson_async = _sig("tdx_dyson_async", [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_int,
                                        C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p])
_itcf = _sig("tdx_itcf", [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_double, C.c_void_p,
                          C.c_int, C.c_void_p, C.c_void_p])

_metrics = _sig("tdx_itcf_metrics", [C.c_void_p, C.c_void_p, C.c_int, C.c_void_p, C.c_int,
                                     C.c_double, C.c_double, C.c_void_p, C.c_void_p])
_dielectric = _sig("tdx_dielectric", [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_double,
                                      C.c_double, C.c_double, C.c_void_p, C.c_void_p,
                                      C.c_void_p, C.c_void_p])
_sgf = _sig("tdx_sg_filter", [C.c_void_p, C.c_void_p, C.c_int, C.POINTER(C.c_int),
                              C.POINTER(C.c_int), C.c_int, C.c_void_p, C.c_void_p, C.c_void_p])
_dpsd = _sig("tdx_derivative_psd", [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_int,
                                    C.c_void_p, C.c_int, C.c_void_p, C.c_void_p])
_sgs = _sig("tdx_sg_scores", [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                              C.c_int, C.c_int, C.c_void_p, C.c_int, C.c_void_p, C.c_void_p])
_resid = _sig("tdx_residual_itcf", [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_void_p,
                                    C.c_int, C.c_double, C.c_void_p, C.c_void_p])
_sgsel = _sig("tdx_sg_select", [c_dbl_p, c_dbl_p, C.c_int, C.c_int, C.c_double, C.c_double,
                                C.c_double, C.c_double, C.POINTER(C.c_int)])
_kgdsf = _sig("tdx_kg_dsf", [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_double,
                            C.c_double, C.c_void_p, C.c_void_p])
_kg_work = _lib.tdx_kg_work_bytes
_kg_work.restype = C.c_size_t
_kg_work.argtypes = [C.c_int64, C.c_int]
_kgsig = _sig("tdx_kg_conductivity", [C.c_void_p, C.POINTER(StatesC), C.POINTER(TransC),
                                      C.c_int64, C.c_void_p, C.c_int, C.c_double, C.c_void_p,
                                      C.c_void_p, C.c_size_t, C.c_void_p])
_eta_ref = _sig("tdx_eta_reference", [c_dbl_p, c_dbl_p, C.c_int, C.c_double,
                                      C.POINTER(C.c_int)])
_itcf_vjp = _sig("tdx_itcf_vjp", [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_double,
                                  C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p,
                                  C.c_void_p, C.c_void_p])
_dsf_vjp = _sig("tdx_dsf_vjp", [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_double,
                                C.c_double, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p])
_dyson_vjp = _sig("tdx_dyson_vjp", [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_int, C.c_int,
                                    C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                    C.c_void_p])
_chi0_vjp = _sig("tdx_chi0_vjp", [C.c_void_p, C.POINTER(TransC), C.c_int64, C.c_int64,
                                  C.c_void_p, C.c_int, C.c_void_p, C.c_int, C.c_double,
                                  C.c_double, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                  C.c_void_p])
_weights_vjp = _sig("tdx_weights_vjp", [C.c_void_p, C.POINTER(StatesC), C.c_int * 3,
                                        C.POINTER(TransC), C.c_int64, C.c_void_p, C.c_void_p,
                                        C.c_void_p, C.c_void_p, C.c_void_p])
_occ_vjp = _sig("tdx_occupations_vjp", [C.c_void_p, C.POINTER(StatesC), C.c_void_p, C.c_void_p,
                                        C.c_void_p, C.c_void_p])
_pair_vjp = _sig("tdx_pair_density_vjp", [C.c_void_p, C.POINTER(StatesC), C.c_int * 3,
                                          C.POINTER(TransC), C.c_int64, C.c_int64, C.c_void_p,
                                          C.c_int, C.c_void_p, C.c_void_p, C.c_void_p])
_dyson_k_vjp = _sig("tdx_dyson_kernel_vjp", [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_int,
                                           C.c_int, C.c_void_p, C.c_void_p, C.c_void_p])
_kmat_vjp = _sig("tdx_kernel_matrix_vjp", [C.c_void_p, C.POINTER(StatesC), C.c_void_p, C.c_int,
                                           C.c_int * 3, C.c_void_p, C.c_void_p, C.c_void_p])
_dens_vjp = _sig("tdx_density_vjp", [C.c_void_p, C.POINTER(StatesC), C.c_int * 3, C.c_void_p,
                                     C.c_void_p, C.c_void_p, C.c_void_p])
_pot_vjp = _sig("tdx_potential_vjp", [C.c_void_p, C.POINTER(Model), C.POINTER(StatesC),
                                      C.c_void_p, C.c_void_p, c_dbl_p, C.c_void_p])

EXPORTED = ["tdx_create", "tdx_destroy", "tdx_last_error", "tdx_abi_version",
            "tdx_set_workspace_limit", "tdx_states_query", "tdx_build_states",
            "tdx_occupations", "tdx_response_basis", "tdx_momentum", "tdx_transitions",
            "tdx_pair_density_bytes", "tdx_pair_density", "tdx_pair_density_range",
            "tdx_pair_density_work_bytes", "tdx_pair_density_async",
            "tdx_chi0", "tdx_kernel_matrix",
            "tdx_xc_kernel_grid", "tdx_kernel_matrix_from_grid",
            "tdx_dyson", "tdx_dyson_noalloc", "tdx_dyson_noalloc_max_bytes", "tdx_dsf",
            "tdx_itcf", "tdx_itcf_metrics", "tdx_eta_reference", "tdx_dielectric", "tdx_sg_filter", "tdx_derivative_psd", "tdx_sg_scores", "tdx_residual_itcf", "tdx_sg_select", "tdx_kg_dsf", "tdx_kg_work_bytes", "tdx_kg_conductivity", "tdx_chi0_plan_create", "tdx_chi0_plan_launch",
            "tdx_chi0_plan_destroy", "tdx_chi0_batched", "tdx_chi0_variants",
            "tdx_chi0_set_config", "tdx_chi0_get_config", "tdx_chi0_set_slice_length", "tdx_chi0_bf16x3_slicing", "tdx_autotune_chi0", "tdx_tune_save",
            "tdx_tune_load", "tdx_dyson_work_bytes", "tdx_dyson_async", "tdx_itcf_vjp",
            "tdx_dsf_vjp", "tdx_dyson_vjp", "tdx_chi0_vjp", "tdx_weights_vjp",
            "tdx_occupations_vjp", "tdx_pair_density_vjp", "tdx_potential_vjp",
            "tdx_dyson_kernel_vjp", "tdx_kernel_matrix_vjp", "tdx_density_vjp"]


def check(code):
    if code != OK:
        raise TdxError(code, _lib.tdx_last_error().decode())
    return code


def abi_version():
    return _abi()


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


def _ptr(t: torch.Tensor):
    assert t.is_cuda and t.is_contiguous()
    return C.c_void_p(t.data_ptr())


# ---------------------------------------------------------------- context
class Context:
    def __init__(self, device: int = 0):
        self.device = device
        h = C.c_void_p()
        check(_create(device, C.byref(h)))
        self.handle = h

    def set_workspace_limit(self, nbytes: int):
        check(_set_limit(self.handle, nbytes))

    def close(self):
        if self.handle:
            _destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ----------------------------------------------------------------- states
def make_model(w, keep=None) -> Model:
    """tdx_model from a workload definition; `keep` holds the host arrays."""
    p = w.potential
    pos = np.ascontiguousarray(np.asarray(p.positions, dtype=np.float64).reshape(-1))
    sn = np.ascontiguousarray(np.asarray(p.shell_n2, dtype=np.int32))
    sv = np.ascontiguousarray(np.asarray(p.shell_v, dtype=np.float64))
    if keep is not None:
        keep.extend([pos, sn, sv])
    m = Model()
    m.cell[:] = list(np.asarray(w.cell, dtype=np.float64).reshape(-1))
    m.kgrid[:] = list(w.kgrid)
    m.ecut_wf = w.ecut_wf
    m.n_bands = w.n_bands
    m.n_electrons = w.n_electrons
    m.f_trunc = w.f_trunc
    m.n_atoms = len(p.positions)
    m.positions = pos.ctypes.data_as(c_dbl_p)
    m.shell_unit = p.shell_unit
    m.n_shells = len(p.shell_n2)
    m.shell_n2 = sn.ctypes.data_as(c_int_p)
    m.shell_v = sv.ctypes.data_as(c_dbl_p)
    m.gauss = int(p.gauss)
    m.z_ion = p.z_ion
    m.sigma = p.sigma
    return m


class States:
    """Device-resident Kohn-Sham states (tensors own the memory)."""

    def __init__(self, dims: StatesDims, device):
        dev = torch.device("cuda", device)
        self.npw = torch.zeros(dims.n_k, dtype=torch.int32, device=dev)
        self.nb = torch.zeros(dims.n_k, dtype=torch.int32, device=dev)
        self.miller = torch.zeros((dims.n_k, dims.npw_max, 3), dtype=torch.int32, device=dev)
        self.eps = torch.zeros((dims.n_k, dims.nb_max), dtype=torch.float64, device=dev)
        self.occ = torch.zeros((dims.n_k, dims.nb_max), dtype=torch.float64, device=dev)
        self.coef = torch.zeros((dims.n_k, dims.nb_max, dims.npw_max), dtype=torch.complex128,
                                device=dev)
        c = StatesC()
        c.n_k, c.npw_max, c.nb_max = dims.n_k, dims.npw_max, dims.nb_max
        c.npw, c.nb, c.miller = self.npw.data_ptr(), self.nb.data_ptr(), self.miller.data_ptr()
        c.eps, c.occ, c.coef = self.eps.data_ptr(), self.occ.data_ptr(), self.coef.data_ptr()
        self.c = c

    @property
    def mu(self):
        return self.c.mu

    @property
    def temperature(self):
        return self.c.temperature

    @property
    def omega_cell(self):
        return self.c.omega_cell

    @property
    def beta(self):
        return self.c.beta

    @property
    def density(self):
        """Electron density n of the FDT (library-computed)."""
        return self.c.density

    @property
    def chi0_pref(self):
        """The chi0 normalisation 2 / (N_k Omega) (library-computed)."""
        return self.c.chi0_pref

    @property
    def n_k(self):
        return self.c.n_k


def states_query(w) -> StatesDims:
    keep = []
    d = StatesDims()
    check(_query(C.byref(make_model(w, keep)), C.byref(d)))
    return d


def build_states(ctx: Context, w, temperature: Optional[float] = None, stream=None) -> States:
    keep = []
    m = make_model(w, keep)
    d = StatesDims()
    check(_query(C.byref(m), C.byref(d)))
    st = States(d, ctx.device)
    T = w.temperatures[0] if temperature is None else temperature
    check(_build(ctx.handle, C.byref(m), T, C.byref(st.c), _stream(stream)))
    return st


def occupations(ctx: Context, st: States, temperature: float, n_electrons: float,
                f_trunc: float = 1e-5, stream=None):
    check(_occ(ctx.handle, C.byref(st.c), temperature, n_electrons, f_trunc, _stream(stream)))


# ---------------------------------------------------------- response basis
def response_basis(cell, kgrid, qj, ecut_chi):
    """(Miller int32 [N_G,3] host array, index of G = 0)."""
    cellc = (C.c_double * 9)(*np.asarray(cell, dtype=np.float64).reshape(-1))
    kg = (C.c_int * 3)(*kgrid)
    q = (C.c_int * 3)(*qj)
    n = C.c_int()
    g0 = C.c_int()
    code = _basis(cellc, kg, q, ecut_chi, None, 0, C.byref(n), C.byref(g0))
    if code not in (OK, ERR_SHAPE):
        check(code)
    out = np.zeros((max(n.value, 1), 3), dtype=np.int32)
    check(_basis(cellc, kg, q, ecut_chi, out.ctypes.data_as(c_int_p), n.value, C.byref(n),
                 C.byref(g0)))
    return out[: n.value], g0.value


# ------------------------------------------------------------- transitions
class Transitions:
    def __init__(self, count, device, paired=False):
        dev = torch.device("cuda", device)
        cap = max(int(count), 1)
        self.count = int(count)
        self.paired = bool(paired)
        self.k = torch.zeros(cap, dtype=torch.int32, device=dev)
        self.n = torch.zeros(cap, dtype=torch.int32, device=dev)
        self.m = torch.zeros(cap, dtype=torch.int32, device=dev)
        self.delta = torch.zeros(cap, dtype=torch.float64, device=dev)
        self.df = torch.zeros(cap, dtype=torch.float64, device=dev)
        self.k_offsets = None
        c = TransC()
        c.capacity = self.count
        c.k, c.n, c.m = self.k.data_ptr(), self.n.data_ptr(), self.m.data_ptr()
        c.delta, c.df = self.delta.data_ptr(), self.df.data_ptr()
        c.paired = int(self.paired)
        self.c = c

    def __len__(self):
        return self.count


def transitions(ctx: Context, st: States, qj, thr: float, stream=None,
                out: Optional[Transitions] = None, paired: bool = False) -> Transitions:
    """Screened transition list; `out` (same size and form) is refilled in
    place.  paired=True keeps one transition of each time-reversal pair
    (tdx.h); chi0 then applies the combined weight."""
    q = (C.c_int * 3)(*qj)
    probe = TransC()
    probe.capacity = 0
    probe.paired = int(paired)
    cnt = C.c_int64()
    code = _trans(ctx.handle, C.byref(st.c), q, thr, C.byref(probe), C.byref(cnt), _stream(stream))
    if code not in (OK, ERR_SHAPE):
        check(code)
    if out is not None and out.count == cnt.value and out.paired == bool(paired):
        tr = out
    else:
        tr = Transitions(cnt.value, ctx.device, paired)
        tr.k_offsets = torch.zeros(st.n_k + 1, dtype=torch.int64, device=st.eps.device)
        tr.c.k_offsets = tr.k_offsets.data_ptr()
    check(_trans(ctx.handle, C.byref(st.c), q, thr, C.byref(tr.c), C.byref(cnt), _stream(stream)))
    return tr


# ---------------------------------------------------------- pair densities
def pair_density_bytes(n_trans, n_g, prec):
    return _lib.tdx_pair_density_bytes(n_trans, n_g, PREC[prec])


def pair_density(ctx: Context, st: States, qj, tr: Transitions, gbasis: torch.Tensor,
                 prec: str = "fp64", stream=None, out: Optional[torch.Tensor] = None,
                 n_trans: Optional[int] = None) -> torch.Tensor:
    """P as a flat uint8 device buffer in the layout tdx.h documents, for the
    first n_trans transitions (all by default); `out` (large enough) is
    overwritten in place."""
    n_g = gbasis.shape[0]
    nt = len(tr) if n_trans is None else int(n_trans)
    nbytes = pair_density_bytes(nt, n_g, prec)
    if out is not None and out.numel() >= nbytes:
        P = out
    else:
        P = torch.empty(max(nbytes, 16), dtype=torch.uint8, device=st.eps.device)
    q = (C.c_int * 3)(*qj)
    check(_pair(ctx.handle, C.byref(st.c), q, C.byref(tr.c), nt, _ptr(gbasis), n_g,
                PREC[prec], _ptr(P), _stream(stream)))
    return P


def pair_density_range(ctx: Context, st: States, qj, tr: Transitions, gbasis: torch.Tensor,
                       t_begin: int, t_end: int, prec: str = "fp64", stream=None,
                       out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """P of the transitions t_begin .. t_end - 1 (row 0 = t_begin) as a flat
    uint8 buffer in the layout of pair_density for t_end - t_begin rows."""
    n_g = gbasis.shape[0]
    nbytes = pair_density_bytes(t_end - t_begin, n_g, prec)
    if out is not None and out.numel() >= nbytes:
        P = out
    else:
        P = torch.empty(max(nbytes, 16), dtype=torch.uint8, device=st.eps.device)
    check(_pair_range(ctx.handle, C.byref(st.c), (C.c_int * 3)(*qj), C.byref(tr.c), int(t_begin),
                      int(t_end), _ptr(gbasis), n_g, PREC[prec], _ptr(P), _stream(stream)))
    return P


def pair_density_work_bytes(st: States, n_trans: int) -> int:
    return _lib.tdx_pair_density_work_bytes(C.byref(st.c), int(n_trans))


def pair_density_async(ctx: Context, st: States, qj, tr: Transitions, gbasis: torch.Tensor,
                       P: torch.Tensor, work: torch.Tensor, prec: str = "bf16x3",
                       t_begin: int = 0, t_end: Optional[int] = None, stream=None):
    """pair_density into the given buffer P with the caller's work buffer
    (pair_density_work_bytes): no allocation, copy or memset, so the call
    can be captured in a HIP graph."""
    t_end = len(tr) if t_end is None else int(t_end)
    check(_pair_async(ctx.handle, C.byref(st.c), (C.c_int * 3)(*qj), C.byref(tr.c), int(t_begin),
                      t_end, _ptr(gbasis), gbasis.shape[0], PREC[prec], _ptr(P), _ptr(work),
                      work.numel() * work.element_size(), _stream(stream)))


def pair_density_view(P: torch.Tensor, n_trans: int, n_g: int, prec: str) -> torch.Tensor:
    """complex view [T, N_G] of an FP64/FP32 pair-density buffer."""
    ld = (n_g + 15) // 16 * 16
    if prec == "fp64":
        v = P[: n_trans * ld * 16].view(torch.complex128)
    elif prec == "fp32":
        v = P[: n_trans * ld * 8].view(torch.complex64)
    else:
        raise ValueError("bf16x3 quads have no complex view")
    return v.view(n_trans, ld)[:, :n_g]


# ------------------------------------------------------------------ chi0
def chi0(ctx: Context, tr: Transitions, P: torch.Tensor, n_g: int, prec: str,
         omega: torch.Tensor, eta: float, pref: float, out: Optional[torch.Tensor] = None,
         stream=None, n_trans: Optional[int] = None) -> torch.Tensor:
    """chi0 over the first n_trans transitions (all by default; P must have
    been written for the same count)."""
    n_w = omega.shape[0]
    nt = len(tr) if n_trans is None else int(n_trans)
    if out is None:
        out = torch.empty((n_w, n_g, n_g), dtype=torch.complex128, device=omega.device)
    check(_chi0(ctx.handle, C.byref(tr.c), nt, _ptr(P), n_g, PREC[prec], _ptr(omega), n_w,
                eta, pref, _ptr(out), _stream(stream)))
    return out


def kernel_matrix(ctx: Context, st: States, qj, gbasis: torch.Tensor, xc: str,
                  dens_grid=(0, 0, 0), stream=None) -> torch.Tensor:
    n_g = gbasis.shape[0]
    K = torch.empty((n_g, n_g), dtype=torch.complex128, device=gbasis.device)
    q = (C.c_int * 3)(*qj)
    dg = (C.c_int * 3)(*dens_grid)
    check(_kmat(ctx.handle, C.byref(st.c), q, _ptr(gbasis), n_g, XC[xc], dg, _ptr(K),
                _stream(stream)))
    return K


def xc_kernel_grid(ctx: Context, st: States, dens_grid, stream=None) -> torch.Tensor:
    """f_xc(G) on the FFT grid for the states' current occupations (ALDA)."""
    fx = torch.empty(tuple(dens_grid), dtype=torch.complex128, device=st.eps.device)
    check(_xcgrid(ctx.handle, C.byref(st.c), (C.c_int * 3)(*dens_grid), _ptr(fx),
                  _stream(stream)))
    return fx


def kernel_matrix_from_grid(ctx: Context, st: States, qj, gbasis: torch.Tensor, xc: str,
                            dens_grid=(0, 0, 0), fxg=None, stream=None) -> torch.Tensor:
    """K for one q from a grid of xc_kernel_grid (None for RPA)."""
    n_g = gbasis.shape[0]
    K = torch.empty((n_g, n_g), dtype=torch.complex128, device=gbasis.device)
    check(_kmat_g(ctx.handle, C.byref(st.c), (C.c_int * 3)(*qj), _ptr(gbasis), n_g, XC[xc],
                  (C.c_int * 3)(*dens_grid), _ptr(fxg) if fxg is not None else None, _ptr(K),
                  _stream(stream)))
    return K


def dyson(ctx: Context, chi0_t: torch.Tensor, K: torch.Tensor, i_g0: int,
          stream=None) -> torch.Tensor:
    n_w, n_g, _ = chi0_t.shape
    out = torch.empty(n_w, dtype=torch.complex128, device=chi0_t.device)
    check(_dyson(ctx.handle, _ptr(chi0_t), _ptr(K), n_g, n_w, i_g0, _ptr(out), _stream(stream)))
    return out


def dsf(ctx: Context, chi00: torch.Tensor, omega: torch.Tensor, beta: float, density: float,
        stream=None) -> torch.Tensor:
    S = torch.empty(omega.shape[0], dtype=torch.float64, device=omega.device)
    check(_dsf(ctx.handle, _ptr(chi00), _ptr(omega), omega.shape[0], beta, density, _ptr(S),
               _stream(stream)))
    return S


def itcf(ctx: Context, S: torch.Tensor, omega: torch.Tensor, beta: float, tau: torch.Tensor,
         stream=None) -> torch.Tensor:
    F = torch.empty(tau.shape[0], dtype=torch.float64, device=tau.device)
    check(_itcf(ctx.handle, _ptr(S), _ptr(omega), omega.shape[0], beta, _ptr(tau),
                tau.shape[0], _ptr(F), _stream(stream)))
    return F


# ------------------------------------------------ eta test in imaginary time
METRICS = ("F(beta/2)", "int_0^beta F", "F~(beta/2)", "int_0^beta F~", "chi(q)")


def itcf_metrics(ctx: Context, F: torch.Tensor, tau: torch.Tensor, beta: float, density: float,
                 stream=None) -> torch.Tensor:
    """[n_set][5] metrics (METRICS) of the rows of F [n_set][n_tau] (Sec. 2, Eq. 2)."""
    F = F.reshape(-1, tau.shape[0]).contiguous()
    m = torch.empty((F.shape[0], 5), dtype=torch.float64, device=F.device)
    check(_metrics(ctx.handle, _ptr(F), F.shape[0], _ptr(tau), tau.shape[0], beta, density,
                   _ptr(m), _stream(stream)))
    return m


def eta_reference(metrics, eta, tol: float = 1e-2) -> int:
    """Index of the reference eta: the largest one of the converged run from the
    smallest eta (tdx.h)."""
    m = np.ascontiguousarray(np.asarray(metrics, dtype=np.float64).reshape(-1, 5))
    e = np.ascontiguousarray(np.asarray(eta, dtype=np.float64))
    r = C.c_int()
    check(_eta_ref(m.ctypes.data_as(c_dbl_p), e.ctypes.data_as(c_dbl_p), len(e), tol,
                   C.byref(r)))
    return r.value


# ------------------------------------------------- dielectric properties
def momentum(cell, kgrid, qj):
    """(q Cartesian [3], |q|^2) of q = sum_i (qj_i / kgrid_i) b_i (tdx_momentum)."""
    cellc = (C.c_double * 9)(*np.asarray(cell, dtype=np.float64).reshape(-1))
    q = (C.c_double * 3)()
    q2 = C.c_double()
    check(_momentum(cellc, (C.c_int * 3)(*kgrid), (C.c_int * 3)(*qj), q, C.byref(q2)))
    return np.array(list(q)), q2.value


def q_squared(cell, kgrid, qj) -> float:
    """|q|^2 (bohr^-2) of q = sum_i (qj_i / kgrid_i) b_i."""
    return momentum(cell, kgrid, qj)[1]


def dielectric(ctx: Context, S: torch.Tensor, omega: torch.Tensor, beta: float, density: float,
               q2: float, stream=None):
    """(chi, eps^{-1}, sigma) [n_w] complex128 from S: Im chi by the FDT, Re chi
    by Kramers-Kronig on the grid, Eqs. A-1 and A-2 (tdx.h)."""
    n = omega.shape[0]
    out = [torch.empty(n, dtype=torch.complex128, device=omega.device) for _ in range(3)]
    check(_dielectric(ctx.handle, _ptr(S), _ptr(omega), n, beta, density, q2, _ptr(out[0]),
                      _ptr(out[1]), _ptr(out[2]), _stream(stream)))
    return tuple(out)


# ------------------------------------- attenuation of narrow-band fluctuations
SG_SCORES = ("RSS", "k", "AICc", "P_freq", "P_curv")
RESIDUAL = ("max|F_n/F|", "Fbar_n/F(beta/2)", "sigma_n/F(beta/2)")


def sg_filter(ctx: Context, S: torch.Tensor, windows, degrees, stream=None):
    """(Sp, hdiag) [n_filt][n_w]: a bank of Savitzky-Golay filters applied to S
    and the smoother diagonals (Sec. 3; tdx.h)."""
    n = S.shape[0]
    win = (C.c_int * len(windows))(*[int(x) for x in windows])
    deg = (C.c_int * len(degrees))(*[int(x) for x in degrees])
    if len(windows) != len(degrees):
        raise ValueError("windows and degrees differ in length")
    Sp = torch.empty((len(windows), n), dtype=torch.float64, device=S.device)
    hd = torch.empty_like(Sp)
    check(_sgf(ctx.handle, _ptr(S.contiguous()), n, win, deg, len(windows), _ptr(Sp), _ptr(hd),
               _stream(stream)))
    return Sp, hd


def derivative_psd(ctx: Context, S: torch.Tensor, omega: torch.Tensor, nu: torch.Tensor,
                   stream=None) -> torch.Tensor:
    """[n_set][n_nu] power of dS/dw at the frequencies nu (Sec. 3, Fig. 3)."""
    S = S.reshape(-1, omega.shape[0]).contiguous()
    out = torch.empty((S.shape[0], nu.shape[0]), dtype=torch.float64, device=S.device)
    check(_dpsd(ctx.handle, _ptr(S), _ptr(omega), omega.shape[0], S.shape[0], _ptr(nu),
                nu.shape[0], _ptr(out), _stream(stream)))
    return out


def sg_scores(ctx: Context, S: torch.Tensor, Sp: torch.Tensor, hdiag: torch.Tensor,
              omega: torch.Tensor, nu: torch.Tensor, stream=None) -> torch.Tensor:
    """[n_filt][5] scores (SG_SCORES) of a filter bank (Sec. 3; tdx.h)."""
    out = torch.empty((Sp.shape[0], 5), dtype=torch.float64, device=S.device)
    check(_sgs(ctx.handle, _ptr(S), _ptr(Sp), _ptr(hdiag), _ptr(omega), omega.shape[0],
               Sp.shape[0], _ptr(nu) if nu.numel() else None, nu.shape[0], _ptr(out),
               _stream(stream)))
    return out


def residual_itcf(ctx: Context, F_ref: torch.Tensor, F_p: torch.Tensor, tau: torch.Tensor,
                  beta: float, stream=None) -> torch.Tensor:
    """[n_set][3] conditions (RESIDUAL) on F_n = F_ref - F_p (Eqs. 5 and 7)."""
    F_p = F_p.reshape(-1, tau.shape[0]).contiguous()
    out = torch.empty((F_p.shape[0], 3), dtype=torch.float64, device=F_p.device)
    check(_resid(ctx.handle, _ptr(F_ref), _ptr(F_p), F_p.shape[0], _ptr(tau), tau.shape[0],
                 beta, _ptr(out), _stream(stream)))
    return out


def sg_select(scores, resid, n_w: int, lam_f: float = 100.0, lam_c: float = 10.0,
              mean_tol: float = 4e-3, sigma_tol: float = 4.2e-5) -> int:
    """Index of the selected filter, or -1 (tdx.h)."""
    sc = np.ascontiguousarray(np.asarray(scores, dtype=np.float64))
    rs = None if resid is None else np.ascontiguousarray(np.asarray(resid, dtype=np.float64))
    best = C.c_int(-1)
    check(_sgsel(sc.ctypes.data_as(c_dbl_p), None if rs is None else rs.ctypes.data_as(c_dbl_p),
                 sc.shape[0], n_w, lam_f, lam_c, mean_tol, sigma_tol, C.byref(best)))
    return best.value


@dataclass
class Attenuation:
    Sp: torch.Tensor          # [n_filt][n_w] filtered spectra
    scores: torch.Tensor      # [n_filt][5] (SG_SCORES)
    resid: torch.Tensor       # [n_filt][3] (RESIDUAL)
    best: dict                # degree -> index of its selected filter (or -1)


def attenuate(ctx: Context, S: torch.Tensor, omega: torch.Tensor, beta: float,
              tau: torch.Tensor, windows, degrees, nu: torch.Tensor, lam_f: float = 100.0,
              lam_c: float = 10.0, mean_tol: float = 4e-3, sigma_tol: float = 4.2e-5,
              stream=None) -> Attenuation:
    """The grid search of Sec. 3 over the (window, degree) pairs: filter bank,
    scores, F of every filtered spectrum (Eq. 1), the residual conditions
    (Eqs. 5 and 7) and the selected window of each degree."""
    Sp, hd = sg_filter(ctx, S, windows, degrees, stream)
    sc = sg_scores(ctx, S, Sp, hd, omega, nu, stream)
    F_ref = itcf(ctx, S, omega, beta, tau, stream)
    F_p = (torch.stack([itcf(ctx, Sp[f], omega, beta, tau, stream) for f in range(Sp.shape[0])])
           if Sp.shape[0] else torch.empty((0, tau.shape[0]), dtype=torch.float64,
                                           device=S.device))
    rs = residual_itcf(ctx, F_ref, F_p, tau, beta, stream)
    sc_h, rs_h = sc.cpu().numpy(), rs.cpu().numpy()
    deg = np.asarray(degrees)
    best = {}
    for d in sorted(set(int(x) for x in degrees)):
        rows = np.nonzero(deg == d)[0]
        b = sg_select(sc_h[rows], rs_h[rows], S.shape[0], lam_f, lam_c, mean_tol, sigma_tol)
        best[d] = int(rows[b]) if b >= 0 else -1
    return Attenuation(Sp, sc, rs, best)


# ---------------------------------------------------- Kubo-Greenwood route
KG_Q2 = 4.0 * math.pi  # the dielectric step at this q^2 gives eps^{-1} = 1 + chi*


def kg_dsf(ctx: Context, sigma: torch.Tensor, omega: torch.Tensor, beta: float, density: float,
           stream=None) -> torch.Tensor:
    """S* = v(q) S [n_w] of the optical limit from a conductivity sigma
    (complex128 [n_w]) (Sec. A.3; tdx.h)."""
    S = torch.empty(omega.shape[0], dtype=torch.float64, device=omega.device)
    check(_kgdsf(ctx.handle, _ptr(sigma.contiguous()), _ptr(omega), omega.shape[0], beta,
                 density, _ptr(S), _stream(stream)))
    return S


def kg_work_bytes(n_trans: int, n_w: int) -> int:
    return int(_kg_work(int(n_trans), int(n_w)))


def kg_conductivity(ctx: Context, st: States, omega: torch.Tensor, eta: float, thr: float,
                    tr: Optional[Transitions] = None, work: Optional[torch.Tensor] = None,
                    stream=None) -> torch.Tensor:
    """Kubo-Greenwood conductivity of the states (complex128 [n_w]), the
    trace average broadened by eta (Sec. A.3; tdx.h), over the q = 0
    transitions screened by thr (built here unless `tr` is that list)."""
    if tr is None:
        tr = transitions(ctx, st, (0, 0, 0), thr, stream=stream)
    n_w = omega.shape[0]
    if work is None:
        work = torch.empty(max(kg_work_bytes(len(tr), n_w), 1), dtype=torch.uint8,
                           device=omega.device)
    sigma = torch.empty(n_w, dtype=torch.complex128, device=omega.device)
    check(_kgsig(ctx.handle, C.byref(st.c), C.byref(tr.c), len(tr), _ptr(omega), n_w, eta,
                 _ptr(sigma), _ptr(work), work.numel(), _stream(stream)))
    return sigma


def kg_dielectric(ctx: Context, S_star: torch.Tensor, omega: torch.Tensor, beta: float,
                  density: float, stream=None):
    """(chi*, eps^{-1}, sigma) from S*: Re chi* by Kramers-Kronig,
    eps^{-1} = 1 + chi*, sigma = i w (1 - eps) / (4 pi) (Sec. A.3)."""
    return dielectric(ctx, S_star, omega, beta, density, KG_Q2, stream)


# ------------------------------------------------------------ reverse mode
# Cotangent convention: real x -> dL = sum xbar dx; complex z ->
# dL = Re sum conj(zbar) dz (PyTorch's convention for complex gradients).
def itcf_vjp(ctx: Context, S: torch.Tensor, omega: torch.Tensor, beta: float, tau: torch.Tensor,
             F_bar: torch.Tensor, stream=None):
    """(S_bar [n_w], tau_bar [n_tau], beta_bar [1]) of F = itcf(S, omega, beta, tau)."""
    dev = S.device
    S_bar = torch.empty_like(S)
    tau_bar = torch.empty_like(tau)
    beta_bar = torch.empty(1, dtype=torch.float64, device=dev)
    check(_itcf_vjp(ctx.handle, _ptr(S), _ptr(omega), omega.shape[0], beta, _ptr(tau),
                    tau.shape[0], _ptr(F_bar), _ptr(S_bar), _ptr(tau_bar), _ptr(beta_bar),
                    _stream(stream)))
    return S_bar, tau_bar, beta_bar


def dsf_vjp(ctx: Context, chi00: torch.Tensor, omega: torch.Tensor, beta: float, density: float,
            S_bar: torch.Tensor, stream=None):
    """(chi00_bar complex [n_w], beta_bar [1]) of S = dsf(chi00, omega, beta, density)."""
    chi_bar = torch.empty_like(chi00)
    beta_bar = torch.empty(1, dtype=torch.float64, device=chi00.device)
    check(_dsf_vjp(ctx.handle, _ptr(chi00), _ptr(omega), omega.shape[0], beta, density,
                   _ptr(S_bar), _ptr(chi_bar), _ptr(beta_bar), _stream(stream)))
    return chi_bar, beta_bar


def dyson_vjp(ctx: Context, chi0_t: torch.Tensor, K: torch.Tensor, i_g0: int,
              chi00_bar: torch.Tensor, stream=None):
    """(u, v) [n_w, n_g] with chi0_bar(w) = u(w) v(w)^H; raises on a singular pivot."""
    n_w, n_g, _ = chi0_t.shape
    dev = chi0_t.device
    u = torch.empty((n_w, n_g), dtype=torch.complex128, device=dev)
    v = torch.empty_like(u)
    work = torch.empty(dyson_work_bytes(n_g, n_w), dtype=torch.uint8, device=dev)
    info = torch.zeros(n_w, dtype=torch.int32, device=dev)
    check(_dyson_vjp(ctx.handle, _ptr(chi0_t), _ptr(K), n_g, n_w, i_g0, _ptr(chi00_bar), _ptr(u),
                     _ptr(v), _ptr(work), _ptr(info), _stream(stream)))
    bad = torch.nonzero(info).flatten()
    if bad.numel():
        raise TdxError(ERR_NUMERIC, f"Dyson matrix singular at frequency {int(bad[0])}")
    return u, v


def chi0_vjp(ctx: Context, tr: Transitions, P: torch.Tensor, n_g: int, omega: torch.Tensor,
             eta: float, pref: float, u: torch.Tensor, v: torch.Tensor, want_rho: bool = False,
             stream=None, t_begin: int = 0, t_end: Optional[int] = None,
             w_out: Optional[torch.Tensor] = None):
    """(w_bar float64 [n, 3] = (df_bar, delta_bar, eta_bar_t), rho_bar complex
    [n, ld] or None) of the transitions t_begin .. t_end - 1 (all by default),
    n = t_end - t_begin, from their FP64 pair densities P (row 0 = t_begin);
    w_bar is written into w_out ([n, 3], contiguous) if given."""
    dev = omega.device
    t_end = len(tr) if t_end is None else int(t_end)
    n = t_end - int(t_begin)
    ld = (n_g + 15) // 16 * 16
    w_bar = (w_out if w_out is not None else
             torch.zeros((max(n, 1), 3), dtype=torch.float64, device=dev))
    rho_bar = (torch.zeros((max(n, 1), ld), dtype=torch.complex128, device=dev)
               if want_rho else None)
    check(_chi0_vjp(ctx.handle, C.byref(tr.c), int(t_begin), t_end, _ptr(P), n_g, _ptr(omega),
                    omega.shape[0], eta, pref, _ptr(u), _ptr(v), _ptr(w_bar),
                    _ptr(rho_bar) if rho_bar is not None else None, _stream(stream)))
    return w_bar[:n], (rho_bar[:n] if rho_bar is not None else None)


def weights_vjp(ctx: Context, st: States, qj, tr: Transitions, w_bar: torch.Tensor,
                occ_bar: torch.Tensor, eps_bar: torch.Tensor, eta_bar: torch.Tensor,
                stream=None):
    """Accumulate occ_bar, eps_bar [n_k, nb_max] and eta_bar [1] from one q's
    w_bar [T, 3] (chi0_vjp over the whole list)."""
    q = (C.c_int * 3)(*qj)
    check(_weights_vjp(ctx.handle, C.byref(st.c), q, C.byref(tr.c), len(tr), _ptr(w_bar),
                       _ptr(occ_bar), _ptr(eps_bar), _ptr(eta_bar), _stream(stream)))


def occupations_vjp(ctx: Context, st: States, occ_bar: torch.Tensor, eps_bar: torch.Tensor,
                    stream=None) -> torch.Tensor:
    """T_bar [1] of the occupations at the states' temperature; eps_bar += through mu."""
    T_bar = torch.empty(1, dtype=torch.float64, device=occ_bar.device)
    check(_occ_vjp(ctx.handle, C.byref(st.c), _ptr(occ_bar), _ptr(eps_bar), _ptr(T_bar),
                   _stream(stream)))
    return T_bar


def pair_density_vjp(ctx: Context, st: States, qj, tr: Transitions, gbasis: torch.Tensor,
                     rho_bar: torch.Tensor, coef_bar: torch.Tensor, stream=None,
                     t_begin: int = 0, t_end: Optional[int] = None):
    """Accumulate coef_bar [n_k, nb_max, npw_max] from rho_bar of the
    transitions t_begin .. t_end - 1 of one q (row 0 = t_begin)."""
    q = (C.c_int * 3)(*qj)
    t_end = len(tr) if t_end is None else int(t_end)
    check(_pair_vjp(ctx.handle, C.byref(st.c), q, C.byref(tr.c), int(t_begin), t_end,
                    _ptr(gbasis), gbasis.shape[0], _ptr(rho_bar), _ptr(coef_bar),
                    _stream(stream)))


def potential_vjp(ctx: Context, w, st: States, eps_bar: torch.Tensor, coef_bar: torch.Tensor,
                  stream=None) -> np.ndarray:
    """Gradient with respect to the tabulated shell values of w's potential."""
    keep = []
    m = make_model(w, keep)
    out = np.zeros(len(w.potential.shell_n2), dtype=np.float64)
    check(_pot_vjp(ctx.handle, C.byref(m), C.byref(st.c), _ptr(eps_bar), _ptr(coef_bar),
                   out.ctypes.data_as(c_dbl_p), _stream(stream)))
    return out


def dyson_kernel_vjp(ctx: Context, chi0_t: torch.Tensor, K: torch.Tensor, i_g0: int,
                     chi00_bar: torch.Tensor, K_bar: Optional[torch.Tensor] = None,
                     stream=None) -> torch.Tensor:
    """K_bar (+=, complex128 [n_g][n_g]) of chi00 = [(1 - chi0 K)^{-1} chi0]_{g0 g0}."""
    n_w, n_g, _ = chi0_t.shape
    if K_bar is None:
        K_bar = torch.zeros((n_g, n_g), dtype=torch.complex128, device=chi0_t.device)
    check(_dyson_k_vjp(ctx.handle, _ptr(chi0_t), _ptr(K), n_g, n_w, i_g0,
                       _ptr(chi00_bar.contiguous()), _ptr(K_bar), _stream(stream)))
    return K_bar


def kernel_matrix_vjp(ctx: Context, st: States, gbasis: torch.Tensor, dens_grid,
                      K_bar: torch.Tensor, fxc_bar: torch.Tensor, stream=None):
    """fxc_bar (+=, float64 [N_r], grid order) from the ALDA part of K."""
    check(_kmat_vjp(ctx.handle, C.byref(st.c), _ptr(gbasis), gbasis.shape[0],
                    (C.c_int * 3)(*dens_grid), _ptr(K_bar), _ptr(fxc_bar), _stream(stream)))


def density_vjp(ctx: Context, st: States, dens_grid, fxc_bar: torch.Tensor,
                occ_bar: torch.Tensor, coef_bar: Optional[torch.Tensor] = None, stream=None):
    """occ_bar (+=) and coef_bar (+=, optional) through the density from fxc_bar."""
    check(_dens_vjp(ctx.handle, C.byref(st.c), (C.c_int * 3)(*dens_grid), _ptr(fxc_bar),
                    _ptr(occ_bar), None if coef_bar is None else _ptr(coef_bar),
                    _stream(stream)))


# --------------------------------------------------------------- pipeline
@dataclass
class QOut:
    qj: tuple
    basis: np.ndarray
    i_g0: int
    n_trans: int
    omega: torch.Tensor
    chi0: Optional[torch.Tensor]
    K: torch.Tensor
    chi00: torch.Tensor
    S: torch.Tensor
    tau: torch.Tensor
    F: torch.Tensor
    beta: float
    density: float


def run_q(ctx: Context, w, st: States, iq: int, prec: str = "fp64", omega=None,
          keep_chi0: bool = True, stream=None, paired: bool = True) -> QOut:
    """transitions -> pair densities -> chi0 -> K -> Dyson -> S -> F for one q
    (over the time-reversal paired transition list unless paired=False)."""
    dev = st.eps.device
    qj = tuple(w.qs[iq])
    T = w.temperatures[iq]
    if abs(st.temperature - T) > 0:
        occupations(ctx, st, T, w.n_electrons, w.f_trunc, stream)
    basis, i_g0 = response_basis(w.cell, w.kgrid, qj, w.ecut_chi[iq])
    gb = torch.from_numpy(basis).to(dev)
    tr = transitions(ctx, st, qj, w.f_trans_thr, stream, paired=paired)
    P = pair_density(ctx, st, qj, tr, gb, prec, stream)
    om = torch.as_tensor(w.omega_grid(iq) if omega is None else np.asarray(omega, dtype=np.float64),
                         device=dev)
    c0 = chi0(ctx, tr, P, len(basis), prec, om, w.eta, st.chi0_pref, stream=stream)
    del P
    K = kernel_matrix(ctx, st, qj, gb, w.xc, w.dens_grid, stream)
    c00 = dyson(ctx, c0, K, i_g0, stream)
    beta, n = st.beta, st.density
    S = dsf(ctx, c00, om, beta, n, stream)
    tau = torch.as_tensor(w.tau_grid(iq), device=dev)
    F = itcf(ctx, S, om, beta, tau, stream)
    return QOut(qj, basis, i_g0, len(tr), om, c0 if keep_chi0 else None, K, c00, S, tau, F,
                beta, n)


# ------------------------------------------------------ batches and tuning
class Chi0Item:
    """One q of a batch; keeps the tensors it points to alive."""

    def __init__(self, tr: Transitions, P: torch.Tensor, n_g: int, omega: torch.Tensor,
                 eta: float, pref: float, out: Optional[torch.Tensor] = None,
                 n_trans: Optional[int] = None, p_rows: int = 0):
        """The first n_trans transitions (all by default) of P, a buffer written
        for p_rows transitions (0: n_trans)."""
        n_w = omega.shape[0]
        self.tr, self.P, self.omega, self.eta, self.pref = tr, P, omega, eta, pref
        self.out = out if out is not None else torch.empty(
            (n_w, n_g, n_g), dtype=torch.complex128, device=omega.device)
        c = Chi0ItemC()
        c.tl = C.pointer(tr.c)
        c.n_trans = len(tr) if n_trans is None else int(n_trans)
        c.p_rows = int(p_rows)
        c.P = P.data_ptr()
        c.n_g = n_g
        c.omega = omega.data_ptr()
        c.n_w = n_w
        c.eta = eta
        c.pref = pref
        c.chi0 = self.out.data_ptr()
        self.c = c


def _item_array(items):
    arr = (Chi0ItemC * len(items))()
    for i, it in enumerate(items):
        arr[i] = it.c
    return arr


class Chi0Plan:
    """Work queue of a ragged batch; launch() is one persistent kernel
    (split-BF16) and can be captured in a HIP graph."""

    def __init__(self, ctx: Context, items, prec: str = "bf16x3"):
        self.ctx, self.items = ctx, list(items)
        self._arr = _item_array(self.items)
        h = C.c_void_p()
        check(_plan_create(ctx.handle, self._arr, len(self.items), PREC[prec], C.byref(h)))
        self.handle = h

    def launch(self, stream=None):
        check(_plan_launch(self.ctx.handle, self.handle, _stream(stream)))

    def close(self):
        if self.handle:
            _plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def chi0_batched(ctx: Context, items, prec: str = "bf16x3", stream=None):
    arr = _item_array(items)
    check(_batched(ctx.handle, arr, len(items), PREC[prec], _stream(stream)))
    return [it.out for it in items]


def chi0_variants(prec: str = "bf16x3") -> int:
    n = C.c_int()
    check(_variants(PREC[prec], C.byref(n)))
    return n.value


def chi0_set_config(ctx: Context, n_g: int, variant: int, slice_log2: int, prec: str = "bf16x3"):
    check(_set_cfg(ctx.handle, PREC[prec], n_g, variant, slice_log2))


def chi0_set_slice_length(ctx: Context, n: int):
    """Fixed chi0 slice length for later calls on ctx (0: chosen per call)."""
    check(_set_slice(ctx.handle, int(n)))


def chi0_bf16x3_slicing(n_cu: int, variant: int, n_trans: int, n_g: int, n_w: int,
                        slice_log2: int = 20):
    """(slice length, slice count) a split-BF16 contraction takes with no fixed
    length (host only; tdx_chi0_bf16x3_slicing)."""
    ln, ns = C.c_int64(), C.c_int()
    check(_bf_slicing(int(n_cu), int(variant), int(n_trans), int(n_g), int(n_w),
                      int(slice_log2), C.byref(ln), C.byref(ns)))
    return ln.value, ns.value


def chi0_get_config(ctx: Context, n_g: int, prec: str = "bf16x3"):
    v, s = C.c_int(), C.c_int()
    check(_get_cfg(ctx.handle, PREC[prec], n_g, C.byref(v), C.byref(s)))
    return v.value, s.value


def autotune_chi0(ctx: Context, probe: Chi0Item, max_trans: int = 1 << 21,
                  prec: str = "bf16x3"):
    v, s, ms = C.c_int(), C.c_int(), C.c_double()
    check(_autotune(ctx.handle, C.byref(probe.c), PREC[prec], max_trans, C.byref(v),
                    C.byref(s), C.byref(ms)))
    return v.value, s.value, ms.value


def tune_save(ctx: Context, path: str):
    check(_tune_save(ctx.handle, path.encode()))


def tune_load(ctx: Context, path: str):
    check(_tune_load(ctx.handle, path.encode()))


def dyson_work_bytes(n_g: int, n_w: int) -> int:
    return _lib.tdx_dyson_work_bytes(n_g, n_w)


def dyson_async(ctx: Context, chi0_t: torch.Tensor, K: torch.Tensor, i_g0: int,
                chi00: torch.Tensor, work: torch.Tensor, info: torch.Tensor, stream=None):
    n_w, n_g, _ = chi0_t.shape
    check(_dyson_async(ctx.handle, _ptr(chi0_t), _ptr(K), n_g, n_w, i_g0, _ptr(chi00),
                       _ptr(work), _ptr(info), _stream(stream)))


@dataclass
class EtaScan:
    eta: np.ndarray        # [n_eta], increasing
    omega: torch.Tensor    # [n_w]
    tau: torch.Tensor      # [n_tau]
    S: torch.Tensor        # [n_eta][n_w]
    F: torch.Tensor        # [n_eta][n_tau]
    metrics: np.ndarray    # [n_eta][5], METRICS
    ref_index: int         # the reference eta: eta[ref_index]
    beta: float
    density: float
    n_trans: int


def eta_scan(ctx: Context, w, st: States, iq: int, etas, prec: str = "bf16x3",
             tol: float = 1e-2, paired: bool = True, stream=None) -> EtaScan:
    """The eta-convergence test in imaginary time (Sec. 2, Eq. 2, Fig. 2): chi0
    for every eta from one set of pair densities (split-BF16: one persistent
    launch for all of them), then Dyson, S and F per eta, the metrics of the
    F and the reference eta."""
    etas = np.asarray(etas, dtype=np.float64)
    if etas.ndim != 1 or len(etas) == 0 or np.any(np.diff(etas) <= 0):
        raise ValueError("etas must be a non-empty increasing sequence")
    dev = st.eps.device
    qj = tuple(w.qs[iq])
    T = w.temperatures[iq]
    if abs(st.temperature - T) > 0:
        occupations(ctx, st, T, w.n_electrons, w.f_trunc, stream)
    basis, i_g0 = response_basis(w.cell, w.kgrid, qj, w.ecut_chi[iq])
    n_g = len(basis)
    gb = torch.from_numpy(basis).to(dev)
    tr = transitions(ctx, st, qj, w.f_trans_thr, stream, paired=paired)
    P = pair_density(ctx, st, qj, tr, gb, prec, stream)
    om = torch.as_tensor(w.omega_grid(iq), device=dev)
    pref = st.chi0_pref
    if prec == "bf16x3":
        items = [Chi0Item(tr, P, n_g, om, float(e), pref) for e in etas]
        plan = Chi0Plan(ctx, items, prec)
        plan.launch(stream)
        chis = [it.out for it in items]
    else:
        plan = None
        chis = [chi0(ctx, tr, P, n_g, prec, om, float(e), pref, stream=stream) for e in etas]
    K = kernel_matrix(ctx, st, qj, gb, w.xc, w.dens_grid, stream)
    beta, n = st.beta, st.density
    tau = torch.as_tensor(w.tau_grid(iq), device=dev)
    S = torch.stack([dsf(ctx, dyson(ctx, c, K, i_g0, stream), om, beta, n, stream) for c in chis])
    F = torch.stack([itcf(ctx, S[i], om, beta, tau, stream) for i in range(len(etas))])
    if plan is not None:
        plan.close()
    del chis, P
    m = itcf_metrics(ctx, F, tau, beta, n, stream).cpu().numpy()
    return EtaScan(etas, om, tau, S, F, m, eta_reference(m, etas, tol), beta, n, len(tr))
