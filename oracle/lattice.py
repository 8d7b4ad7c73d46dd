"""Oracle geometry: reciprocal lattice, Monkhorst-Pack grid, plane-wave spheres.

Test infrastructure only (see the package docstring).
"""
from __future__ import annotations

import itertools
import math

import numpy as np


def reciprocal(cell) -> np.ndarray:
    """Rows b_i with a_i . b_j = 2 pi delta_ij."""
    A = np.asarray(cell, dtype=np.float64)
    return 2.0 * math.pi * np.linalg.inv(A).T


def volume(cell) -> float:
    return abs(float(np.linalg.det(np.asarray(cell, dtype=np.float64))))


def mp_kpoints(kgrid):
    """Monkhorst-Pack points in reduced coordinates.

    k_r = sum_i (2 r_i + 1 - N_i) / (2 N_i) b_i, r_i = 0..N_i-1, flattened
    with r_3 fastest.  The set is closed under k -> -k.
    Returns (reduced (N_k,3), multi-index (N_k,3)).
    """
    N = np.asarray(kgrid)
    idx = np.array(list(itertools.product(range(N[0]), range(N[1]), range(N[2]))))
    red = (2 * idx + 1 - N) / (2.0 * N)
    return red, idx


def kindex(r, kgrid) -> int:
    return int((r[0] * kgrid[1] + r[1]) * kgrid[2] + r[2])


def kq_map(kgrid, qj):
    """For q = sum_i qj_i / N_i b_i: k_r + q = k_{r'} + G_s.

    Returns (kp index (N_k,), G_s Miller (N_k,3)).
    """
    N = np.asarray(kgrid)
    _, idx = mp_kpoints(kgrid)
    s = idx + np.asarray(qj)
    rp = np.mod(s, N)
    gs = (s - rp) // N
    kp = (rp[:, 0] * N[1] + rp[:, 1]) * N[2] + rp[:, 2]
    return kp.astype(np.int64), gs.astype(np.int64)


def gsphere(B, kred, ecut):
    """All Miller triples m with 1/2 |k + m.B|^2 <= ecut.

    Sorted by |k+G|^2, ties by Miller triple (lexicographic).  The order is
    internal to the oracle: nothing it returns depends on it.
    """
    B = np.asarray(B)
    kc = np.asarray(kred) @ B
    A = 2.0 * math.pi * np.linalg.inv(B).T          # rows a_i
    kmax = math.sqrt(2.0 * ecut)
    bound = [int(math.floor((kmax + np.linalg.norm(kc)) * np.linalg.norm(A[i])
                            / (2 * math.pi))) + 1 for i in range(3)]
    rng = [np.arange(-b, b + 1) for b in bound]
    m = np.array(np.meshgrid(*rng, indexing="ij")).reshape(3, -1).T
    p = kc + m @ B
    e = 0.5 * np.einsum("ij,ij->i", p, p)
    keep = e <= ecut
    m, e = m[keep], e[keep]
    order = np.lexsort((m[:, 2], m[:, 1], m[:, 0], e))
    return m[order].astype(np.int64)


def response_basis(B, qred, ecut_chi):
    """B(q) = {G : 1/2 |q+G|^2 <= E_chi, q + G != 0}, with G = 0 required.

    The reported response element is G = 0, i.e. the q+G = q component.
    Returns (Miller (N_G,3), index of G = 0).
    """
    m = gsphere(B, qred, ecut_chi)
    p = (np.asarray(qred) + m) @ np.asarray(B)
    nz = np.einsum("ij,ij->i", p, p) > 1e-20
    m = m[nz]
    hit = np.where(~m.any(axis=1))[0]
    if len(hit) != 1:
        raise ValueError("G = 0 must lie inside the response basis")
    return m, int(hit[0])
