"""Plain FP64 CPU oracle for the Tamm-Dancoff BSE Hamiltonian.

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
CPU-baseline leg of the benchmark, never by the product library.  The heavy
loops live in oracle.c (built into liboracle.so by ``oracle.build``); this
module marshals numpy arrays and adds the small dense steps (eigensolve,
spectrum, adjoint) in numpy.

Paper: J. Yan, K. W. Jacobsen, K. S. Thygesen, "Optical properties of bulk
semiconductors and graphene/boron-nitride: the Bethe-Salpeter equation with
derivative discontinuity-corrected DFT energies", PRB 86, 045208 (2012).
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np

HARTREE_EV = 27.211386245988
_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None


def lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(_HERE, "liboracle.so")
        if not os.path.exists(path):
            from . import build as _b
            _b.build()
        _LIB = ctypes.CDLL(path)
        P = ctypes.c_void_p
        i = ctypes.c_int
        _LIB.oracle_fold.argtypes = [P, i, i, P, P]
        _LIB.oracle_pair_density_full.argtypes = [P, P, P, P, P, i, P]
        _LIB.oracle_pair_density_sep.argtypes = [P, P, P, P, P, i, P]
        _LIB.oracle_pair_density_batch.argtypes = [P, i, P, i, P, P, P, P, i, i, P]
        _LIB.oracle_build_blocks.argtypes = [P, P, i, i, ctypes.c_double, i, P, P, P, P, P, P, P, i, i, P]
        _LIB.oracle_build_blocks.restype = i
        _LIB.oracle_num_threads.restype = i
    return _LIB


def _p(a: np.ndarray):
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.c_void_p)


def num_threads() -> int:
    return int(lib().oracle_num_threads())


def fold(kmesh, ka: int, kb: int):
    """(iq, m0) with k' - k = q + G0 (Sec. III.A: q mesh shaped like the k mesh)."""
    km = np.asarray(kmesh, dtype=np.int32)
    iq = np.zeros(1, dtype=np.int32)
    m0 = np.zeros(3, dtype=np.int32)
    lib().oracle_fold(_p(km), int(ka), int(kb), _p(iq), _p(m0))
    return int(iq[0]), m0


def pair_density(grid, ua, ub, m0, gvec, separable=False):
    """n(m) = sum_j conj(ua) ub exp(-2 pi i (m - m0).j / N) on the listed Miller indices."""
    g = np.asarray(grid, dtype=np.int32)
    ua = np.ascontiguousarray(ua, dtype=np.complex128)
    ub = np.ascontiguousarray(ub, dtype=np.complex128)
    m0 = np.ascontiguousarray(m0, dtype=np.int32)
    gv = np.ascontiguousarray(gvec, dtype=np.int32)
    out = np.zeros(len(gv), dtype=np.complex128)
    fn = lib().oracle_pair_density_sep if separable else lib().oracle_pair_density_full
    fn(_p(g), _p(ua), _p(ub), _p(m0), _p(gv), len(gv), _p(out))
    return out


def pair_density_items(sys, items, separable=True):
    """Batch of pair densities: items = [(ka, a, kb, b), ...] with the fold of (ka, kb).
    Returns [n][ng_max] (entries past ng(q) are zero)."""
    items = list(items)
    arr = np.zeros((len(items), 6), dtype=np.int32)
    m0s = np.zeros((len(items), 3), dtype=np.int32)
    for i, (ka, a, kb, b) in enumerate(items):
        iq, m0 = fold(sys.kmesh, ka, kb)
        arr[i, :5] = (ka, a, kb, b, iq)
        m0s[i] = m0
    out = np.zeros((len(items), sys.ng_max), dtype=np.complex128)
    g = np.asarray(sys.grid, dtype=np.int32)
    lib().oracle_pair_density_batch(_p(g), sys.nb, _p(sys.u), sys.ng_max, _p(sys.ng), _p(sys.gvec),
                                    _p(arr), _p(m0s), len(items), int(separable), _p(out))
    return out


def build_blocks(sys, blocks, separable=True):
    """H blocks for the ordered k pairs in ``blocks`` ([n][2]), each [nv*nc][nv*nc] in eV."""
    blocks = np.ascontiguousarray(np.asarray(blocks, dtype=np.int32).reshape(-1, 2))
    nt = sys.nv * sys.nc
    out = np.zeros((len(blocks), nt, nt), dtype=np.complex128)
    g = np.asarray(sys.grid, dtype=np.int32)
    km = np.asarray(sys.kmesh, dtype=np.int32)
    rc = lib().oracle_build_blocks(_p(g), _p(km), sys.nv, sys.nc, sys.omega_cell, sys.ng_max,
                                   _p(sys.ng), _p(sys.gvec), _p(sys.vx), _p(sys.u), _p(sys.eps),
                                   _p(sys.W), _p(blocks), len(blocks), int(separable), _p(out))
    assert rc == 0
    return out


def build_H(sys, separable=True):
    """The whole Hamiltonian: every one of the Nk^2 blocks computed on its own."""
    nk, nt = sys.nk, sys.nv * sys.nc
    blocks = np.array([(a, b) for a in range(nk) for b in range(nk)], dtype=np.int32)
    out = build_blocks(sys, blocks, separable)
    H = out.reshape(nk, nk, nt, nt).transpose(0, 2, 1, 3).reshape(nk * nt, nk * nt)
    return np.ascontiguousarray(H)


def exciton_energies(H, n=10):
    """Lowest n eigenvalues of the Hermitian H (LAPACK zheevd through numpy)."""
    return np.linalg.eigvalsh(H)[:n]
