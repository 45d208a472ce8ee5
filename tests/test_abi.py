"""The C-ABI library loads, exports every declared entry point and rejects bad
arguments on the host side (no device work is enqueued).  CPU only."""
import ctypes
import os
import re

import numpy as np
import pytest

import bse_synth as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    import paper_1206_3518_amd as P
    if not os.path.exists(P.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    return P, P.lib()


def test_exports_every_declared_symbol():
    P, L = _lib()
    hdr = open(os.path.join(ROOT, "include", "bse.h")).read()
    declared = set(re.findall(r"^(?:size_t|int|const char \*)\s*(bse_\w+)\s*\(", hdr, re.M))
    assert declared == set(P.SYMBOLS)
    for name in declared:
        assert hasattr(L, name)


def _fake_struct(P, s):
    st = P.bse_system()
    st.grid[:] = s.grid
    st.kmesh[:] = s.kmesh
    st.nv, st.nc = s.nv, s.nc
    st.omega_cell = s.omega_cell
    st.ng_max = s.ng_max
    ng = np.ascontiguousarray(s.ng, dtype=np.int32)
    gv = np.ascontiguousarray(s.gvec, dtype=np.int32)
    st.ng = ng.ctypes.data
    st.gvec = gv.ctypes.data
    # device pointers are never dereferenced on these paths
    for f in ("vx", "u", "eps", "W", "H"):
        setattr(st, f, 0x1000)
    return st, (ng, gv)


def test_workspace_size_and_host_errors():
    P, L = _lib()
    s = B.make_config(0)
    st, keep = _fake_struct(P, s)
    n = L.bse_workspace_size(ctypes.byref(st), 1, 0, 0)
    nt = s.nv * s.nc
    npairs = s.nk * (s.nk + 1) // 2
    # X + RV + RC + Z rows of ng_max complex
    assert n >= 16 * s.ng_max * (s.ns + 3 * npairs * nt)
    # workspace too small: refused before any enqueue
    rc = L.bse_build_H(ctypes.byref(st), 1, 0, 0, ctypes.c_void_p(0x1000), 4096, None)
    assert rc == -3 and "workspace" in P.bse_last_error()
    # null workspace
    rc = L.bse_build_H(ctypes.byref(st), 1, 0, 0, None, n, None)
    assert rc == -1
    # bad precision
    rc = L.bse_build_H(ctypes.byref(st), 1, 7, 0, ctypes.c_void_p(0x1000), n, None)
    assert rc == -1
    # unsupported grid
    st2, keep2 = _fake_struct(P, s)
    st2.grid[0] = st2.grid[1] = st2.grid[2] = 20  # no plane kernel, directly or with rotated axes
    assert L.bse_build_H(ctypes.byref(st2), 1, 0, 0, ctypes.c_void_p(0x1000), n, None) == -2
    # null input pointer
    st3, keep3 = _fake_struct(P, s)
    st3.u = None
    assert L.bse_build_H(ctypes.byref(st3), 1, 0, 0, ctypes.c_void_p(0x1000), n, None) == -1
    # sphere exceeding the grid window
    st4, keep4 = _fake_struct(P, s)
    gv = keep4[1].copy()
    gv[1, 1] = (15, 0, 0)
    keep4 = (keep4[0], gv)
    st4.gvec = gv.ctypes.data
    assert L.bse_build_H(ctypes.byref(st4), 1, 0, 0, ctypes.c_void_p(0x1000), n, None) == -2
    # time reversal asked for on a sphere that is not closed under G -> -G:
    # the last point of S(0) replaced by G = 0 leaves its partner without an image
    st5, keep5 = _fake_struct(P, s)
    gv = keep5[1].copy()
    gv[0, s.ng[0] - 1] = (0, 0, 0)
    keep5 = (keep5[0], gv)
    st5.gvec = gv.ctypes.data
    assert L.bse_build_H(ctypes.byref(st5), 1, 0, P.BSE_TIME_REVERSAL, ctypes.c_void_p(0x1000), n, None) == -2
    assert "time reversal" in P.bse_last_error()
    # FP32 pair densities only with a mixed precision, in the build, the
    # autotuner and the backward; the backward takes no build-only flag
    assert L.bse_build_H(ctypes.byref(st), 1, P.BSE_FP64, P.BSE_FP32_PAIRDENS, ctypes.c_void_p(0x1000), n,
                         None) == -1
    assert "mixed" in P.bse_last_error()
    assert L.bse_autotune(ctypes.byref(st), 1, P.BSE_FP64, P.BSE_FP32_PAIRDENS, None, None, ctypes.c_void_p(0x1000),
                          n, None) == -1
    assert L.bse_build_H_backward(ctypes.byref(st), ctypes.c_void_p(0x1000), None, None, None, None, None,
                                  P.BSE_FP64, P.BSE_FP32_PAIRDENS, ctypes.c_void_p(0x1000), n, None) == -1
    assert L.bse_build_H_backward(ctypes.byref(st), ctypes.c_void_p(0x1000), None, None, None, None, None,
                                  P.BSE_FP64, P.BSE_VALIDATE, ctypes.c_void_p(0x1000), n, None) == -1
    # exciton momentum: out of range; with time reversal; in the backward
    st6, keep6 = _fake_struct(P, s)
    st6.qexc = s.nk
    assert L.bse_build_H(ctypes.byref(st6), 1, 0, 0, ctypes.c_void_p(0x1000), n, None) == -1
    assert "qexc" in P.bse_last_error()
    st6.qexc = 1
    assert L.bse_build_H(ctypes.byref(st6), 1, 0, P.BSE_TIME_REVERSAL, ctypes.c_void_p(0x1000), n, None) == -1
    assert "TIME_REVERSAL" in P.bse_last_error()
    # the backward at finite Q gives dW and deps, not the density gradients
    assert L.bse_build_H_backward(ctypes.byref(st6), ctypes.c_void_p(0x1000), ctypes.c_void_p(0x1000), None,
                                  ctypes.c_void_p(0x1000), None, None, P.BSE_FP64, 0, ctypes.c_void_p(0x1000), n,
                                  None) == -7
    assert "momentum" in P.bse_last_error()
    assert L.bse_build_H_backward(ctypes.byref(st6), ctypes.c_void_p(0x1000), ctypes.c_void_p(0x1000), None, None,
                                  None, None, P.BSE_FP64, P.BSE_TIME_REVERSAL, ctypes.c_void_p(0x1000), n, None) == -1
    assert "TIME_REVERSAL" in P.bse_last_error()
    # W of the irreducible q points: maps missing, out of range, not bijective,
    # moving G = 0 of q = 0
    s7 = B.make_system(B.cell_fcc(7.0), (16, 16, 16), (2, 2, 2), 2, 2, 3.0, seed=71)
    reps, wsrc, wmap = B.point_group_maps(s7)
    n7 = None
    for mutate, code, word in [
            (lambda ws, wm: None, 0, None),
            (lambda ws, wm: ws.__setitem__((1, 0), len(reps)), -1, "wsrc"),
            (lambda ws, wm: ws.__setitem__((1, 1), 2), -1, "wsrc"),
            (lambda ws, wm: wm.__setitem__((2, 0), s7.ng[2]), -1, "wmap"),
            (lambda ws, wm: wm.__setitem__((2, 1), wm[2, 2]), -2, "permutation"),
            (lambda ws, wm: wm.__setitem__((0, slice(0, 2)), wm[0, 1::-1].copy()), -2, "wmap[0][0]")]:
        ws_, wm_ = wsrc.copy(), wmap.copy()
        mutate(ws_, wm_)
        st7, keep7 = _fake_struct(P, s7)
        st7.nirr, st7.wsrc, st7.wmap = len(reps), ws_.ctypes.data, wm_.ctypes.data
        if code == 0:
            n7 = L.bse_workspace_size(ctypes.byref(st7), 1, 0, 0)
            assert n7 > 0
            # the backward unfolds W into its workspace: a small one is refused on the host
            assert L.bse_build_H_backward(ctypes.byref(st7), ctypes.c_void_p(0x1000), ctypes.c_void_p(0x1000), None,
                                          None, None, None, P.BSE_FP64, 0, ctypes.c_void_p(0x1000), 4096, None) == -3
            assert "workspace" in P.bse_last_error()
            n7b = L.bse_workspace_size(ctypes.byref(st7), 1, 0, 0)
            assert n7b >= 2 * 16 * s7.nk * s7.ng_max ** 2  # the unfolded W and dW at every q
            st7.nirr = s7.nk + 1
            assert L.bse_build_H(ctypes.byref(st7), 1, 0, 0, ctypes.c_void_p(0x1000), n7, None) == -1
            assert "nirr" in P.bse_last_error()
            st7.nirr, st7.wmap = len(reps), None
            assert L.bse_build_H(ctypes.byref(st7), 1, 0, 0, ctypes.c_void_p(0x1000), n7, None) == -1
            # the screening needs, per matrix, a q that maps to it by the identity
            st7.wmap = wm_.ctypes.data
            assert L.bse_screening_workspace(ctypes.byref(st7)) > 0
            ws_[:, 1] = 1
            assert L.bse_screening_workspace(ctypes.byref(st7)) == 0
            assert "identity" in P.bse_last_error()
            continue
        assert L.bse_build_H(ctypes.byref(st7), 1, 0, 0, ctypes.c_void_p(0x1000), 1 << 40, None) == code
        assert word in P.bse_last_error()
    # the workspace grows for the FP32 copy of u
    n32 = L.bse_workspace_size(ctypes.byref(st), 1, P.BSE_BF16X3, P.BSE_FP32_PAIRDENS)
    assert n32 >= n + 8 * s.nk * (s.nv + s.nc) * int(np.prod(s.grid))
    # pair densities: bad kind and out-of-range k pair
    out = ctypes.c_void_p(0x1000)
    assert L.bse_pair_density(ctypes.byref(st), 9, None, 0, None, out, ctypes.c_void_p(0x1000), n, None) == -1
    kp = np.array([[0, s.nk]], dtype=np.int32)
    assert L.bse_pair_density(ctypes.byref(st), 1, kp.ctypes.data, 1, None, out, ctypes.c_void_p(0x1000), n,
                              None) == -1


def test_chunk_budget_bounds_the_workspace():
    """The per-pair arrays hold one chunk of k pairs: a smaller budget gives a
    smaller workspace; the default comes back with 0."""
    P, L = _lib()
    s = B.make_config(0)
    st, keep = _fake_struct(P, s)
    n_default = L.bse_workspace_size(ctypes.byref(st), 1, 0, 0)
    assert L.bse_set_chunk_budget(64 << 10) == 0
    try:
        n_small = L.bse_workspace_size(ctypes.byref(st), 1, 0, 0)
    finally:
        assert L.bse_set_chunk_budget(0) == 0
    per_pair = 16 * s.ng_max * (2 * s.nv ** 2 + s.nc ** 2)
    npairs = s.nk * (s.nk + 1) // 2
    assert n_small < n_default
    assert n_default - n_small >= per_pair * (npairs // 2)
    assert L.bse_workspace_size(ctypes.byref(st), 1, 0, 0) == n_default
