"""Python binding of libbse.so, the MI355X Tamm-Dancoff BSE Hamiltonian builder.

Argument marshalling only: every step of the computation runs in the HIP
kernels behind the C ABI declared in include/bse.h.  PyTorch provides device
memory and the current HIP stream.  The library must be built
(``python -m paper_1206_3518_amd.build`` or ``__graft_entry__.build()``); there
is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os
from typing import List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbse.so")
_LIB = None

BSE_OK = 0
BSE_FP64, BSE_SPLIT_FP32, BSE_BF16X3 = 0, 1, 2
BSE_VALIDATE, BSE_PERSISTENT, BSE_TIME_REVERSAL, BSE_FP32_PAIRDENS = 1, 2, 8, 16
BSE_PD_EXCH, BSE_PD_VV, BSE_PD_CC, BSE_PD_DIPOLE = 0, 1, 2, 3
PRECISIONS = {"fp64": BSE_FP64, "split_fp32": BSE_SPLIT_FP32, "bf16x3": BSE_BF16X3}
HARTREE_EV = 27.211386245988


class BseError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"bse status {code}: {msg}")
        self.code = code


class bse_tuning(ctypes.Structure):
    _fields_ = [("persistent", ctypes.c_int), ("ktile", ctypes.c_int), ("wg_per_cu", ctypes.c_int),
                ("pd_ms", ctypes.c_float), ("s1_rows", ctypes.c_int), ("s1_ms", ctypes.c_float),
                ("order", ctypes.c_int)]


class bse_system(ctypes.Structure):
    _fields_ = [("grid", ctypes.c_int * 3), ("kmesh", ctypes.c_int * 3), ("nv", ctypes.c_int),
                ("nc", ctypes.c_int), ("omega_cell", ctypes.c_double), ("ng_max", ctypes.c_int),
                ("ng", ctypes.c_void_p), ("gvec", ctypes.c_void_p), ("vx", ctypes.c_void_p),
                ("u", ctypes.c_void_p), ("eps", ctypes.c_void_p), ("W", ctypes.c_void_p),
                ("H", ctypes.c_void_p), ("qexc", ctypes.c_int), ("nirr", ctypes.c_int),
                ("wsrc", ctypes.c_void_p), ("wmap", ctypes.c_void_p)]


SYMBOLS = ["bse_workspace_size", "bse_pair_density", "bse_build_H", "bse_build_H_backward",
           "bse_autotune", "bse_autotune_last", "bse_transition_dipoles", "bse_transition_dipoles_workspace",
           "bse_spectrum", "bse_screening", "bse_screening_workspace", "bse_haydock_spectrum", "bse_haydock_workspace", "bse_spectrum_noalloc", "bse_build_H_full", "bse_build_H_full_workspace", "bse_profile", "bse_profile_read", "bse_set_chunk_budget", "bse_release_host_state",
           "bse_last_error"]
STAGES = ["vscale", "pd_exch", "pd_vv", "pd_cc", "exchange", "direct1", "direct2", "mirror", "rotate", "tr_fill", "to_f32", "split_w"]


def lib():
    """Loads libbse.so; raises if it has not been built."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        P, I, D, S = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_size_t
        L.bse_workspace_size.argtypes = [P, I, I, I]
        L.bse_workspace_size.restype = S
        L.bse_pair_density.argtypes = [P, I, P, I, P, P, P, S, P]
        L.bse_pair_density.restype = I
        L.bse_build_H.argtypes = [P, I, I, I, P, S, P]
        L.bse_build_H.restype = I
        L.bse_build_H_backward.argtypes = [P, P, P, P, P, P, P, I, I, P, S, P]
        L.bse_build_H_backward.restype = I
        L.bse_autotune.argtypes = [P, I, I, I, ctypes.c_char_p, P, P, S, P]
        L.bse_autotune.restype = I
        L.bse_autotune_last.argtypes = [P, I]
        L.bse_autotune_last.restype = I
        L.bse_transition_dipoles.argtypes = [P, P, P, I, P, P, S, P]
        L.bse_transition_dipoles.restype = I
        L.bse_transition_dipoles_workspace.argtypes = [P]
        L.bse_transition_dipoles_workspace.restype = S
        L.bse_spectrum.argtypes = [I, I, P, P, P, I, I, D, I, D, D, D, P, P, S, P]
        L.bse_spectrum.restype = I
        L.bse_screening.argtypes = [P, P, D, P, P, S, P]
        L.bse_screening.restype = I
        L.bse_screening_workspace.argtypes = [P]
        L.bse_screening_workspace.restype = S
        L.bse_build_H_full.argtypes = [P, P, I, I, P, S, P]
        L.bse_build_H_full.restype = I
        L.bse_build_H_full_workspace.argtypes = [P]
        L.bse_build_H_full_workspace.restype = S
        L.bse_haydock_spectrum.argtypes = [I, P, P, I, I, I, D, I, D, D, D, P, P, P, S, P]
        L.bse_haydock_spectrum.restype = I
        L.bse_haydock_workspace.argtypes = [I, I, I]
        L.bse_haydock_workspace.restype = S
        L.bse_spectrum_noalloc.argtypes = [I, I, P, P, P, I, I, D, I, D, D, D, P, P]
        L.bse_spectrum_noalloc.restype = I
        L.bse_set_chunk_budget.argtypes = [S]
        L.bse_set_chunk_budget.restype = I
        L.bse_release_host_state.argtypes = []
        L.bse_release_host_state.restype = I
        L.bse_profile.argtypes = [I]
        L.bse_profile.restype = I
        L.bse_profile_read.argtypes = [P, P, I, I]
        L.bse_profile_read.restype = I
        L.bse_last_error.argtypes = []
        L.bse_last_error.restype = ctypes.c_char_p
        _LIB = L
    return _LIB


def bse_last_error() -> str:
    return lib().bse_last_error().decode()


def _check(rc):
    if rc != BSE_OK:
        raise BseError(rc, bse_last_error())


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


class DeviceSystem:
    """Device-resident inputs of one crystal (and its output H).  With
    ``irreducible_W`` (a system carrying W_irr, wsrc, wmap), only the W
    matrices of the irreducible q points go to the device and the library
    unfolds W(q) through the maps."""

    def __init__(self, sys, device="cuda", H=None, irreducible_W=False):
        import torch
        self.src = sys
        self.device = torch.device(device)
        self.grid = tuple(sys.grid)
        self.kmesh = tuple(sys.kmesh)
        self.nv, self.nc = int(sys.nv), int(sys.nc)
        self.omega_cell = float(sys.omega_cell)
        self.ng_max = int(sys.ng_max)
        self.ng = np.ascontiguousarray(sys.ng, dtype=np.int32)
        self.gvec = np.ascontiguousarray(sys.gvec, dtype=np.int32)
        self.u = torch.from_numpy(np.ascontiguousarray(sys.u)).to(self.device)
        self.eps = torch.from_numpy(np.ascontiguousarray(sys.eps, dtype=np.float64)).to(self.device)
        self.nirr, self.wsrc, self.wmap = 0, None, None
        if irreducible_W:
            if getattr(sys, "W_irr", None) is None:
                raise ValueError("irreducible_W needs a system with W_irr, wsrc and wmap")
            self.W = torch.from_numpy(np.ascontiguousarray(sys.W_irr)).to(self.device)
            self.nirr = int(sys.W_irr.shape[0])
            self.wsrc = np.ascontiguousarray(sys.wsrc, dtype=np.int32)
            self.wmap = np.ascontiguousarray(sys.wmap, dtype=np.int32)
        else:
            self.W = torch.from_numpy(np.ascontiguousarray(sys.W)).to(self.device)
        self.vx = torch.from_numpy(np.ascontiguousarray(sys.vx, dtype=np.float64)).to(self.device)
        self.nk = int(np.prod(self.kmesh))
        self.ns = self.nk * self.nv * self.nc
        self.qexc = int(getattr(sys, "qexc", 0))  # exciton momentum (q-mesh index); vx is v(Q+G) on S(Q)
        self.H = H if H is not None else torch.empty((self.ns, self.ns), dtype=torch.complex128, device=self.device)

    def struct(self) -> bse_system:
        s = bse_system()
        s.grid[:] = self.grid
        s.kmesh[:] = self.kmesh
        s.nv, s.nc = self.nv, self.nc
        s.omega_cell = self.omega_cell
        s.ng_max = self.ng_max
        s.ng = self.ng.ctypes.data
        s.gvec = self.gvec.ctypes.data
        s.vx = self.vx.data_ptr()
        s.u = self.u.data_ptr()
        s.eps = self.eps.data_ptr()
        s.W = self.W.data_ptr()
        s.H = self.H.data_ptr() if self.H is not None else None
        s.qexc = self.qexc
        s.nirr = self.nirr
        s.wsrc = self.wsrc.ctypes.data if self.wsrc is not None else None
        s.wmap = self.wmap.ctypes.data if self.wmap is not None else None
        return s


def _structs(systems: Sequence[DeviceSystem]):
    arr = (bse_system * len(systems))()
    for i, s in enumerate(systems):
        arr[i] = s.struct()
    return arr


def bse_workspace_size(systems, precision=BSE_FP64, flags=0) -> int:
    systems = systems if isinstance(systems, (list, tuple)) else [systems]
    arr = _structs(systems)
    n = lib().bse_workspace_size(arr, len(systems), int(precision), int(flags))
    if n == 0:
        raise BseError(-1, bse_last_error())
    return int(n)


def workspace(nbytes, device="cuda"):
    import torch
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


def bse_build_H(systems, precision=BSE_FP64, flags=0, ws=None, stream=None):
    """Enqueues the build of H for each system into its .H tensor."""
    systems = systems if isinstance(systems, (list, tuple)) else [systems]
    arr = _structs(systems)
    if ws is None:
        ws = workspace(bse_workspace_size(systems, precision, flags), systems[0].device)
    _check(lib().bse_build_H(arr, len(systems), int(precision), int(flags), _ptr(ws), ws.numel(), _stream(stream)))
    return [s.H for s in systems]


def bse_autotune(systems, precision=BSE_FP64, cache_path=None, ws=None, stream=None, flags=0) -> dict:
    """Times the candidate pair-density dispatches for this batch, then the
    stage-1 contraction tile shapes, and keeps the fastest for later builds of
    the same shape; returns the choice.  flags: BSE_FP32_PAIRDENS tunes the
    FP32 pair-density kernel (mixed precisions)."""
    arr = _structs(systems)
    if ws is None:
        ws = workspace(bse_workspace_size(systems, precision, flags), systems[0].device)
    out = bse_tuning()
    path = None if cache_path is None else os.fsencode(str(cache_path))
    _check(lib().bse_autotune(arr, len(systems), int(precision), int(flags), path, ctypes.byref(out), _ptr(ws),
                              ws.numel(), _stream(stream)))
    return {"persistent": out.persistent, "ktile": out.ktile, "wg_per_cu": out.wg_per_cu, "pd_ms": out.pd_ms,
            "s1_rows": out.s1_rows, "s1_ms": out.s1_ms, "order": out.order}


def bse_autotune_last() -> list:
    """The candidates the last bse_autotune (this thread) timed, with their times."""
    arr = (bse_tuning * 32)()
    n = lib().bse_autotune_last(arr, 32)
    if n < 0:
        raise BseError(n, bse_last_error())
    return [{"persistent": arr[i].persistent, "ktile": arr[i].ktile, "wg_per_cu": arr[i].wg_per_cu,
             "pd_ms": arr[i].pd_ms, "s1_rows": arr[i].s1_rows, "s1_ms": arr[i].s1_ms,
             "order": arr[i].order} for i in range(min(n, 32))]


def bse_pair_density(system: DeviceSystem, kind, kpairs=None, ws=None, stream=None, cell=None):
    """Pair densities of one kind (see include/bse.h) as a complex128 tensor."""
    import torch
    nv, nc, nk, ngm = system.nv, system.nc, system.nk, system.ng_max
    kp = None
    if kind == BSE_PD_EXCH:
        shape = (nk, nv, nc, ngm)
    elif kind in (BSE_PD_VV, BSE_PD_CC):
        kp = np.ascontiguousarray(np.asarray(kpairs, dtype=np.int32).reshape(-1, 2))
        nb = nv if kind == BSE_PD_VV else nc
        shape = (len(kp), nb, nb, ngm)
    elif kind == BSE_PD_DIPOLE:
        shape = (nk, nv, nc, 3)
    else:
        raise ValueError(kind)
    out = torch.empty(shape, dtype=torch.complex128, device=system.device)
    if ws is None:
        n = bse_workspace_size([system])
        if kind == BSE_PD_DIPOLE:
            n = max(n, system.u.numel() * 16)
        ws = workspace(n, system.device)
    cell_arr = None
    if cell is None and kind == BSE_PD_DIPOLE:
        cell = system.src.cell
    if cell is not None:
        cell_arr = np.ascontiguousarray(cell, dtype=np.float64)
    st = system.struct()
    _check(lib().bse_pair_density(ctypes.byref(st), int(kind), kp.ctypes.data if kp is not None else None,
                                  0 if kp is None else len(kp),
                                  cell_arr.ctypes.data if cell_arr is not None else None, _ptr(out),
                                  _ptr(ws), ws.numel(), _stream(stream)))
    return out


def bse_profile(enable: bool):
    _check(lib().bse_profile(1 if enable else 0))


def bse_profile_read(reset=True):
    """{stage: (total ms, launches)} of the bse_build_H launches timed so far."""
    n = len(STAGES)
    ms = (ctypes.c_double * n)()
    cnt = (ctypes.c_longlong * n)()
    _check(lib().bse_profile_read(ms, cnt, n, 1 if reset else 0))
    return {STAGES[i]: (ms[i], cnt[i]) for i in range(n)}


def build_H(sys_or_dev, precision="fp64", flags=0, ws=None):
    """Convenience: H (complex128, on the GPU) of one system."""
    d = sys_or_dev if isinstance(sys_or_dev, DeviceSystem) else DeviceSystem(sys_or_dev)
    p = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    bse_build_H([d], p, flags, ws)
    return d.H


def bse_build_H_backward(system: DeviceSystem, dH, want_dW=True, want_deps=True, precision=BSE_FP64, flags=0,
                         ws=None, stream=None, want_densities=False):
    """(dL/dW, dL/deps) for dL/dH = dH (complex128 [NS][NS], PyTorch convention);
    with want_densities also (dL/dX [Nk][nv][nc][ng_max], dL/drho_vv
    [npairs][nv][nv][ng_max], dL/drho_cc [npairs][nc][nc][ng_max]) for the
    pairs k <= k' in lexicographic order."""
    import torch
    p = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    dH = dH.contiguous()
    dW = torch.empty_like(system.W) if want_dW else None
    deps = torch.empty_like(system.eps) if want_deps else None
    dX = drv = drc = None
    if want_densities:
        nk, nv, nc, ngm = system.nk, system.nv, system.nc, system.ng_max
        npairs = nk * (nk + 1) // 2
        kw = dict(dtype=torch.complex128, device=system.W.device)
        dX = torch.empty((nk, nv, nc, ngm), **kw)
        drv = torch.empty((npairs, nv, nv, ngm), **kw)
        drc = torch.empty((npairs, nc, nc, ngm), **kw)
    if ws is None:
        ws = workspace(bse_workspace_size([system], p, flags), system.device)
    st = system.struct()
    _check(lib().bse_build_H_backward(ctypes.byref(st), _ptr(dH), _ptr(dW), _ptr(deps), _ptr(dX), _ptr(drv),
                                      _ptr(drc), p, int(flags), _ptr(ws), ws.numel(), _stream(stream)))
    if want_densities:
        return dW, deps, dX, drv, drc
    return dW, deps


def _autograd():
    import torch

    class BuildH(torch.autograd.Function):
        """H(W, eps) with the adjoint kernel as its backward.  u, v and the
        cell are constants; dW is projected onto Hermitian, time-reversal
        symmetric W when ``project``."""

        @staticmethod
        def forward(ctx, W, eps, system, precision, project):
            d = DeviceSystem.__new__(DeviceSystem)
            d.__dict__.update(system.__dict__)
            d.W = W.detach().contiguous()
            d.eps = eps.detach().contiguous()
            d.H = torch.empty((d.ns, d.ns), dtype=torch.complex128, device=d.device)
            bse_build_H([d], PRECISIONS.get(precision, precision))
            ctx.system = d
            ctx.precision = precision
            ctx.project = project
            return d.H

        @staticmethod
        def backward(ctx, dH):
            flags = BSE_PROJECT_DW if ctx.project else 0
            dW, deps = bse_build_H_backward(ctx.system, dH, ctx.needs_input_grad[0], ctx.needs_input_grad[1],
                                            ctx.precision, flags)
            return dW, deps, None, None, None

    return BuildH


BSE_PROJECT_DW = 4
_BUILDH = None


def build_H_autograd(system: DeviceSystem, W, eps, precision="fp64", project=True):
    """Differentiable H(W, eps) for one system (see BuildH)."""
    global _BUILDH
    if _BUILDH is None:
        _BUILDH = _autograd()
    return _BUILDH.apply(W, eps, system, precision, project)


def bse_transition_dipoles(system: DeviceSystem, qhats, ws=None, stream=None, cell=None):
    """Transition dipoles d[p][S] (Hartree atomic units, complex128 [nq][NS])
    for the polarisations qhats ([nq][3])."""
    import torch
    q = np.ascontiguousarray(np.asarray(qhats, dtype=np.float64).reshape(-1, 3))
    cell_arr = np.ascontiguousarray(system.src.cell if cell is None else cell, dtype=np.float64)
    st = system.struct()
    if ws is None:
        n = lib().bse_transition_dipoles_workspace(ctypes.byref(st))
        if n == 0:
            raise BseError(-1, bse_last_error())
        ws = workspace(n, system.device)
    d = torch.empty((len(q), system.ns), dtype=torch.complex128, device=system.device)
    _check(lib().bse_transition_dipoles(ctypes.byref(st), cell_arr.ctypes.data, q.ctypes.data, len(q), _ptr(d),
                                        _ptr(ws), ws.numel(), _stream(stream)))
    return d


def bse_spectrum(E, A, d, nk, omega_cell, nw, w0_eV, w1_eV, eta_eV, ws=None, stream=None):
    """eps2 on nw points of [w0, w1] (eV) from exciton energies E (eV, [nlam]),
    eigenvectors A ([ns][nlam] complex) and transition dipoles d ([nq][ns] or
    [ns]), averaged over the nq polarisations."""
    import torch
    E = E.contiguous()
    A = A.contiguous()
    d = d.reshape(-1, A.shape[0]).contiguous()
    ns, nlam = A.shape
    eps2 = torch.empty(nw, dtype=torch.float64, device=A.device)
    if ws is None:
        ws = workspace(8 * nlam, A.device)
    _check(lib().bse_spectrum(ns, nlam, _ptr(E), _ptr(A), _ptr(d), d.shape[0], int(nk), float(omega_cell), int(nw),
                              float(w0_eV), float(w1_eV), float(eta_eV), _ptr(eps2), _ptr(ws), ws.numel(),
                              _stream(stream)))
    return eps2


def bse_set_chunk_budget(nbytes=0):
    """Bytes of per-pair arrays per chunk of k pairs (0: the library default)."""
    _check(lib().bse_set_chunk_budget(int(nbytes)))


def bse_build_H_full_workspace(system: DeviceSystem) -> int:
    st = system.struct()
    n = lib().bse_build_H_full_workspace(ctypes.byref(st))
    if n == 0:
        raise BseError(-1, bse_last_error())
    return int(n)


def bse_build_H_full(system: DeviceSystem, H2=None, flags=0, ws=None, stream=None):
    """The Hamiltonian beyond the Tamm-Dancoff approximation, [[A, B],
    [-B^H, -conj(A)]] (complex128 [2 NS][2 NS] on the GPU), FP64."""
    import torch
    ns = system.ns
    if H2 is None:
        H2 = torch.empty((2 * ns, 2 * ns), dtype=torch.complex128, device=system.device)
    if ws is None:
        ws = workspace(bse_build_H_full_workspace(system), system.device)
    st = system.struct()
    _check(lib().bse_build_H_full(ctypes.byref(st), _ptr(H2), BSE_FP64, int(flags), _ptr(ws), ws.numel(),
                                  _stream(stream)))
    return H2


def bse_screening_workspace(system: DeviceSystem) -> int:
    st = system.struct()
    n = lib().bse_screening_workspace(ctypes.byref(st))
    if n == 0:
        raise BseError(-1, bse_last_error())
    return int(n)


def bse_screening(system: DeviceSystem, vq, head, ws=None, stream=None):
    """Static RPA W [Nk][ng_max][ng_max] (complex128, device) of ``system``'s
    nv occupied and nc empty bands; vq [Nk][ng_max] the bare Coulomb table.
    A system made with ``irreducible_W`` gets W at its irreducible q points
    only, [nirr][ng_max][ng_max]."""
    import torch
    vq = torch.as_tensor(np.ascontiguousarray(vq, dtype=np.float64)).to(system.device) \
        if not isinstance(vq, torch.Tensor) else vq.contiguous()
    st = system.struct()
    if ws is None:
        ws = workspace(bse_screening_workspace(system), system.device)
    nw = system.nirr if system.nirr > 0 else system.nk
    W = torch.empty((nw, system.ng_max, system.ng_max), dtype=torch.complex128, device=system.device)
    _check(lib().bse_screening(ctypes.byref(st), _ptr(vq), float(head), _ptr(W), _ptr(ws), ws.numel(),
                               _stream(stream)))
    return W


def bse_haydock_spectrum(H, d, nk, omega_cell, niter, nw, w0_eV, w1_eV, eta_eV, want_coef=False, ws=None,
                         stream=None):
    """eps2 on nw points of [w0, w1] (eV) from H (complex128 [ns][ns], eV) and
    the dipoles d ([nq][ns] or [ns]) by the Haydock recursion of niter steps;
    with want_coef also the recurrence coefficients [nq][niter][2] (eV)."""
    import torch
    H = H.contiguous()
    ns = H.shape[0]
    d = d.reshape(-1, ns).contiguous()
    nq = d.shape[0]
    eps2 = torch.empty(nw, dtype=torch.float64, device=H.device)
    coef = torch.empty((nq, niter, 2), dtype=torch.float64, device=H.device) if want_coef else None
    if ws is None:
        n = lib().bse_haydock_workspace(ns, nq, int(niter))
        if n == 0:
            raise BseError(-1, "bad Haydock sizes")
        ws = workspace(n, H.device)
    _check(lib().bse_haydock_spectrum(ns, _ptr(H), _ptr(d), nq, int(niter), int(nk), float(omega_cell), int(nw),
                                      float(w0_eV), float(w1_eV), float(eta_eV), _ptr(eps2), _ptr(coef), _ptr(ws),
                                      ws.numel(), _stream(stream)))
    return (eps2, coef) if want_coef else eps2


def absorption_haydock(system: DeviceSystem, H, qhats=((1, 0, 0), (0, 1, 0), (0, 0, 1)), niter=500, nw=1001,
                       w0=0.0, w1=10.0, eta=0.1):
    """eps2(w) averaged over the polarisations qhats without diagonalising H:
    dipoles and the Haydock recursion in the library."""
    d = bse_transition_dipoles(system, qhats)
    return bse_haydock_spectrum(H, d, system.nk, system.omega_cell, niter, nw, w0, w1, eta)


NOALLOC_MAX_NLAM = 1048576


def bse_spectrum_noalloc(E, A, d, nk, omega_cell, nw, w0_eV, w1_eV, eta_eV, eps2=None, stream=None):
    """bse_spectrum without a workspace (the library's static device scratch);
    eps2 may be given so that the call allocates nothing."""
    import torch
    d = d.reshape(-1, A.shape[0])
    ns, nlam = A.shape
    if eps2 is None:
        eps2 = torch.empty(nw, dtype=torch.float64, device=A.device)
    _check(lib().bse_spectrum_noalloc(ns, nlam, _ptr(E), _ptr(A), _ptr(d), d.shape[0], int(nk), float(omega_cell),
                                      int(nw), float(w0_eV), float(w1_eV), float(eta_eV), _ptr(eps2),
                                      _stream(stream)))
    return eps2


def bse_release_host_state():
    _check(lib().bse_release_host_state())


def absorption(system: DeviceSystem, H, qhats=((1, 0, 0), (0, 1, 0), (0, 0, 1)), nw=1001, w0=0.0, w1=10.0, eta=0.1):
    """eps2(w) averaged over the polarisations qhats: FP64 host eigensolve of H
    (numpy LAPACK), then the dipoles and the spectrum in the library."""
    import torch
    E, A = np.linalg.eigh(H.cpu().numpy())
    Ed = torch.from_numpy(E).to(system.device)
    Ad = torch.from_numpy(np.ascontiguousarray(A)).to(system.device)
    d = bse_transition_dipoles(system, qhats)
    return bse_spectrum(Ed, Ad, d, system.nk, system.omega_cell, nw, w0, w1, eta)
