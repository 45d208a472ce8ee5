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


def k_plus_q(kmesh, k: int, q: int) -> int:
    """Mesh index of k + q: each integer component added modulo the mesh."""
    n1, n2, n3 = (int(x) for x in kmesh)
    a = ((k // (n2 * n3)) + (q // (n2 * n3))) % n1
    b = ((k // n3) % n2 + (q // n3) % n2) % n2
    c = (k % n3 + q % n3) % n3
    return (a * n2 + b) * n3 + c


def build_blocks_exciton(sys, blocks, separable=True):
    """Blocks (k, k') of the Hamiltonian at exciton momentum Q = q-mesh point
    ``sys.qexc`` (the e-h basis S = (n k, m k+q) of the BSE eigenproblem of
    Sec. II.C, written out in the Tamm-Dancoff block: hole v at k, electron c
    at k + Q), each [nv*nc][nv*nc] in eV:

      H_SS' = (e_{c,k+Q} - e_{v,k}) delta_SS' + c (2 Vbar_SS' - D_SS')
      Vbar_SS' = sum_{G in S(Q), G != 0} conj(n_{vk,c k+Q}(G)) v(Q+G) n_{v'k',c'k'+Q}(G)
      D_SS'    = sum_{G,G' in S(q)} conj(n_{vk,v'k'}(G)) W_GG'(q) n_{c k+Q,c'k'+Q}(G'),

    k' - k = q + G0 (Eqs. V_eh and W_SS; sys.vx holds v(Q+G) on the sphere of
    Q).  Each block comes from the direct sums of the pair density, each pair
    with the fold of its own two k points (so the conduction densities of
    (k+Q, k'+Q) carry their own G0)."""
    blocks = [(int(a), int(b)) for a, b in np.asarray(blocks).reshape(-1, 2)]
    nk, nv, nc = sys.nk, sys.nv, sys.nc
    nt = nv * nc
    Q = int(getattr(sys, "qexc", 0))
    kq = [k_plus_q(sys.kmesh, k, Q) for k in range(nk)]
    c = HARTREE_EV / (nk * sys.omega_cell)
    ngq = int(sys.ng[Q])
    v = np.array(sys.vx[:ngq], dtype=np.float64)
    v[np.all(sys.gvec[Q, :ngq] == 0, axis=1)] = 0.0  # G = 0 left out (Vbar)
    ks = sorted({k for b in blocks for k in b})
    # exchange rows n_{vk, c k+Q} on the sphere of Q
    items = [(k, a, kq[k], nv + b) for k in ks for a in range(nv) for b in range(nc)]
    for k in ks:
        assert fold(sys.kmesh, k, kq[k])[0] == Q
    Xr = pair_density_items(sys, items, separable)[:, :ngq].reshape(len(ks), nt, ngq)
    X = {k: Xr[i] for i, k in enumerate(ks)}
    out = np.zeros((len(blocks), nt, nt), dtype=np.complex128)
    for bi, (ka, kb) in enumerate(blocks):
        iq, _ = fold(sys.kmesh, ka, kb)
        assert fold(sys.kmesh, kq[ka], kq[kb])[0] == iq
        ng = int(sys.ng[iq])
        it = [(ka, a, kb, b) for a in range(nv) for b in range(nv)]
        it += [(kq[ka], nv + a, kq[kb], nv + b) for a in range(nc) for b in range(nc)]
        n = pair_density_items(sys, it, separable)[:, :ng]
        rv = n[: nv * nv].reshape(nv, nv, ng)
        rc = n[nv * nv:].reshape(nc, nc, ng)
        D = np.einsum("abg,gh,cdh->acbd", np.conj(rv), sys.W[iq, :ng, :ng], rc).reshape(nt, nt)
        V = (np.conj(X[ka]) * v) @ X[kb].T
        blk = c * (2.0 * V - D)
        if ka == kb:
            de = (sys.eps[kq[ka], nv:][None, :] - sys.eps[ka, :nv][:, None]).reshape(-1)
            blk[np.diag_indices(nt)] += de
        out[bi] = blk
    return out


def build_H_exciton(sys, separable=True):
    """The whole Hamiltonian at exciton momentum ``sys.qexc``: every one of
    the Nk^2 blocks of ``build_blocks_exciton``.  Q = 0 is ``build_H``."""
    nk, nt = sys.nk, sys.nv * sys.nc
    blocks = [(a, b) for a in range(nk) for b in range(nk)]
    out = build_blocks_exciton(sys, blocks, separable)
    H = out.reshape(nk, nk, nt, nt).transpose(0, 2, 1, 3).reshape(nk * nt, nk * nt)
    return np.ascontiguousarray(H)


def build_H_full(sys, separable=True):
    """The Bethe-Salpeter Hamiltonian beyond the Tamm-Dancoff approximation
    (optical limit, Q = 0), from the general definition of Sec. II.C and the
    appendix over the basis of e-h states (n = v, m = c) and h-e states
    (n = c, m = v), S = (n k, m k):

      H_ab = (e_{m_a} - e_{n_a}) delta_ab - (f_{m_a} - f_{n_a}) K_ab,   f_v = 1, f_c = 0,
      K_ab = c (2 Vbar_ab - D_ab),
      Vbar_ab = sum_{G != 0} conj(n_{n_a k_a, m_a k_a}(G)) v(G) n_{n_b k_b, m_b k_b}(G),
      D_ab    = sum_{G,G'} conj(n_{n_a k_a, n_b k_b}(G)) W_GG'(q) n_{m_a k_a, m_b k_b}(G'),

    k_b - k_a = q + G0 (Eqs. V_eh and W_SS).  States are ordered e-h first,
    then h-e, each as S = (k nv + v) nc + c; the result is [2 NS][2 NS] in eV.
    Every block is computed from its own pair densities: no symmetry of the
    blocks is assumed (the e-h block is the Tamm-Dancoff H)."""
    nk, nv, nc, nb = sys.nk, sys.nv, sys.nc, sys.nb
    ns = sys.ns
    c = HARTREE_EV / (nk * sys.omega_cell)
    # states: (kind, k, v, c) -> (n band, m band, factor -(f_m - f_n), energy)
    st = []
    for kind in (0, 1):
        for k in range(nk):
            for v in range(nv):
                for cc in range(nc):
                    n, m = (v, nv + cc) if kind == 0 else (nv + cc, v)
                    fac = 1.0 if kind == 0 else -1.0  # -(f_m - f_n)
                    st.append((k, n, m, fac, sys.eps[k, m] - sys.eps[k, n]))
    ng0 = int(sys.ng[0])
    v0 = np.array(sys.vx[:ng0], dtype=np.float64)
    v0[np.all(sys.gvec[0, :ng0] == 0, axis=1)] = 0.0
    items = [(k, n, k, m) for (k, n, m, _, _) in st]
    X = pair_density_items(sys, items, separable)[:, :ng0]
    K = 2.0 * c * (np.conj(X) * v0) @ X.T
    # direct term: every band pair of every ordered (k, k')
    D = np.zeros_like(K)
    idx = {}
    for a, (k, n, m, _, _) in enumerate(st):
        idx.setdefault(k, []).append((a, n, m))
    for ka in range(nk):
        for kb in range(nk):
            iq, _ = fold(sys.kmesh, ka, kb)
            ng = int(sys.ng[iq])
            it = [(ka, i, kb, j) for i in range(nb) for j in range(nb)]
            rho = pair_density_items(sys, it, separable)[:, :ng].reshape(nb, nb, ng)
            Z = np.einsum("ijg,gh->ijh", np.conj(rho), sys.W[iq, :ng, :ng])
            for a, na, ma in idx[ka]:
                for b, nb_, mb in idx[kb]:
                    D[a, b] = np.dot(Z[na, nb_], rho[ma, mb])
    K -= c * D
    fac = np.array([x[3] for x in st])
    H = fac[:, None] * K
    H[np.diag_indices(2 * ns)] += np.array([x[4] for x in st])
    return H


def coupling_blocks(sys, blocks, separable=True):
    """Blocks (k, k') of the coupling block B of ``build_H_full`` (e-h row
    (v k, c k), h-e column (c' k', v' k')), each [nv*nc][nv*nc] in eV, rows
    (v, c) and columns (v', c'):

      B = c (2 Vbar - D),
      Vbar = sum_{G != 0} conj(n_{vk,ck}(G)) v(G) n_{c'k',v'k'}(G),
      D    = sum_{G,G'} conj(n_{vk,c'k'}(G)) W_GG'(q) n_{ck,v'k'}(G'),  k' - k = q + G0,

    from the direct sums of the pair density (Eqs. V_eh and W_SS)."""
    blocks = [(int(a), int(b)) for a, b in np.asarray(blocks).reshape(-1, 2)]
    nk, nv, nc = sys.nk, sys.nv, sys.nc
    nt = nv * nc
    c = HARTREE_EV / (nk * sys.omega_cell)
    ng0 = int(sys.ng[0])
    v0 = np.array(sys.vx[:ng0], dtype=np.float64)
    v0[np.all(sys.gvec[0, :ng0] == 0, axis=1)] = 0.0
    ks = sorted({k for b in blocks for k in b})
    eh = [(k, a, k, nv + b) for k in ks for a in range(nv) for b in range(nc)]   # n_{vk, ck}
    he = [(k, nv + b, k, a) for k in ks for a in range(nv) for b in range(nc)]   # n_{ck, vk}, rows (v, c)
    Xe = pair_density_items(sys, eh, separable)[:, :ng0].reshape(len(ks), nt, ng0)
    Xh = pair_density_items(sys, he, separable)[:, :ng0].reshape(len(ks), nt, ng0)
    at = {k: i for i, k in enumerate(ks)}
    out = np.zeros((len(blocks), nt, nt), dtype=np.complex128)
    for bi, (ka, kb) in enumerate(blocks):
        iq, _ = fold(sys.kmesh, ka, kb)
        ng = int(sys.ng[iq])
        it = [(ka, a, kb, nv + b) for a in range(nv) for b in range(nc)]      # n_{vk, c'k'}
        it += [(ka, nv + b, kb, a) for b in range(nc) for a in range(nv)]     # n_{ck, v'k'}
        n = pair_density_items(sys, it, separable)[:, :ng]
        rvc = n[:nt].reshape(nv, nc, ng)
        rcv = n[nt:].reshape(nc, nv, ng)
        D = np.einsum("axg,gh,cbh->acbx", np.conj(rvc), sys.W[iq, :ng, :ng], rcv).reshape(nt, nt)
        V = (np.conj(Xe[at[ka]]) * v0) @ Xh[at[kb]].T
        out[bi] = c * (2.0 * V - D)
    return out


def exciton_energies(H, n=10):
    """Lowest n eigenvalues of the Hermitian H (LAPACK zheevd through numpy)."""
    return np.linalg.eigvalsh(H)[:n]


def adjoint(sys, Gbar, qs=None, separable=True):
    """Adjoint of the block-by-block map (W, eps) -> H of ``build_H`` (at
    exciton momentum Q = ``sys.qexc``: of ``build_H_exciton``).

    Gbar = dL/dRe H + i dL/dIm H (the PyTorch convention for a real L of a
    complex H).  With dL = Re sum conj(Gbar) dH and S = (k v c):
      dL/dW_{GG'}(q) = -c sum_{(k,k') folding to q} sum_{vv'cc'} Gbar_SS' n_{vk,v'k'}(G) conj(n_{c k+Q,c' k'+Q}(G'))
      dL/de_{c,k+Q} = sum_v Re Gbar_SS,   dL/de_vk = -sum_c Re Gbar_SS
    (direct term and transition energies of Sec. II.C).  ``qs`` restricts dW
    to those q.  Returns (dW [Nk][ng_max][ng_max], deps [Nk][nb]).
    """
    nk, nv, nc, nb = sys.nk, sys.nv, sys.nc, sys.nb
    nt = nv * nc
    c = HARTREE_EV / (nk * sys.omega_cell)
    Q = int(getattr(sys, "qexc", 0))
    kq = [k_plus_q(sys.kmesh, k, Q) for k in range(nk)]
    dW = np.zeros((nk, sys.ng_max, sys.ng_max), dtype=np.complex128)
    pairs = []
    for ka in range(nk):
        for kb in range(nk):
            iq, _ = fold(sys.kmesh, ka, kb)
            if qs is None or iq in qs:
                pairs.append((ka, kb, iq))
    items = []
    for ka, kb, _ in pairs:
        items += [(ka, v, kb, v2) for v in range(nv) for v2 in range(nv)]
        items += [(kq[ka], nv + c1, kq[kb], nv + c2) for c1 in range(nc) for c2 in range(nc)]
    rho = pair_density_items(sys, items, separable) if items else None
    per = nv * nv + nc * nc
    for i, (ka, kb, iq) in enumerate(pairs):
        ng = sys.ng[iq]
        blk = rho[i * per:(i + 1) * per, :ng]
        rv = blk[: nv * nv].reshape(nv, nv, ng)
        rc = blk[nv * nv:].reshape(nc, nc, ng)
        gb = Gbar[ka * nt:(ka + 1) * nt, kb * nt:(kb + 1) * nt].reshape(nv, nc, nv, nc)
        dW[iq, :ng, :ng] += -c * np.einsum("acbd,abg,cdh->gh", gb, rv, np.conj(rc))
    deps = np.zeros((nk, nb))
    dg = np.real(np.diag(Gbar)).reshape(nk, nv, nc)
    deps[kq, nv:] = dg.sum(axis=1)
    deps[:, :nv] = -dg.sum(axis=2)
    return dW, deps


def upper_pairs(nk):
    """Ordered k pairs k <= k' in lexicographic order: the independent pair
    densities when the lower k blocks of H are the mirror of the upper ones."""
    return [(a, b) for a in range(nk) for b in range(a, nk)]


def densities(sys, separable=True, pairs=None):
    """The pair densities that H is made of (Sec. II.B): X [Nk][nv][nc][ng_max]
    = n_{vk,ck} on S(0), and for every upper pair (k, k') (lexicographic)
    rv [np][nv][nv][ng_max] = n_{vk,v'k'}, rc [np][nc][nc][ng_max] =
    n_{ck,c'k'} on S(q(k, k')); ``pairs`` (indices into ``upper_pairs``)
    restricts rv and rc to those pairs."""
    nk, nv, nc = sys.nk, sys.nv, sys.nc
    xi = [(k, v, k, nv + c) for k in range(nk) for v in range(nv) for c in range(nc)]
    X = pair_density_items(sys, xi, separable).reshape(nk, nv, nc, sys.ng_max)
    up = upper_pairs(nk)
    items = []
    for ka, kb in (up if pairs is None else [up[p] for p in pairs]):
        items += [(ka, v, kb, v2) for v in range(nv) for v2 in range(nv)]
        items += [(ka, nv + c1, kb, nv + c2) for c1 in range(nc) for c2 in range(nc)]
    rho = pair_density_items(sys, items, separable)
    per = nv * nv + nc * nc
    rho = rho.reshape(-1, per, sys.ng_max)
    rv = rho[:, : nv * nv].reshape(-1, nv, nv, sys.ng_max)
    rc = rho[:, nv * nv:].reshape(-1, nc, nc, sys.ng_max)
    return X, rv, rc


def H_from_densities(sys, X, rv, rc):
    """H of Sec. II.C assembled from given pair densities: the exchange over
    every (k, k') block, the direct term over the upper pairs k <= k', and the
    lower blocks of the direct term as the conjugate transpose of the upper
    ones.  With the densities of ``densities`` and a Hermitian,
    time-reversal symmetric W this is ``build_H``."""
    nk, nv, nc = sys.nk, sys.nv, sys.nc
    nt = nv * nc
    c = HARTREE_EV / (nk * sys.omega_cell)
    ng0 = sys.ng[0]
    v = np.array(sys.vx[:ng0], dtype=np.float64)
    v[0] = 0.0  # G = 0 left out of the exchange
    N = X[..., :ng0].reshape(sys.ns, ng0)
    H = 2.0 * c * (np.conj(N) * v) @ N.T
    D = np.zeros_like(H)
    for p, (ka, kb) in enumerate(upper_pairs(nk)):
        iq, _ = fold(sys.kmesh, ka, kb)
        ng = sys.ng[iq]
        Wq = sys.W[iq, :ng, :ng]
        blk = np.einsum("abg,gh,cdh->acbd", np.conj(rv[p, :, :, :ng]), Wq, rc[p, :, :, :ng]).reshape(nt, nt)
        D[ka * nt:(ka + 1) * nt, kb * nt:(kb + 1) * nt] = blk
        if ka != kb:
            D[kb * nt:(kb + 1) * nt, ka * nt:(ka + 1) * nt] = np.conj(blk).T
    H -= c * D
    de = (sys.eps[:, nv:][:, None, :] - sys.eps[:, :nv][:, :, None]).reshape(-1)
    H[np.diag_indices(sys.ns)] += de
    return H


def adjoint_densities(sys, Gbar, X=None, rv=None, rc=None, pairs=None):
    """Gradient of L (dL = Re sum conj(Gbar) dH) with respect to the pair
    densities that ``H_from_densities`` takes, in the PyTorch convention
    dL/dz = dL/dRe z + i dL/dIm z:
      dX_S(m)      = 2c v(m) sum_S' (conj(Gbar_SS') + Gbar_S'S) X_S'(m)      (m != 0)
      drv_vv'(g)   = -c sum_cc' conj(Geff_SS') (W rc_cc')(g)
      drc_cc'(g')  = -c sum_vv' Geff_SS' (W^H rv_vv')(g')
    with Geff = Gbar + Gbar^H on the blocks k < k' (their mirror images
    depend on the same densities) and Geff = Gbar on k = k'.
    ``pairs`` (indices into ``upper_pairs``) says which pairs rv and rc hold.
    Returns (dX, drv, drc) shaped like (X, rv, rc)."""
    if X is None:
        X, rv, rc = densities(sys, pairs=pairs)
    nk, nv, nc = sys.nk, sys.nv, sys.nc
    nt = nv * nc
    c = HARTREE_EV / (nk * sys.omega_cell)
    ng0 = sys.ng[0]
    v = np.array(sys.vx[:ng0], dtype=np.float64)
    v[0] = 0.0
    N = X[..., :ng0].reshape(sys.ns, ng0)
    G2 = np.conj(Gbar) + Gbar.T
    dX = np.zeros_like(X)
    dX[..., :ng0] = (2.0 * c * v * (G2 @ N)).reshape(nk, nv, nc, ng0)
    drv = np.zeros_like(rv)
    drc = np.zeros_like(rc)
    up = upper_pairs(nk)
    for p, (ka, kb) in enumerate(up if pairs is None else [up[i] for i in pairs]):
        iq, _ = fold(sys.kmesh, ka, kb)
        ng = sys.ng[iq]
        Wq = sys.W[iq, :ng, :ng]
        gb = Gbar[ka * nt:(ka + 1) * nt, kb * nt:(kb + 1) * nt]
        if ka != kb:
            gb = gb + np.conj(Gbar[kb * nt:(kb + 1) * nt, ka * nt:(ka + 1) * nt]).T
        geff = gb.reshape(nv, nc, nv, nc)
        wrc = np.einsum("gh,cdh->cdg", Wq, rc[p, :, :, :ng])
        whrv = np.einsum("gh,abg->abh", np.conj(Wq), rv[p, :, :, :ng])
        drv[p, :, :, :ng] = -c * np.einsum("acbd,cdg->abg", np.conj(geff), wrc)
        drc[p, :, :, :ng] = -c * np.einsum("acbd,abh->cdh", geff, whrv)
    return dX, drv, drc


def tr_orbit(sys, iq, g, gp):
    """The entries of W tied to W_{g g'}(q) by Hermiticity and time reversal
    (Sec. III.A with T = 1), as (q, g, g', conjugated) tuples."""
    n = np.array(sys.kmesh)
    n1, n2, n3 = sys.kmesh
    iv = np.array([iq // (n2 * n3), (iq // n3) % n2, iq % n3])
    qb = (-iv) % n
    t = (-iv - qb) // n
    iqb = int((qb[0] * n2 + qb[1]) * n3 + qb[2])
    lut = {tuple(m): i for i, m in enumerate(sys.gvec[iqb, : sys.ng[iqb]])}
    m, mp = sys.gvec[iq, g], sys.gvec[iq, gp]
    gb, gpb = lut[tuple(t - m)], lut[tuple(t - mp)]
    return {(iq, g, gp, False), (iq, gp, g, True), (iqb, gb, gpb, True), (iqb, gpb, gb, False)}


def orbit_direction(sys, iq, g, gp, h):
    """A perturbation of W that keeps it Hermitian and time-reversal
    symmetric: h at (q, g, g') and the tied entries accordingly."""
    D = np.zeros_like(sys.W)
    for q, a, b, cj in tr_orbit(sys, iq, g, gp):
        D[q, a, b] += np.conj(h) if cj else h
    return D


def signed_freq(N):
    """Signed DFT frequencies of an N-point axis with the Nyquist term set to 0."""
    f = np.fft.fftfreq(N, 1.0 / N)
    if N % 2 == 0:
        f[N // 2] = 0.0
    return f


def grad_matrix(sys):
    """<u_vk| grad |u_ck> (Cartesian, bohr^-1) for every k, v, c: the k.p
    matrix element of Sec. II.B with the derivative taken spectrally,
      <u|grad|u'> = (i / N_r) sum_m G_m conj(U(m)) U'(m),  U = unnormalised DFT of u,
    G_m = sum_d m_d b_d with signed frequencies and the Nyquist planes removed.
    Returns [Nk][nv][nc][3] complex."""
    N1, N2, N3 = sys.grid
    b = 2.0 * math.pi * np.linalg.inv(sys.cell).T
    f = [signed_freq(N) for N in (N1, N2, N3)]
    out = np.zeros((sys.nk, sys.nv, sys.nc, 3), dtype=np.complex128)
    for k in range(sys.nk):
        U = np.fft.fftn(sys.u[k].reshape(sys.nb, N1, N2, N3), axes=(1, 2, 3))
        for d in range(3):
            sh = [1, 1, 1]
            sh[d] = -1
            w = f[d].reshape(sh)
            # S_d[v][c] = sum_m m_d conj(U_v) U_c
            Sd = np.einsum("vxyz,cxyz->vc", np.conj(U[: sys.nv]), U[sys.nv:] * w)
            out[k, :, :, :] += (1j / sys.nr) * Sd[:, :, None] * b[d][None, None, :]
    return out


def transition_dipoles(sys, qhat):
    """d_S = qhat . <u_vk|grad|u_ck> / (e_ck - e_vk) in Hartree atomic units
    (the q -> 0 limit of the pair density, Sec. II.B, up to the phase -i)."""
    D = grad_matrix(sys) @ np.asarray(qhat, dtype=np.float64)
    de = (sys.eps[:, None, sys.nv:] - sys.eps[:, : sys.nv, None]) / HARTREE_EV
    return (D / de).reshape(-1)


def spectrum(E, A, d, pref, w):
    """eps2(w) = pref sum_l |t_l|^2 eta / ((w - E_l)^2 + eta^2) with t_l = sum_S A[S][l] d_S:
    the imaginary part of the macroscopic dielectric function from the spectral
    representation of Sec. II.C with the Tamm-Dancoff overlap matrix = identity.
    E, w in Hartree; w = (grid, eta)."""
    grid, eta = w
    t = A.T @ d
    wt = np.abs(t) ** 2
    return pref * np.sum(wt[None, :] * eta / ((grid[:, None] - E[None, :]) ** 2 + eta ** 2), axis=1)


def lanczos(H, v, m):
    """The Lanczos three-term recurrence (Lanczos 1950) on the Hermitian H from
    the start vector v, as the Haydock recursion method uses it for the
    resolvent of Eq. resolvent (appendix; Tamm-Dancoff, overlap = identity):
      q_0 = v / |v|,  w = H q_j - b_{j-1} q_{j-1},  a_j = Re q_j^H w,
      w -= a_j q_j,  b_j = |w|,  q_{j+1} = w / b_j,
    for j = 0 .. m-1, without reorthogonalisation.  Returns (a, b), length m."""
    H = np.asarray(H)
    q = np.asarray(v, dtype=np.complex128) / np.linalg.norm(v)
    qp = np.zeros_like(q)
    bp = 0.0
    a = np.zeros(m)
    b = np.zeros(m)
    for j in range(m):
        w = H @ q - bp * qp
        a[j] = np.real(np.vdot(q, w))
        w = w - a[j] * q
        b[j] = np.linalg.norm(w)
        qp, q, bp = q, (w / b[j] if b[j] > 0.0 else np.zeros_like(w)), b[j]
    return a, b


def continued_fraction(a, b, z):
    """g(z) = 1 / (z - a_0 - b_0^2 / (z - a_1 - b_1^2 / (... / (z - a_{m-1})))):
    the (0, 0) element of (z - T)^-1 for the tridiagonal T of the recurrence,
    i.e. q_0^H (z - H)^-1 q_0 to the order the recurrence reaches."""
    z = np.asarray(z, dtype=np.complex128)
    t = 1.0 / (z - a[-1])
    for j in range(len(a) - 2, -1, -1):
        t = 1.0 / (z - a[j] - b[j] ** 2 * t)
    return t


def haydock_spectrum(H, d, pref, w, m):
    """eps2(w) of ``spectrum`` from the resolvent instead of the eigenpairs:
    sum_l |t_l|^2 eta / ((w - E_l)^2 + eta^2) = -Im v^H (w + i eta - H)^-1 v
    with v = conj(d) (t_l = sum_S A[S][l] d_S), evaluated by ``lanczos`` from
    v and ``continued_fraction``.  H, w and eta in Hartree; w = (grid, eta)."""
    grid, eta = w
    v = np.conj(np.asarray(d, dtype=np.complex128))
    a, b = lanczos(H, v, m)
    g = continued_fraction(a, b, grid + 1j * eta)
    return pref * np.vdot(v, v).real * (-np.imag(g))


def screened_interaction(sys, vq, head):
    """Static RPA screened interaction W(q) on the spheres of ``sys`` from its
    nv occupied and nc empty bands (Eq. chi0_GG at omega = 0 with occupations
    1 and 0, Eq. epsilon_-1 with the RPA kernel, Sec. III.A for W):
      chi0_GG'(q) = (2 / Omega) sum_k sum_{n,n'} (f_nk - f_n'k+q) n(G) conj(n(G')) / (e_nk - e_n'k+q),
      n = n_{nk,n'k+q} (the pair density of Sec. II.B), Omega = Nk Omega_cell,
      eps_GG' = delta_GG' - v^1/2(q+G) chi0_GG' v^1/2(q+G'),
      W_GG' = v^1/2(q+G) [eps^-1]_GG' v^1/2(q+G').
    The n, n' sum runs over (occupied, empty) and (empty, occupied) pairs, the
    only ones with f_nk != f_n'k+q.  vq [Nk][ng_max]: v(q+G) on each sphere
    (4 pi inside; the entry of G = 0 at q = 0 is not used).  At q = 0 the
    G = 0 row and column are left out of eps; W_00(0) = head and the wings are
    zero (the divergent head of Sec. II.C is replaced by a given value).
    Energies in eV, W in the units of v.  Returns W [Nk][ng_max][ng_max]."""
    nk, nv, nc = sys.nk, sys.nv, sys.nc
    n = np.array(sys.kmesh)
    omega = nk * sys.omega_cell
    W = np.zeros((nk, sys.ng_max, sys.ng_max), dtype=np.complex128)
    for q in range(nk):
        qv = np.array([q // (n[1] * n[2]), (q // n[2]) % n[1], q % n[2]])
        items, wts = [], []
        for k in range(nk):
            kv = np.array([k // (n[1] * n[2]), (k // n[2]) % n[1], k % n[2]])
            t = (kv + qv) % n
            kq = int((t[0] * n[1] + t[1]) * n[2] + t[2])
            for v in range(nv):
                for c in range(nc):
                    # occupied at k, empty at k + q
                    items.append((k, v, kq, nv + c))
                    wts.append(1.0 / ((sys.eps[k, v] - sys.eps[kq, nv + c]) / HARTREE_EV))
                    # empty at k, occupied at k + q
                    items.append((k, nv + c, kq, v))
                    wts.append(-1.0 / ((sys.eps[k, nv + c] - sys.eps[kq, v]) / HARTREE_EV))
        ng = sys.ng[q]
        rho = pair_density_items(sys, items)[:, :ng]
        chi0 = (2.0 / omega) * (rho.T * np.array(wts)) @ np.conj(rho)
        sv = np.sqrt(vq[q, :ng])
        g0 = 1 if q == 0 else 0
        e = np.eye(ng - g0) - sv[g0:, None] * chi0[g0:, g0:] * sv[None, g0:]
        W[q, g0:ng, g0:ng] = sv[g0:, None] * np.linalg.inv(e) * sv[None, g0:]
        if q == 0:
            W[0, 0, 0] = head
    return W


def unfold_W(W_irr, wsrc, wmap, ng):
    """W(q) at every q of the mesh from the matrices at the irreducible q
    points (Sec. III.A).  For q = T q_IBZ + G0 the screened interaction is that
    of q_IBZ at the rotated vectors T^-1(G + G0); for q = -T q_IBZ + G0 it is
    the complex conjugate at -T^-1(G + G0).  The rotated vectors are given as
    positions in the sphere of q_IBZ, wmap[q][G], with wsrc[q] = (index of
    q_IBZ, 1 when the time-reversed relation applies).  Entries past ng(q)
    stay zero.  Returns [Nk][ng_max][ng_max]."""
    nk, ngm = len(ng), W_irr.shape[1]
    W = np.zeros((nk, ngm, ngm), dtype=np.complex128)
    for q in range(nk):
        src, tr = int(wsrc[q][0]), int(wsrc[q][1])
        n = int(ng[q])
        for g in range(n):
            for gp in range(n):
                w = W_irr[src, wmap[q][g], wmap[q][gp]]
                W[q, g, gp] = np.conj(w) if tr else w
    return W


def fold_dW(dW, wsrc, wmap, ng, nirr, ng_max):
    """Gradient of a real L with respect to the matrices at the irreducible q
    points (the PyTorch convention dL/dRe + i dL/dIm), given its gradient
    with respect to W(q) at every q: the adjoint of the real-linear map of
    ``unfold_W`` (Sec. III.A).  Each entry (G, G') of W(q) reads the source
    entry (wmap[q][G], wmap[q][G']) itself, or its complex conjugate for the
    time-reversed images, so the source entry collects dW(q)[G][G'], or its
    conjugate, from every q and entry that read it.  Returns
    [nirr][ng_max][ng_max]."""
    out = np.zeros((nirr, ng_max, ng_max), dtype=np.complex128)
    for q in range(len(ng)):
        src, tr = int(wsrc[q][0]), int(wsrc[q][1])
        n = int(ng[q])
        for g in range(n):
            for gp in range(n):
                v = dW[q, g, gp]
                out[src, wmap[q][g], wmap[q][gp]] += np.conj(v) if tr else v
    return out
