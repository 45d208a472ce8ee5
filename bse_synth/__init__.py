"""Seeded synthetic inputs for the Tamm-Dancoff BSE Hamiltonian build.

This module is shared by the CPU oracle tests, the GPU tests and the benchmark.
It produces only *inputs*: periodic parts u_nk(r) of Bloch functions on a real
space grid, band energies, the plane-wave basis (G-spheres) of every momentum
transfer q, the bare Coulomb kernel on the q=0 sphere, and a screened
interaction W_GG'(q).  It contains none of the Hamiltonian arithmetic (no pair
densities, no exchange or direct terms, no k-pair folding).

Everything upstream of the Hamiltonian in the paper (ground-state DFT, the RPA
response and the inversion of the dielectric matrix) is replaced by seeded
random draws that have the structure the paper's quantities have:

* u_nk: complex Gaussian per grid point, orthonormalised per k (QR), so that
  sum_r |u|^2 = 1 and the bands at one k are orthogonal.
* eps: valence energies uniform in [-3, 0] eV, conduction in [1, 4] eV.
* W_GG'(q) = v^1/2(q+G) [eps^-1]_GG' v^1/2(q+G') with eps^-1 = (I + A A^H/N_G)^-1
  for a complex Gaussian A (Hermitian, positive definite), following the form
  of the statically screened interaction in Sec. III.A (4 pi inside v).
* The q = 0 head is fixed to 4 pi * 0.1 / Omega_cell and the wings are zero
  (the paper integrates the divergence out analytically, Sec. II.C; the
  synthetic value stands in for that result).
* W obeys the time-reversal relation of Sec. III.A with T = identity:
  W_{G,G'}(q) = conj(W_{-G-G0,-G'-G0}(qbar)) where -q = qbar + G0 folds back
  into the mesh.  Without it the Hamiltonian is not Hermitian.

Random numbers come from numpy PCG64 streams spawned from SeedSequence(seed):
[wave functions (one child per k), energies, W (one child per q), system draws].
"""
from __future__ import annotations

import dataclasses
import hashlib
import math
from typing import List, Optional, Sequence

import numpy as np

HARTREE_EV = 27.211386245988  # CODATA 2018


@dataclasses.dataclass
class System:
    name: str
    cell: np.ndarray          # (3,3) rows a1, a2, a3 in bohr
    grid: tuple               # (N1, N2, N3); N3 fastest in u
    kmesh: tuple              # (n1, n2, n3); k index (i1*n2 + i2)*n3 + i3
    nv: int
    nc: int
    ecut: float               # Hartree, sphere 1/2 |q+G|^2 <= ecut
    coulomb: str              # "bulk" or "slab"
    slab_L: float             # truncation length (slab only)
    head: float               # W_00(q=0), bohr units as stored
    ng: np.ndarray            # int32 [Nk]            sphere size per q index
    gvec: np.ndarray          # int32 [Nk][ng_max][3] Miller indices, padded with 0
    vx: np.ndarray            # float64 [ng_max]      v(G) on the q=0 sphere, entry 0 = 0
    u: np.ndarray             # complex128 [Nk][nb][Nr]
    eps: np.ndarray           # float64 [Nk][nb] eV, bands 0..nv-1 valence
    W: np.ndarray             # complex128 [Nk][ng_max][ng_max], padding zero
    seed: int
    qexc: int = 0             # exciton momentum Q as a q-mesh index (0: optical limit);
                              # vx then holds v(Q+G) on the sphere of Q
    # W from the irreducible q points (with_point_group_W): W_irr [nirr][ng_max][ng_max],
    # wsrc [Nk][2] = (irreducible index, 1 if conjugated), wmap [Nk][ng_max] = position in
    # the irreducible sphere of +-T^-1 (G + G0) for each G of the sphere of q (-1: padding)
    W_irr: Optional[np.ndarray] = None
    wsrc: Optional[np.ndarray] = None
    wmap: Optional[np.ndarray] = None

    @property
    def nk(self) -> int:
        return int(np.prod(self.kmesh))

    @property
    def nb(self) -> int:
        return self.nv + self.nc

    @property
    def nr(self) -> int:
        return int(np.prod(self.grid))

    @property
    def ns(self) -> int:
        return self.nk * self.nv * self.nc

    @property
    def ng_max(self) -> int:
        return int(self.gvec.shape[1])

    @property
    def omega_cell(self) -> float:
        return abs(float(np.linalg.det(self.cell)))

    def digest(self) -> str:
        h = hashlib.sha256()
        for a in (self.cell, self.ng, self.gvec, self.vx, self.u, self.eps, self.W):
            h.update(np.ascontiguousarray(a).tobytes())
        return h.hexdigest()[:16]


# ----------------------------------------------------------------------------
# lattices

def cell_sc(a: float) -> np.ndarray:
    return a * np.eye(3)


def cell_fcc(a: float) -> np.ndarray:
    return 0.5 * a * np.array([[0.0, 1.0, 1.0], [1.0, 0.0, 1.0], [1.0, 1.0, 0.0]])


def cell_hex(a: float, c: float) -> np.ndarray:
    return np.array([[a, 0.0, 0.0], [-0.5 * a, 0.5 * math.sqrt(3.0) * a, 0.0], [0.0, 0.0, c]])


def reciprocal(cell: np.ndarray) -> np.ndarray:
    """Rows b_d with a_i . b_j = 2 pi delta_ij."""
    return 2.0 * math.pi * np.linalg.inv(cell).T


def q_vector(cell: np.ndarray, kmesh: Sequence[int], iq: int) -> np.ndarray:
    n1, n2, n3 = kmesh
    i3 = iq % n3
    i2 = (iq // n3) % n2
    i1 = iq // (n2 * n3)
    frac = np.array([i1 / n1, i2 / n2, i3 / n3])
    return frac @ reciprocal(cell)


def gsphere(cell: np.ndarray, qv: np.ndarray, ecut: float) -> np.ndarray:
    """Miller indices m with 1/2 |q + sum_d m_d b_d|^2 <= ecut.

    Ordered by (|q+G|^2 rounded to 1e-12, m1, m2, m3), so that at q = 0 the
    first entry is G = 0.
    """
    b = reciprocal(cell)
    gmax = math.sqrt(2.0 * ecut)
    lens = np.linalg.norm(cell, axis=1)
    frac = np.linalg.solve(b.T, qv)  # q in units of b
    rng = [np.arange(int(math.floor(-frac[d] - gmax * lens[d] / (2 * math.pi))) - 1,
                     int(math.ceil(-frac[d] + gmax * lens[d] / (2 * math.pi))) + 2) for d in range(3)]
    m = np.stack(np.meshgrid(*rng, indexing="ij"), axis=-1).reshape(-1, 3)
    p = qv[None, :] + m @ b
    g2 = np.einsum("ij,ij->i", p, p)
    keep = 0.5 * g2 <= ecut * (1.0 + 1e-13)
    m = m[keep]
    g2 = np.round(g2[keep], 12)
    order = np.lexsort((m[:, 2], m[:, 1], m[:, 0], g2))
    return m[order].astype(np.int32)


def coulomb(p: np.ndarray, kind: str, slab_L: float) -> np.ndarray:
    """Bare Coulomb kernel 4 pi/|p|^2 (bulk) or its 2-D truncated form (slab,
    cell axis 3 along z).  Entries with p = 0 return 0; callers treat them."""
    p2 = np.einsum("ij,ij->i", p, p)
    out = np.zeros(len(p))
    nz = p2 > 1e-20
    out[nz] = 4.0 * math.pi / p2[nz]
    if kind == "slab":
        ppar = np.sqrt(p[:, 0] ** 2 + p[:, 1] ** 2)
        out[nz] *= 1.0 - np.exp(-ppar[nz] * slab_L / 2.0) * np.cos(p[nz, 2] * slab_L / 2.0)
    elif kind != "bulk":
        raise ValueError(kind)
    return out


def kindex(kmesh, i):
    n1, n2, n3 = kmesh
    return (i[0] * n2 + i[1]) * n3 + i[2]


def ktriplet(kmesh, k):
    n1, n2, n3 = kmesh
    return np.array([k // (n2 * n3), (k // n3) % n2, k % n3])


# ----------------------------------------------------------------------------
# generator

def make_system(cell, grid, kmesh, nv, nc, ecut, *, coulomb_kind="bulk", slab_L=0.0,
                head_factor=0.1, seed=1206, name="custom", wf="gaussian", wf_ecut=None,
                time_reversal=False, ss: Optional[np.random.SeedSequence] = None) -> System:
    """A synthetic system.  With ``time_reversal`` the wave functions and band
    energies obey time reversal without spin-orbit coupling: for kbar the mesh
    point of -k, -k = kbar - K with K a lattice vector (``k_partner``), and
    u_{n,kbar}(r_j) = exp(-i K . r_j) conj(u_{n,k}(r_j)), eps_{n,kbar} = eps_{n,k}
    for kbar != k.  At points that are their own partner u is drawn like any
    other (an eigensolver leaves a free phase per band there)."""
    cell = np.asarray(cell, dtype=np.float64)
    grid = tuple(int(x) for x in grid)
    kmesh = tuple(int(x) for x in kmesh)
    nk = int(np.prod(kmesh))
    nb = nv + nc
    nr = int(np.prod(grid))
    omega = abs(float(np.linalg.det(cell)))
    head = 4.0 * math.pi * head_factor / omega
    b = reciprocal(cell)

    if ss is None:
        ss = np.random.SeedSequence(seed)
    ss_wf, ss_eps, ss_w, _ = ss.spawn(4)

    # plane-wave basis per q
    spheres = [gsphere(cell, q_vector(cell, kmesh, iq), ecut) for iq in range(nk)]
    ng = np.array([len(s) for s in spheres], dtype=np.int32)
    ng_max = int(ng.max())
    gvec = np.zeros((nk, ng_max, 3), dtype=np.int32)
    for iq, s in enumerate(spheres):
        gvec[iq, : len(s)] = s
    assert np.all(gvec[0, 0] == 0), "G=0 must lead the q=0 sphere"
    # every shifted sphere must fit the grid without aliasing
    allm = np.concatenate(spheres)
    for d in range(3):
        span = int(allm[:, d].max() - allm[:, d].min()) + 1 + (1 if kmesh[d] > 1 else 0)
        if span > grid[d]:
            raise ValueError(f"G-sphere spans {span} > grid {grid[d]} along axis {d}")

    vx = np.zeros(ng_max)
    vx[: ng[0]] = coulomb(spheres[0] @ b, coulomb_kind, slab_L)
    vx[0] = 0.0

    # wave functions
    u = np.empty((nk, nb, nr), dtype=np.complex128)
    kids = ss_wf.spawn(nk)
    if wf == "bandlimited":
        msph = gsphere(cell, np.zeros(3), wf_ecut)
    elif wf != "gaussian":
        raise ValueError(wf)
    for k in range(nk):
        kb, K = k_partner(kmesh, k)
        if time_reversal and kb < k:
            u[k] = u_partner(u[kb], grid, K)
            continue
        rng = np.random.Generator(np.random.PCG64(kids[k]))
        if wf == "gaussian":
            z = rng.standard_normal((nr, nb)) + 1j * rng.standard_normal((nr, nb))
        else:
            # random coefficients on a small sphere of plane waves, then inverse DFT
            c = rng.standard_normal((len(msph), nb)) + 1j * rng.standard_normal((len(msph), nb))
            spec = np.zeros(grid + (nb,), dtype=np.complex128)
            spec[msph[:, 0] % grid[0], msph[:, 1] % grid[1], msph[:, 2] % grid[2]] = c
            z = np.fft.ifftn(spec, axes=(0, 1, 2)).reshape(nr, nb)
        q, _ = np.linalg.qr(z)
        u[k] = q.T

    # energies
    rng = np.random.Generator(np.random.PCG64(ss_eps))
    eps = np.empty((nk, nb))
    eps[:, :nv] = rng.uniform(-3.0, 0.0, size=(nk, nv))
    eps[:, nv:] = rng.uniform(1.0, 4.0, size=(nk, nc))
    if time_reversal:
        for k in range(nk):
            kb, _ = k_partner(kmesh, k)
            if kb < k:
                eps[k] = eps[kb]

    # screened interaction, one representative per time-reversal orbit
    W = np.zeros((nk, ng_max, ng_max), dtype=np.complex128)
    done = np.zeros(nk, dtype=bool)
    wkids = ss_w.spawn(nk)
    n = np.array(kmesh)
    for iq in range(nk):
        if done[iq]:
            continue
        rng = np.random.Generator(np.random.PCG64(wkids[iq]))
        s = spheres[iq]
        g = len(s)
        qv = q_vector(cell, kmesh, iq)
        A = rng.standard_normal((g, g)) + 1j * rng.standard_normal((g, g))
        M = np.eye(g) + (A @ A.conj().T) / g
        Lc = np.linalg.cholesky(M)
        Li = np.linalg.solve(Lc, np.eye(g))
        einv = Li.conj().T @ Li
        v = coulomb(qv[None, :] + s @ b, coulomb_kind, slab_L)
        sv = np.sqrt(v)
        Wq = sv[:, None] * einv * sv[None, :]
        if iq == 0:
            Wq[0, :] = 0.0
            Wq[:, 0] = 0.0
            Wq[0, 0] = head
        Wq = 0.5 * (Wq + Wq.conj().T)
        # time-reversal partner: -iq = qbar + n t
        iv = ktriplet(kmesh, iq)
        qb = (-iv) % n
        t = (-iv - qb) // n
        iqb = kindex(kmesh, qb)
        sb = spheres[iqb]
        lut = {tuple(m): i for i, m in enumerate(sb)}
        perm = np.array([lut[tuple(t - m)] for m in s])
        if iqb == iq:
            Wq = 0.5 * (Wq + np.conj(Wq[np.ix_(perm, perm)]))
            W[iq, :g, :g] = Wq
        else:
            W[iq, :g, :g] = Wq
            Wb = np.zeros((g, g), dtype=np.complex128)
            Wb[np.ix_(perm, perm)] = np.conj(Wq)
            W[iqb, :g, :g] = Wb
            done[iqb] = True
        done[iq] = True

    return System(name=name, cell=cell, grid=grid, kmesh=kmesh, nv=nv, nc=nc, ecut=ecut,
                  coulomb=coulomb_kind, slab_L=slab_L, head=head, ng=ng, gvec=gvec, vx=vx,
                  u=u, eps=eps, W=W, seed=seed)


def coulomb_table(sys: System) -> np.ndarray:
    """v(q + G) on the sphere of every q, [Nk][ng_max] (4 pi inside; bulk or
    the slab's truncated form; zero at q = 0, G = 0 and in the padding): the
    bare interaction that the screening turns into W."""
    b = reciprocal(sys.cell)
    out = np.zeros((sys.nk, sys.ng_max))
    for iq in range(sys.nk):
        g = sys.ng[iq]
        p = q_vector(sys.cell, sys.kmesh, iq)[None, :] + sys.gvec[iq, :g] @ b
        out[iq, :g] = coulomb(p, sys.coulomb, sys.slab_L)
    return out


# ----------------------------------------------------------------------------
# point-group symmetry of the q mesh (Sec. III.A)

def point_group(cell: np.ndarray, kmesh, proper: bool = False) -> List[np.ndarray]:
    """The point-group operations of the lattice (with ``proper`` only its
    rotations, the group of a crystal without inversion) that also map the
    Gamma-centred mesh onto itself, as integer matrices M acting on
    coordinates in the basis of the reciprocal vectors: T q has coordinates
    M f when q has f.  Found among the matrices with entries in {-1, 0, 1}
    whose Cartesian form is orthogonal (48 for cubic cells, 24 for hexagonal
    ones).  The identity comes first."""
    b = reciprocal(cell)                 # rows b_d: q = f @ b
    n = np.array(kmesh)
    ops = []
    for code in range(3 ** 9):
        d = [(code // 3 ** i) % 3 - 1 for i in range(9)]
        Mi = np.array(d, dtype=np.int64).reshape(3, 3)
        if abs(round(np.linalg.det(Mi))) != 1:
            continue
        R = b.T @ Mi @ np.linalg.inv(b.T)   # b^T M = R b^T
        if np.abs(R @ R.T - np.eye(3)).max() > 1e-9:
            continue
        if proper and np.linalg.det(R) < 0:
            continue
        # the mesh i / n maps onto itself: n_d M_de / n_e must be integers
        if np.any((Mi * n[:, None]) % n[None, :] != 0):
            continue
        ops.append(Mi)
    ident = [i for i, M in enumerate(ops) if np.array_equal(M, np.eye(3, dtype=np.int64))][0]
    ops.insert(0, ops.pop(ident))
    return ops


def _mesh_op(M: np.ndarray, kmesh) -> np.ndarray:
    """M in units of the mesh: the integer matrix taking the triplet i of q
    (coordinates i / n) to n * (M (i / n))."""
    n = np.array(kmesh, dtype=np.int64)
    return (M * n[:, None]) // n[None, :]


def irreducible_q(cell: np.ndarray, kmesh, proper: bool = False):
    """Irreducible q points of the mesh under the point group and time
    reversal: (ops, reps, assign) with, for every q, assign[q] = (rep, op
    index, s, G0) such that q = s T_op q_rep + G0 (s = -1: the time-reversed
    image), G0 in reciprocal-lattice coordinates.  Each irreducible point is
    the first mesh point of its orbit and maps to itself by the identity."""
    ops = point_group(cell, kmesh, proper)
    n = np.array(kmesh)
    nk = int(np.prod(n))
    assign = [None] * nk
    reps = []
    for q in range(nk):
        if assign[q] is not None:
            continue
        reps.append(q)
        iq = ktriplet(kmesh, q)
        for oi, M in enumerate(ops):
            for s in (1, -1):
                # s T q_rep in mesh units; the mesh point it folds to, and
                # G0 = q - s T q_rep
                tm = s * (_mesh_op(M, kmesh) @ iq)
                tgt = kindex(kmesh, tm % n)
                if assign[tgt] is None:
                    assign[tgt] = (q, oi, s, ((tm % n) - tm) // n)
    return ops, reps, assign


def _sphere_map(sys: System, ops_inv, q, rep, oi, s, g0):
    """Position in the sphere of rep of s T^-1 (G + G0) for each G of the
    sphere of q (-1 past ng(q))."""
    ng = int(sys.ng[q])
    if ng != int(sys.ng[rep]):
        raise ValueError(f"spheres of q = {q} and its irreducible point {rep} differ in size")
    pos = {tuple(m): g for g, m in enumerate(sys.gvec[rep, :ng])}
    out = np.full(sys.ng_max, -1, dtype=np.int32)
    for g in range(ng):
        m = s * (ops_inv[oi] @ (sys.gvec[q, g].astype(np.int64) + g0))
        out[g] = pos[tuple(int(x) for x in m)]
    return out


def point_group_maps(sys: System, proper: bool = False):
    """The index maps that give W at every q from W at the irreducible q
    points (Sec. III.A): (reps, wsrc [Nk][2], wmap [Nk][ng_max]) with
    wsrc[q] = (position of the irreducible point in reps, 1 for the
    time-reversed relation) and wmap[q][G] the position of s T^-1(G + G0) in
    the sphere of the irreducible point (-1 past ng(q))."""
    ops, reps, assign = irreducible_q(sys.cell, sys.kmesh, proper)
    inv = [np.rint(np.linalg.inv(M)).astype(np.int64) for M in ops]
    at = {q: i for i, q in enumerate(reps)}
    wsrc = np.zeros((sys.nk, 2), dtype=np.int32)
    wmap = np.full((sys.nk, sys.ng_max), -1, dtype=np.int32)
    for q in range(sys.nk):
        rep, oi, s, g0 = assign[q]
        wsrc[q] = (at[rep], 1 if s < 0 else 0)
        wmap[q] = _sphere_map(sys, inv, q, rep, oi, s, g0)
    return reps, wsrc, wmap


def with_point_group_W(sys: System, proper: bool = False) -> System:
    """The same inputs with W made symmetric under the cubic point group (or
    its rotations only, ``proper``) and time reversal, stored both ways: W at
    every q, and W_irr at the irreducible q points with the maps of
    ``point_group_maps``.  W at each irreducible point is the average of W
    over the operations that leave that point in place (images taken as in
    Sec. III.A); every other W(q) is its image through the maps."""
    ops, reps, assign = irreducible_q(sys.cell, sys.kmesh, proper)
    inv = [np.rint(np.linalg.inv(M)).astype(np.int64) for M in ops]
    reps2, wsrc, wmap = point_group_maps(sys, proper)
    assert reps2 == reps
    n = np.array(sys.kmesh)
    ngm = sys.ng_max

    def image(Wr, mp, ng, conj):
        X = np.zeros((ngm, ngm), dtype=np.complex128)
        X[:ng, :ng] = Wr[np.ix_(mp[:ng], mp[:ng])]
        return np.conj(X) if conj else X

    W_irr = np.zeros((len(reps), ngm, ngm), dtype=np.complex128)
    for i, q in enumerate(reps):
        iq = ktriplet(sys.kmesh, q)
        ng = int(sys.ng[q])
        acc = np.zeros((ngm, ngm), dtype=np.complex128)
        cnt = 0
        for oi, M in enumerate(ops):
            for s in (1, -1):
                tm = s * (_mesh_op(M, sys.kmesh) @ iq)
                if kindex(sys.kmesh, tm % n) != q:
                    continue
                acc += image(sys.W[q], _sphere_map(sys, inv, q, q, oi, s, ((tm % n) - tm) // n), ng, s < 0)
                cnt += 1
        W_irr[i] = acc / cnt
    W = np.zeros_like(sys.W)
    for q in range(sys.nk):
        W[q] = image(W_irr[wsrc[q, 0]], wmap[q], int(sys.ng[q]), wsrc[q, 1] != 0)
    tag = "-ibzO" if proper else "-ibz"
    return dataclasses.replace(sys, W=W, W_irr=W_irr, wsrc=wsrc, wmap=wmap, name=f"{sys.name}{tag}")


def k_plus(kmesh, k: int, q: int) -> int:
    """Mesh index of k + q (each component modulo the mesh)."""
    n = np.array(kmesh)
    return kindex(kmesh, (ktriplet(kmesh, k) + ktriplet(kmesh, q)) % n)


def with_exciton_momentum(sys: System, qexc: int) -> System:
    """The same inputs with exciton momentum Q = q-mesh point ``qexc``: the
    electron of S = (k, v, c) sits at k + Q, and vx becomes v(Q + G) on the
    sphere of Q (the entry of G = 0 set to zero, wherever it sits)."""
    vx = coulomb_table(sys)[qexc].copy()
    g0 = np.flatnonzero(np.all(sys.gvec[qexc, : sys.ng[qexc]] == 0, axis=1))
    vx[g0] = 0.0
    return dataclasses.replace(sys, qexc=int(qexc), vx=vx, name=f"{sys.name}-Q{qexc}")


def k_partner(kmesh, k: int):
    """(kbar, K): kbar the mesh index of -k, K the integer triplet with
    -k = kbar - K in units of the mesh (each entry 0 or 1)."""
    n = np.array(kmesh)
    iv = ktriplet(kmesh, k)
    kb = (-iv) % n
    return kindex(kmesh, kb), (kb + iv) // n


def tr_phase(grid, K) -> np.ndarray:
    """exp(-i K . r_j) on the grid points r_j = j / N (flattened like u)."""
    j = np.indices(grid).reshape(3, -1).T
    return np.exp(-2j * np.pi * (j @ (np.asarray(K, dtype=np.float64) / np.array(grid))))


def u_partner(uk: np.ndarray, grid, K) -> np.ndarray:
    """Wave functions at kbar from those at k under time reversal: [nb, nr]."""
    return np.conj(uk) * tr_phase(grid, K)[None, :]


def tr_partner(sys: System, iq: int):
    """Index bookkeeping of time reversal on the q mesh and the spheres:
    (qbar, perm) with -q = qbar + t (t a lattice vector) and perm[g] the
    index of t - m_g in the sphere of qbar (-1 if it is not there)."""
    n = np.array(sys.kmesh)
    iv = ktriplet(sys.kmesh, iq)
    qb = (-iv) % n
    t = (-iv - qb) // n
    iqb = kindex(sys.kmesh, qb)
    lut = {tuple(m): i for i, m in enumerate(sys.gvec[iqb, :sys.ng[iqb]])}
    perm = np.array([lut.get(tuple(t - m), -1) for m in sys.gvec[iq, :sys.ng[iq]]])
    return iqb, perm


def symmetric_direction(sys: System, iq: int, g: int, h: int, z: complex) -> np.ndarray:
    """A change of W that keeps it Hermitian and time-reversal symmetric:
    z at (q, g, h), conj(z) at (q, h, g), and the conjugate images at the
    time-reversal partner; each distinct (entry, conjugated) image once, so
    an entry that is its own image gets z + conj(z) (an imaginary z there
    gives a zero direction)."""
    D = np.zeros_like(sys.W)
    for (q, a, b), v in symmetric_entries(sys, iq, g, h, z).items():
        D[q, a, b] = v
    return D


def symmetric_entries(sys: System, iq: int, g: int, h: int, z: complex) -> dict:
    """The non-zero entries {(q, g, g'): value} of ``symmetric_direction``."""
    iqb, perm = tr_partner(sys, iq)
    images = {(iq, g, h, False), (iq, h, g, True), (iqb, int(perm[g]), int(perm[h]), True),
              (iqb, int(perm[h]), int(perm[g]), False)}
    out = {}
    for q, a, b, cj in images:
        out[(q, a, b)] = out.get((q, a, b), 0.0) + (np.conj(z) if cj else z)
    return {k: v for k, v in out.items() if v != 0}


# ----------------------------------------------------------------------------
# the named workloads

CONFIG_NAMES = {
    0: "tiny-sc16-k2-b2x2",
    1: "si-fcc24-k4-b3x3",
    2: "si-fcc32-k8-b4x4",
    3: "hbn-hex24x24x96-ragged16-b4x4",
    4: "si-fcc32-k8-b4x4-backward",
}

A_SI = 10.26        # bohr (5.431 angstrom)
A_HBN = 4.74        # bohr
C_HBN = 30.0        # bohr: 15 bohr of vacuum on each side of the sheet
HBN_MESHES = (6, 8, 9, 12)


def make_config(i: int, seed: Optional[int] = None, **over):
    """Workload i (0..4).  Config 3 returns a list of 16 systems."""
    if seed is None:
        seed = 1206 + i
    if i == 0:
        kw = dict(cell=cell_sc(10.0), grid=(16, 16, 16), kmesh=(2, 2, 2), nv=2, nc=2, ecut=3.0)
    elif i == 1:
        kw = dict(cell=cell_fcc(A_SI), grid=(24, 24, 24), kmesh=(4, 4, 4), nv=3, nc=3, ecut=6.0)
    elif i in (2, 4):
        kw = dict(cell=cell_fcc(A_SI), grid=(32, 32, 32), kmesh=(8, 8, 8), nv=4, nc=4, ecut=8.0)
    elif i == 3:
        nsys = over.pop("nsys", 16)
        return make_hbn_batch(seed, nsys=nsys, **over)
    else:
        raise ValueError(i)
    kw.update(over)
    return make_system(seed=seed, name=CONFIG_NAMES[i], **kw)


def hbn_draws(seed: int, nsys: int = 16) -> List[int]:
    ss = np.random.SeedSequence(seed)
    _, _, _, ss_sys = ss.spawn(4)
    rng = np.random.Generator(np.random.PCG64(ss_sys))
    return [int(x) for x in rng.choice(HBN_MESHES, size=nsys)]


def make_hbn_batch(seed: int, nsys: int = 16, grid=(24, 24, 96), ecut=9.0, nv=4, nc=4,
                   meshes: Optional[Sequence[int]] = None, time_reversal=False,
                   only: Optional[Sequence[int]] = None) -> List[System]:
    """``nsys`` hexagonal cells with k meshes n x n x 1 (n drawn per system).
    ``only``: generate just these members of the batch (identical to the
    same members of the whole batch)."""
    ss = np.random.SeedSequence(seed)
    _, _, _, ss_sys = ss.spawn(4)
    kids = ss_sys.spawn(nsys)
    if meshes is None:
        meshes = hbn_draws(seed, nsys)
    out = []
    for s in (range(nsys) if only is None else only):
        n = int(meshes[s])
        out.append(make_system(cell_hex(A_HBN, C_HBN), grid, (n, n, 1), nv, nc, ecut,
                               coulomb_kind="slab", slab_L=C_HBN, seed=seed,
                               name=f"hbn{s}-k{n}", ss=kids[s], time_reversal=time_reversal))
    return out
