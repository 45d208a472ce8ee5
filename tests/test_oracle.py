"""Pins of the CPU oracle against facts fixed outside of it: values the paper
prints, closed forms, library routines and invariants.  CPU only."""
import dataclasses
import json
import math
import os

import numpy as np
import pytest

import bse_synth as B
import oracle as O

HERE = os.path.dirname(os.path.abspath(__file__))


def small_system(**kw):
    base = dict(cell=B.cell_fcc(7.0), grid=(8, 8, 8), kmesh=(2, 2, 1), nv=2, nc=2, ecut=2.0, seed=7)
    base.update(kw)
    return B.make_system(**base)


# ---------------------------------------------------------------- G-sphere

def test_si_sphere_holds_169_vectors():
    """Sec. IV.B prints 169 G vectors for the local-field cutoff; Si lattice from Sec. IV.A."""
    gold = json.load(open(os.path.join(HERE, "golden", "si_gsphere.json")))
    a = gold["a_angstrom"] / gold["bohr_angstrom"]
    for e in gold["ecut_eV_inside"]:
        m = B.gsphere(B.cell_fcc(a), np.zeros(3), e / B.HARTREE_EV)
        assert len(m) == gold["count"]


def test_sphere_is_closed_under_inversion_at_gamma():
    m = B.gsphere(B.cell_fcc(B.A_SI), np.zeros(3), 6.0)
    s = {tuple(x) for x in m}
    assert all(tuple(-x) in s for x in m)
    assert tuple(m[0]) == (0, 0, 0)


# ---------------------------------------------------------------- fold

@pytest.mark.parametrize("kmesh", [(2, 2, 2), (4, 3, 1), (3, 1, 5)])
def test_fold_reconstructs_k_difference(kmesh):
    n = np.array(kmesh)
    nk = int(np.prod(kmesh))
    for ka in range(nk):
        for kb in range(nk):
            iq, m0 = O.fold(kmesh, ka, kb)
            d = B.ktriplet(kmesh, kb) - B.ktriplet(kmesh, ka)
            qv = B.ktriplet(kmesh, iq)
            assert np.all((qv >= 0) & (qv < n))
            assert np.all(d == qv + n * m0)
            assert np.all((m0 == 0) | (m0 == -1))


# ---------------------------------------------------------------- pair densities

def _fft_reference(grid, ua, ub, m0, gv):
    p = (np.conj(ua) * ub).reshape(grid)
    F = np.fft.fftn(p)  # unnormalised forward DFT, exp(-2 pi i m.j/N)
    f = gv - m0
    return F[f[:, 0] % grid[0], f[:, 1] % grid[1], f[:, 2] % grid[2]]


@pytest.mark.parametrize("grid,m0", [((8, 8, 8), (0, 0, 0)), ((6, 8, 10), (-1, 0, -1)), ((5, 7, 4), (0, -1, 0))])
def test_pair_density_equals_library_dft(grid, m0):
    rng = np.random.default_rng(3)
    nr = int(np.prod(grid))
    ua = rng.standard_normal(nr) + 1j * rng.standard_normal(nr)
    ub = rng.standard_normal(nr) + 1j * rng.standard_normal(nr)
    gv = np.array([[a, b, c] for a in range(-2, 3) for b in range(-3, 3) for c in range(-1, 2)], dtype=np.int32)
    ref = _fft_reference(grid, ua, ub, np.array(m0), gv)
    full = O.pair_density(grid, ua, ub, m0, gv)
    sep = O.pair_density(grid, ua, ub, m0, gv, separable=True)
    scale = np.abs(ref).max()
    assert np.abs(full - ref).max() <= 1e-13 * scale
    assert np.abs(sep - ref).max() <= 1e-13 * scale


def test_pair_density_of_plane_waves_is_kronecker():
    grid = (6, 8, 10)
    j = np.stack(np.meshgrid(*[np.arange(n) for n in grid], indexing="ij"), -1).reshape(-1, 3)
    nr = len(j)

    def pw(m):
        return np.exp(2j * np.pi * (j @ (np.array(m) / np.array(grid)))) / math.sqrt(nr)

    Ma, Mb, m0 = np.array([1, -2, 3]), np.array([0, 1, -1]), np.array([-1, 0, -1])
    gv = np.array([[a, b, c] for a in range(-3, 3) for b in range(-4, 4) for c in range(-5, 5)], dtype=np.int32)
    out = O.pair_density(grid, pw(Ma), pw(Mb), m0, gv, separable=True)
    hit = np.all(((gv - m0) - (Mb - Ma)) % np.array(grid) == 0, axis=1)
    assert hit.sum() == 1
    assert abs(out[hit][0] - 1.0) < 1e-13
    assert np.abs(out[~hit]).max() < 1e-13


def test_pair_density_orthonormality_and_parseval():
    s = small_system()
    grid = s.grid
    allm = np.array([[a, b, c] for a in range(-4, 4) for b in range(-4, 4) for c in range(-4, 4)], dtype=np.int32)
    nb = s.nb
    for a in range(nb):
        for b in range(nb):
            n0 = O.pair_density(grid, s.u[1, a], s.u[1, b], (0, 0, 0), np.zeros((1, 3), np.int32))[0]
            assert abs(n0 - (1.0 if a == b else 0.0)) < 1e-13
    n = O.pair_density(grid, s.u[0, 1], s.u[3, 2], (0, -1, 0), allm, separable=True)
    lhs = np.sum(np.abs(n) ** 2)
    rhs = s.nr * np.sum(np.abs(s.u[0, 1] * s.u[3, 2]) ** 2)
    assert abs(lhs - rhs) <= 1e-12 * rhs


# ---------------------------------------------------------------- Hamiltonian

def _full_grid_system(s, w):
    """Same wave functions, but every sphere is the whole grid, v == 1 off G=0 and W = w I."""
    g = np.array(s.grid)
    allm = np.array([[a, b, c] for a in range(-(g[0] // 2), g[0] - g[0] // 2)
                     for b in range(-(g[1] // 2), g[1] - g[1] // 2)
                     for c in range(-(g[2] // 2), g[2] - g[2] // 2)], dtype=np.int32)
    order = np.lexsort((allm[:, 2], allm[:, 1], allm[:, 0], np.abs(allm).sum(1)))
    allm = allm[order]
    nk, ngm = s.nk, len(allm)
    gvec = np.ascontiguousarray(np.broadcast_to(allm, (nk, ngm, 3))).astype(np.int32)
    ng = np.full(nk, ngm, dtype=np.int32)
    vx = np.ones(ngm)
    vx[0] = 0.0
    W = np.zeros((nk, ngm, ngm), dtype=np.complex128)
    W[:, np.arange(ngm), np.arange(ngm)] = w
    return dataclasses.replace(s, gvec=gvec, ng=ng, vx=vx, W=W)


def test_blocks_match_real_space_closed_forms():
    """Full-grid sphere, v = 1 and W = w I: by Parseval the exchange and direct
    terms become real-space sums (the G0 shift only permutes the grid)."""
    s0 = small_system(grid=(6, 6, 6), ecut=1.0)
    w = 0.37
    s = _full_grid_system(s0, w)
    nv, nc, nb, nt = s.nv, s.nc, s.nb, s.nv * s.nc
    c = B.HARTREE_EV / (s.nk * s.omega_cell)
    blocks = [(0, 0), (0, 3), (3, 1), (2, 2), (1, 2)]
    got = O.build_blocks(s, blocks)
    u = s.u
    for bi, (ka, kb) in enumerate(blocks):
        for v in range(nv):
            for c1 in range(nc):
                for v2 in range(nv):
                    for c2 in range(nc):
                        uv, uc = u[ka, v], u[ka, nv + c1]
                        uv2, uc2 = u[kb, v2], u[kb, nv + c2]
                        Vb = s.nr * np.sum(uv * np.conj(uc) * np.conj(uv2) * uc2)
                        D = w * s.nr * np.sum(uv * np.conj(uv2) * np.conj(uc) * uc2)
                        h = c * (2 * Vb - D)
                        if ka == kb and v == v2 and c1 == c2:
                            h += s.eps[ka, nv + c1] - s.eps[ka, v]
                        assert abs(got[bi, v * nc + c1, v2 * nc + c2] - h) < 1e-12 * max(1.0, abs(h))


@pytest.mark.parametrize("m11", [(1, 1, 1), (1, 1, 0)])
def test_hand_built_two_band_two_k(m11):
    """One valence and one conduction band, k mesh 2x1x1, every u a single plane
    wave: each pair density is a Kronecker delta and H is a closed-form 2x2.
    m11 = (1,1,1) makes the off-diagonal element an off-diagonal entry of W(q)
    (so a transposed W fails); (1,1,0) makes it carry the exchange term."""
    s0 = B.make_system(B.cell_fcc(7.0), (8, 8, 8), (2, 1, 1), 1, 1, 4.0, seed=11)
    grid = np.array(s0.grid)
    j = np.stack(np.meshgrid(*[np.arange(n) for n in grid], indexing="ij"), -1).reshape(-1, 3)
    M = {(0, 0): np.array([0, 0, 0]), (0, 1): np.array([1, 0, 0]),
         (1, 0): np.array([0, 1, 0]), (1, 1): np.array(m11)}  # (k, band) -> plane wave
    u = np.zeros_like(s0.u)
    for (k, b), m in M.items():
        u[k, b] = np.exp(2j * np.pi * (j @ (m / grid))) / math.sqrt(s0.nr)
    s = dataclasses.replace(s0, u=u)
    H = O.build_H(s)

    c = B.HARTREE_EV / (s.nk * s.omega_cell)

    def gidx(iq, m):
        rows = np.where(np.all(s.gvec[iq, : s.ng[iq]] == m, axis=1))[0]
        return int(rows[0]) if len(rows) else None

    ref = np.zeros((2, 2), dtype=np.complex128)
    for ka in range(2):
        for kb in range(2):
            iq = (kb - ka) % 2
            m0 = np.array([(kb - ka - iq) // 2, 0, 0])
            h = 0.0
            xa = M[(ka, 1)] - M[(ka, 0)]
            xb = M[(kb, 1)] - M[(kb, 0)]
            if np.all(xa == xb):
                g = gidx(0, xa)
                if g is not None:
                    h += 2 * s.vx[g]
            gv = gidx(iq, M[(kb, 0)] - M[(ka, 0)] + m0)
            gc = gidx(iq, M[(kb, 1)] - M[(ka, 1)] + m0)
            if gv is not None and gc is not None:
                h -= s.W[iq, gv, gc]
            h *= c
            if ka == kb:
                h += s.eps[ka, 1] - s.eps[ka, 0]
            ref[ka, kb] = h
    # the off-diagonal element must actually probe the kernel (not zero by construction)
    assert abs(ref[0, 1]) > 1e-6
    assert np.abs(H - ref).max() < 1e-12
    e = np.linalg.eigvalsh(ref)
    tr, det = np.trace(ref).real, np.linalg.det(ref).real
    disc = math.sqrt(tr * tr / 4 - det)
    assert np.allclose(e, [tr / 2 - disc, tr / 2 + disc], atol=1e-12)
    assert np.allclose(O.exciton_energies(H, 2), e, atol=1e-12)


def test_H_is_hermitian_with_time_reversal_W():
    s = B.make_config(0)
    H = O.build_H(s)
    K = H - np.diag(np.diag(H))
    assert np.abs(H - H.conj().T).max() <= 1e-12 * np.abs(K).max()


def test_H_not_hermitian_without_time_reversal():
    """The Hermiticity check is sensitive: break the TR relation of W and it fails."""
    s = small_system(kmesh=(3, 1, 1))
    W = s.W.copy()
    W[1] *= 1.7  # still Hermitian, but no longer the TR image of W(q = 2)
    H = O.build_H(dataclasses.replace(s, W=W))
    K = H - np.diag(np.diag(H))
    assert np.abs(H - H.conj().T).max() > 1e-3 * np.abs(K).max()


def test_zero_interaction_gives_transition_energies():
    s = small_system()
    s = dataclasses.replace(s, W=np.zeros_like(s.W), vx=np.zeros_like(s.vx))
    H = O.build_H(s)
    d = np.array([s.eps[k, s.nv + c] - s.eps[k, v] for k in range(s.nk) for v in range(s.nv) for c in range(s.nc)])
    assert np.abs(H - np.diag(d)).max() < 1e-14
    assert np.all(d > 0)


def test_gauge_covariance():
    s = small_system()
    rng = np.random.default_rng(5)
    th = rng.uniform(0, 2 * np.pi, size=(s.nk, s.nb))
    s2 = dataclasses.replace(s, u=s.u * np.exp(1j * th)[:, :, None])
    H1, H2 = O.build_H(s), O.build_H(s2)
    phi = np.array([np.exp(1j * (th[k, s.nv + c] - th[k, v])) for k in range(s.nk) for v in range(s.nv)
                    for c in range(s.nc)])
    assert np.abs(H2 - np.conj(phi)[:, None] * H1 * phi[None, :]).max() < 1e-13
    assert np.allclose(np.linalg.eigvalsh(H1), np.linalg.eigvalsh(H2), atol=1e-12)


def test_separable_and_full_sums_agree_on_H():
    s = small_system(grid=(6, 6, 8))
    assert np.abs(O.build_H(s, separable=True) - O.build_H(s, separable=False)).max() < 1e-13
