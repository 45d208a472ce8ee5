"""Pins of the oracle's Hamiltonian at finite exciton momentum Q (the e-h
basis S = (n k, m k+q) of the BSE eigenproblem of Sec. II.C; Eqs. V_eh and
W_SS with the electron at k + Q).  CPU only."""
import dataclasses

import numpy as np
import pytest

import bse_synth as B
import oracle as O


def small_system(**kw):
    base = dict(cell=B.cell_fcc(7.0), grid=(8, 8, 8), kmesh=(3, 1, 1), nv=2, nc=2, ecut=2.0, seed=11)
    base.update(kw)
    return B.make_system(**base)


def test_zero_momentum_is_the_optical_hamiltonian():
    """Q = 0 through the finite-Q assembly (every block from batched pair
    densities) equals the block-by-block oracle of the optical limit."""
    for s in (B.make_config(0), small_system(kmesh=(2, 2, 1))):
        H0 = O.build_H(s)
        H1 = O.build_H_exciton(s)
        K = np.abs(H0 - np.diag(np.diag(H0))).max()
        assert np.abs(H0 - H1).max() <= 1e-12 * K


def test_mesh_addition():
    km = (3, 2, 4)
    for k in range(24):
        for q in range(24):
            kq = O.k_plus_q(km, k, q)
            a = np.array(B.ktriplet(km, k)) + np.array(B.ktriplet(km, q))
            assert np.array_equal(np.array(B.ktriplet(km, kq)), a % np.array(km))


def _full_grid(s, w):
    """Every sphere the whole grid, v = 1 off G = 0, W = w I."""
    g = np.array(s.grid)
    allm = np.array([[a, b, c] for a in range(-(g[0] // 2), g[0] - g[0] // 2)
                     for b in range(-(g[1] // 2), g[1] - g[1] // 2)
                     for c in range(-(g[2] // 2), g[2] - g[2] // 2)], dtype=np.int32)
    order = np.lexsort((allm[:, 2], allm[:, 1], allm[:, 0], np.abs(allm).sum(1)))
    allm = allm[order]
    ngm = len(allm)
    gvec = np.ascontiguousarray(np.broadcast_to(allm, (s.nk, ngm, 3))).astype(np.int32)
    vx = np.ones(ngm)
    W = np.zeros((s.nk, ngm, ngm), dtype=np.complex128)
    W[:, np.arange(ngm), np.arange(ngm)] = w
    return dataclasses.replace(s, gvec=gvec, ng=np.full(s.nk, ngm, dtype=np.int32), vx=vx, W=W)


@pytest.mark.parametrize("Q", [1, 2])
def test_full_grid_closed_forms_with_shifted_conduction_pairs(Q):
    """Whole-grid spheres, v = 1 and W = w I: by Parseval both terms become
    real-space sums.  On a 3-point mesh the pairs (k+Q, k'+Q) of the direct
    term and (k, k+Q) of the exchange wrap differently from (k, k'), so the
    closed forms carry the phases exp(2 pi i (m0' - m0).j / N) and
    exp(2 pi i m0x.j / N); a G0 taken from the wrong pair fails them.  The
    exchange drops the G = 0 term, which at Q != 0 is not zero."""
    w = 0.37
    s = _full_grid(small_system(grid=(6, 6, 6), ecut=1.0), w)
    s = dataclasses.replace(s, qexc=Q)
    nv, nc, nt = s.nv, s.nc, s.nv * s.nc
    c = B.HARTREE_EV / (s.nk * s.omega_cell)
    H = O.build_H_exciton(s)
    grid = np.array(s.grid)
    j = np.indices(s.grid).reshape(3, -1).T
    ph = lambda m0: np.exp(2j * np.pi * (j @ (np.asarray(m0) / grid)))
    kq = [O.k_plus_q(s.kmesh, k, Q) for k in range(s.nk)]
    u = s.u
    wraps = set()
    for ka in range(s.nk):
        for kb in range(s.nk):
            _, m0 = O.fold(s.kmesh, ka, kb)
            _, m0c = O.fold(s.kmesh, kq[ka], kq[kb])
            _, mxa = O.fold(s.kmesh, ka, kq[ka])
            _, mxb = O.fold(s.kmesh, kb, kq[kb])
            wraps.add(tuple(m0c - m0))
            for v in range(nv):
                for c1 in range(nc):
                    xa = np.conj(u[ka, v]) * u[kq[ka], nv + c1] * ph(mxa)
                    for v2 in range(nv):
                        for c2 in range(nc):
                            xb = np.conj(u[kb, v2]) * u[kq[kb], nv + c2] * ph(mxb)
                            Vb = s.nr * np.sum(np.conj(xa) * xb) - np.conj(np.sum(xa)) * np.sum(xb)
                            D = w * s.nr * np.sum(u[ka, v] * np.conj(u[kb, v2]) * np.conj(u[kq[ka], nv + c1])
                                                  * u[kq[kb], nv + c2] * ph(m0c - m0))
                            h = c * (2 * Vb - D)
                            if ka == kb and v == v2 and c1 == c2:
                                h += s.eps[kq[ka], nv + c1] - s.eps[ka, v]
                            got = H[ka * nt + v * nc + c1, kb * nt + v2 * nc + c2]
                            assert abs(got - h) < 1e-12 * max(1.0, abs(h))
    assert len(wraps) > 1  # some conduction pairs wrap differently from their (k, k')


def test_hermitian_at_finite_momentum_and_sensitive_to_time_reversal():
    s = B.with_exciton_momentum(small_system(), 1)
    H = O.build_H_exciton(s)
    K = np.abs(H - np.diag(np.diag(H))).max()
    assert np.abs(H - H.conj().T).max() <= 1e-12 * K
    W = s.W.copy()
    W[1] *= 1.7  # Hermitian, no longer the TR image of W(q = 2)
    H = O.build_H_exciton(dataclasses.replace(s, W=W))
    assert np.abs(H - H.conj().T).max() > 1e-3 * K


def test_zero_interaction_gives_shifted_transition_energies():
    s = B.with_exciton_momentum(small_system(kmesh=(2, 2, 1)), 3)
    s = dataclasses.replace(s, W=np.zeros_like(s.W), vx=np.zeros_like(s.vx))
    H = O.build_H_exciton(s)
    kq = [B.k_plus(s.kmesh, k, 3) for k in range(s.nk)]
    d = np.array([s.eps[kq[k], s.nv + c] - s.eps[k, v] for k in range(s.nk) for v in range(s.nv)
                  for c in range(s.nc)])
    assert np.abs(H - np.diag(d)).max() < 1e-14


def test_generator_coulomb_of_the_exciton_momentum():
    """vx of the finite-Q inputs is v(Q+G) = 4 pi / |Q+G|^2 on the sphere of
    Q, zero at G = 0 only."""
    s = small_system()
    t = B.with_exciton_momentum(s, 1)
    b = B.reciprocal(s.cell)
    ng = s.ng[1]
    p = B.q_vector(s.cell, s.kmesh, 1)[None, :] + s.gvec[1, :ng] @ b
    want = 4 * np.pi / np.sum(p * p, axis=1)
    want[np.all(s.gvec[1, :ng] == 0, axis=1)] = 0.0
    assert np.allclose(t.vx[:ng], want, rtol=1e-14, atol=0)
    assert np.count_nonzero(t.vx[:ng] == 0.0) == 1
