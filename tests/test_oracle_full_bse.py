"""Pins of the oracle's Hamiltonian beyond the Tamm-Dancoff approximation
(e-h and h-e states of the BSE eigenproblem, Sec. II.C and the appendix;
optical limit).  CPU only."""
import dataclasses

import numpy as np

import bse_synth as B
import oracle as O


def small_system(**kw):
    base = dict(cell=B.cell_fcc(7.0), grid=(8, 8, 8), kmesh=(2, 2, 1), nv=2, nc=2, ecut=2.0, seed=13)
    base.update(kw)
    return B.make_system(**base)


def _blocks(H, ns):
    return H[:ns, :ns], H[:ns, ns:], H[ns:, :ns], H[ns:, ns:]


def test_resonant_block_is_the_tamm_dancoff_hamiltonian():
    for s in (B.make_config(0), small_system()):
        A = O.build_H(s)
        H = O.build_H_full(s)
        K = np.abs(A - np.diag(np.diag(A))).max()
        assert np.abs(H[: s.ns, : s.ns] - A).max() <= 1e-12 * K


def test_block_structure_and_paired_spectrum():
    """With Hermitian, time-reversal-consistent W, an inversion-closed sphere
    at q = 0 and an even v, the h-e blocks are fixed by the e-h ones:
    H = [[A, B], [-B^H, -conj(A)]], and the eigenvalues come in pairs E, -E."""
    for s in (B.make_config(0), small_system()):
        H = O.build_H_full(s)
        A, Bc, C, Dm = _blocks(H, s.ns)
        K = np.abs(A - np.diag(np.diag(A))).max()
        assert np.abs(Dm + np.conj(A)).max() <= 1e-12 * K
        assert np.abs(C + Bc.conj().T).max() <= 1e-12 * K
        assert np.abs(Bc).max() > 1e-2 * K  # the coupling is not negligible here
        ev = np.linalg.eigvals(H)
        pos = np.sort(ev.real[ev.real > 0])
        neg = np.sort(-ev.real[ev.real < 0])
        assert len(pos) == len(neg) == s.ns
        assert np.abs(pos - neg).max() <= 1e-10 * np.abs(ev).max()


def test_relation_fails_without_time_reversal_of_W():
    s = small_system(kmesh=(3, 1, 1))
    W = s.W.copy()
    W[1] *= 1.7  # Hermitian, no longer the TR image of W(q = 2)
    H = O.build_H_full(dataclasses.replace(s, W=W))
    A, Bc, C, Dm = _blocks(H, s.ns)
    K = np.abs(A - np.diag(np.diag(A))).max()
    assert np.abs(C + Bc.conj().T).max() > 1e-3 * K
    assert np.abs(Bc - Bc.T).max() > 1e-3 * K  # nor is the coupling block symmetric


def test_coupling_block_is_symmetric():
    """B^T = B (not B^H) for Hermitian, time-reversal-consistent W and an even
    v, with wave functions that carry no symmetry: the GPU contracts only the
    blocks k <= k' of B and writes the others as their transposes."""
    for s in (B.make_config(0), small_system(kmesh=(3, 1, 1)), small_system(kmesh=(2, 2, 1))):
        H = O.build_H_full(s)
        A, Bc, _, _ = _blocks(H, s.ns)
        K = np.abs(A - np.diag(np.diag(A))).max()
        assert np.abs(Bc - Bc.T).max() <= 1e-12 * K
        assert np.abs(Bc - Bc.conj().T).max() > 1e-3 * np.abs(Bc).max()


def test_zero_interaction_gives_plus_and_minus_transition_energies():
    s = small_system()
    s = dataclasses.replace(s, W=np.zeros_like(s.W), vx=np.zeros_like(s.vx))
    H = O.build_H_full(s)
    d = np.array([s.eps[k, s.nv + c] - s.eps[k, v] for k in range(s.nk) for v in range(s.nv) for c in range(s.nc)])
    assert np.abs(H - np.diag(np.concatenate([d, -d]))).max() < 1e-14


def test_coupling_block_full_grid_closed_form():
    """Whole-grid spheres, v = 1 off G = 0 and W = w I: by Parseval the
    coupling block B[(k v c), (k' v' c')] = K[(v k, c k), (c' k', v' k')]
    becomes real-space sums; its exchange keeps the G = 0 term of the mixed
    densities out explicitly."""
    s0 = small_system(grid=(6, 6, 6), ecut=1.0, kmesh=(3, 1, 1))
    g = np.array(s0.grid)
    allm = np.array([[a, b, c] for a in range(-(g[0] // 2), g[0] - g[0] // 2)
                     for b in range(-(g[1] // 2), g[1] - g[1] // 2)
                     for c in range(-(g[2] // 2), g[2] - g[2] // 2)], dtype=np.int32)
    allm = allm[np.lexsort((allm[:, 2], allm[:, 1], allm[:, 0], np.abs(allm).sum(1)))]
    ngm = len(allm)
    w = 0.41
    W = np.zeros((s0.nk, ngm, ngm), dtype=np.complex128)
    W[:, np.arange(ngm), np.arange(ngm)] = w
    s = dataclasses.replace(s0, gvec=np.ascontiguousarray(np.broadcast_to(allm, (s0.nk, ngm, 3))).astype(np.int32),
                            ng=np.full(s0.nk, ngm, dtype=np.int32), vx=np.ones(ngm), W=W)
    nv, nc, nt, ns = s.nv, s.nc, s.nv * s.nc, s.ns
    c = B.HARTREE_EV / (s.nk * s.omega_cell)
    H = O.build_H_full(s)
    u = s.u
    j = np.indices(s.grid).reshape(3, -1).T
    for ka in range(s.nk):
        for kb in range(s.nk):
            _, m0 = O.fold(s.kmesh, ka, kb)
            ph = np.exp(2j * np.pi * (j @ (m0 / g)))
            for v in range(nv):
                for c1 in range(nc):
                    x = np.conj(u[ka, v]) * u[ka, nv + c1]
                    for v2 in range(nv):
                        for c2 in range(nc):
                            y = np.conj(u[kb, nv + c2]) * u[kb, v2]
                            Vb = s.nr * np.sum(np.conj(x) * y) - np.conj(np.sum(x)) * np.sum(y)
                            f = np.conj(u[ka, v]) * u[kb, nv + c2] * ph
                            gg = np.conj(u[ka, nv + c1]) * u[kb, v2] * ph
                            D = w * s.nr * np.sum(np.conj(f) * gg)
                            want = c * (2 * Vb - D)
                            got = H[ka * nt + v * nc + c1, ns + kb * nt + v2 * nc + c2]
                            assert abs(got - want) < 1e-12 * max(1.0, abs(want))


def test_sampled_coupling_blocks_equal_the_whole_matrix():
    """The block-by-block coupling oracle (used on large shapes) against the
    coupling block of the whole beyond-TDA matrix."""
    for s in (B.make_config(0), small_system(kmesh=(3, 1, 1))):
        H = O.build_H_full(s)
        ns, nt = s.ns, s.nv * s.nc
        blocks = [(a, b) for a in range(s.nk) for b in range(s.nk)]
        got = O.coupling_blocks(s, blocks)
        scale = np.abs(H[:ns, ns:]).max()
        for (a, b), blk in zip(blocks, got):
            assert np.abs(H[a * nt:(a + 1) * nt, ns + b * nt:ns + (b + 1) * nt] - blk).max() <= 1e-12 * scale
