"""Pins of the oracle's static RPA screened interaction (Eq. chi0_GG at
omega = 0, Eq. epsilon_-1, Sec. III.A).  CPU only."""
import dataclasses
import math

import numpy as np

import bse_synth as B
import oracle as O


def _plane_wave_system():
    """Simple-cubic a = 8 bohr, 8^3 grid, k mesh 2 x 1 x 1, one occupied and
    two empty bands, each a single plane wave: every pair density is a
    Kronecker delta, so chi0(q) and W(q) are diagonal in closed form."""
    s = B.make_system(B.cell_sc(8.0), (8, 8, 8), (2, 1, 1), 1, 2, 2.0, seed=5)
    grid = np.array(s.grid)
    j = np.stack(np.meshgrid(*[np.arange(n) for n in grid], indexing="ij"), -1).reshape(-1, 3)
    pw = lambda m: np.exp(2j * np.pi * (j @ (np.asarray(m) / grid))) / math.sqrt(s.nr)
    mill = {(0, 0): (0, 0, 0), (0, 1): (1, 0, 0), (0, 2): (0, 1, 0),   # (k, band): Miller index
            (1, 0): (0, 0, 1), (1, 1): (-1, 0, 0), (1, 2): (0, -1, 1)}
    u = np.zeros_like(s.u)
    for (k, n), m in mill.items():
        u[k, n] = pw(m)
    eps = np.array([[-1.0, 2.0, 3.0], [-0.5, 2.5, 4.0]])
    return dataclasses.replace(s, u=u, eps=eps), mill


def test_plane_wave_bands_give_diagonal_closed_form():
    s, mill = _plane_wave_system()
    vq = B.coulomb_table(s)
    head = 0.123
    W = O.screened_interaction(s, vq, head)
    omega = s.nk * s.omega_cell
    for q in range(s.nk):
        ng = s.ng[q]
        lut = {tuple(m): g for g, m in enumerate(s.gvec[q, :ng])}
        chi = np.zeros(ng)
        for k in range(s.nk):
            kq = (k + q) % 2
            t = ((k + q) - kq) // 2  # k + q = kq + t b1 (the mesh point kq lies a lattice vector back)
            for a, b in ((0, 1), (0, 2), (1, 0), (2, 0)):
                fa, fb = (1.0 if a == 0 else 0.0), (1.0 if b == 0 else 0.0)
                # psi_k^* psi_kq e^{-i(q+G).r} = u_a^* u_b e^{-i(G + t b1).r}: for plane
                # waves n_{a k, b kq}(G) = 1 where G = m_b(kq) - m_a(k) - t b1
                m = np.array(mill[(kq, b)]) - np.array(mill[(k, a)]) - np.array([t, 0, 0])
                g = lut.get(tuple(m))
                if g is None:
                    continue
                chi[g] += 2.0 / omega * (fa - fb) / ((s.eps[k, a] - s.eps[kq, b]) / O.HARTREE_EV)
        want = vq[q, :ng] / (1.0 - vq[q, :ng] * chi)
        if q == 0:
            want[0] = head
        got = W[q, :ng, :ng]
        assert np.abs(np.diag(got) - want).max() <= 1e-12 * np.abs(want).max(), q
        assert np.abs(got - np.diag(np.diag(got))).max() <= 1e-14 * np.abs(want).max(), q
        assert np.count_nonzero(chi) >= 2


def test_screening_is_hermitian_and_weakens_the_bare_interaction():
    """eps = 1 - v^1/2 chi0 v^1/2 >= 1 because chi0 <= 0, so W = v^1/2 eps^-1
    v^1/2 is Hermitian with v - W positive semidefinite (G != 0 at q = 0);
    time-reversal symmetric inputs give a W that obeys Sec. III.A's relation."""
    s = B.make_system(B.cell_fcc(8.0), (12, 12, 12), (2, 2, 1), 2, 4, 2.0, seed=6, time_reversal=True)
    vq = B.coulomb_table(s)
    W = O.screened_interaction(s, vq, 0.1)
    n = np.array(s.kmesh)
    for q in range(s.nk):
        ng = s.ng[q]
        Wq = W[q, :ng, :ng]
        assert np.abs(Wq - Wq.conj().T).max() <= 1e-12 * np.abs(Wq).max()
        g0 = 1 if q == 0 else 0
        d = np.diag(vq[q, g0:ng]) - Wq[g0:, g0:]
        assert np.linalg.eigvalsh(d).min() >= -1e-10 * np.abs(Wq).max()
        assert np.linalg.eigvalsh(d).max() > 1e-6 * np.abs(Wq).max()  # screening is not nothing
        iqb, perm = B.tr_partner(s, q)
        assert np.abs(Wq - np.conj(W[iqb][np.ix_(perm, perm)])).max() <= 1e-10 * np.abs(Wq).max()


def test_large_gap_leaves_the_bare_interaction():
    """Empty bands pushed 1e6 eV up: chi0 ~ 1e-6 of its size, W -> v."""
    s = B.make_system(B.cell_sc(8.0), (12, 12, 12), (2, 1, 1), 1, 2, 2.0, seed=7)
    eps = s.eps.copy()
    eps[:, s.nv:] += 1e6
    s = dataclasses.replace(s, eps=eps)
    vq = B.coulomb_table(s)
    W = O.screened_interaction(s, vq, 0.1)
    for q in range(s.nk):
        ng = s.ng[q]
        g0 = 1 if q == 0 else 0
        ref = np.diag(vq[q, g0:ng])
        assert np.abs(W[q, g0:ng, g0:ng] - ref).max() <= 1e-5 * np.abs(ref).max()


def test_orientation_of_chi0_with_a_two_plane_wave_band():
    """One k point, u_v = e^{i0.r}, u_c = (e^{iG1.r} + i e^{iG2.r}) / sqrt 2:
    n_vc(G) = 1/sqrt2 at G1, i/sqrt2 at G2, n_cv = the conjugate at -G1, -G2,
    so chi0 = (2/Omega) sum w n(G) conj(n(G')) has chi0_{G1,G2} = i/(Omega D)
    (D = e_c - e_v in Hartree); a transposed or conjugated chi0 has -i.  W is
    then v^1/2 (1 - v^1/2 chi0 v^1/2)^-1 v^1/2 on those four G."""
    s = B.make_system(B.cell_sc(8.0), (8, 8, 8), (1, 1, 1), 1, 1, 2.0, seed=8)
    grid = np.array(s.grid)
    j = np.stack(np.meshgrid(*[np.arange(n) for n in grid], indexing="ij"), -1).reshape(-1, 3)
    pw = lambda m: np.exp(2j * np.pi * (j @ (np.asarray(m) / grid))) / math.sqrt(s.nr)
    m1, m2 = (1, 0, 0), (0, 1, 1)
    u = np.zeros_like(s.u)
    u[0, 0] = pw((0, 0, 0))
    u[0, 1] = (pw(m1) + 1j * pw(m2)) / math.sqrt(2)
    s = dataclasses.replace(s, u=u, eps=np.array([[-1.0, 3.0]]))
    vq = B.coulomb_table(s)
    W = O.screened_interaction(s, vq, 0.1)
    lut = {tuple(m): g for g, m in enumerate(s.gvec[0, : s.ng[0]])}
    idx = [lut[m1], lut[m2], lut[tuple(-np.array(m1))], lut[tuple(-np.array(m2))]]
    D = 4.0 / O.HARTREE_EV
    c = 2.0 / s.omega_cell / (-D)  # (2 / Omega) (f_v - f_c) / (e_v - e_c) = the weight of both orders
    nvc = np.array([1, 1j, 0, 0]) / math.sqrt(2)
    ncv = np.array([0, 0, 1, -1j]) / math.sqrt(2)
    chi = c * (np.outer(nvc, nvc.conj()) + np.outer(ncv, ncv.conj()))
    assert abs(chi[0, 1] - 1j / (s.omega_cell * D)) <= 1e-12 * abs(chi[0, 1])
    sv = np.sqrt(vq[0, idx])
    want = sv[:, None] * np.linalg.inv(np.eye(4) - sv[:, None] * chi * sv[None, :]) * sv[None, :]
    got = W[0][np.ix_(idx, idx)]
    assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max()
    # every other G keeps the bare interaction
    rest = [g for g in range(1, s.ng[0]) if g not in idx]
    assert np.abs(np.diag(W[0])[rest] - vq[0, rest]).max() <= 1e-12 * vq[0, rest].max()
