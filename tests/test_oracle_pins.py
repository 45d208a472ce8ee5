"""Pins of the oracle's transition dipoles, its symmetric W directions and its
k.p matrix elements against values fixed by hand or by an independent
evaluation.  CPU only."""
import dataclasses
import math

import numpy as np
import pytest

import bse_synth as B
import oracle as O


def _grid_points(grid):
    return np.stack(np.meshgrid(*[np.arange(n) for n in grid], indexing="ij"), -1).reshape(-1, 3)


def _plane_wave_pair_system():
    """Simple-cubic cell a = 10 bohr, 8^3 grid, one k point, one valence and one
    conduction band: u_v = e^{i Ga.r}, u_c = (e^{i Ga.r} + e^{i Gb.r}) / sqrt 2
    with Ga = (2 pi / 10, 0, 0), Gb = (0, 2 pi / 10, 0); e_v = -1 eV, e_c = +1 eV."""
    s = B.make_system(B.cell_sc(10.0), (8, 8, 8), (1, 1, 1), 1, 1, 1.0, seed=1)
    grid = np.array(s.grid)
    j = _grid_points(grid)
    pw = lambda m: np.exp(2j * np.pi * (j @ (np.asarray(m) / grid))) / math.sqrt(s.nr)
    u = np.zeros_like(s.u)
    u[0, 0] = pw([1, 0, 0])
    u[0, 1] = (pw([1, 0, 0]) + pw([0, 1, 0])) / math.sqrt(2)
    eps = np.array([[-1.0, 1.0]])
    return dataclasses.replace(s, u=u, eps=eps)


def test_transition_dipole_of_plane_waves_in_hartree_units():
    """<u_v|grad|u_c> = i Ga / sqrt 2 (bohr^-1) and e_c - e_v = 2 eV =
    2 / 27.211386245988 Ha, so d_x = i (2 pi / 10) / sqrt 2 / (2 / 27.211386245988)
    = 6.044850183796866 i bohr (computed by hand to 30 digits).  A division by
    the energy difference in eV instead of Hartree would give 0.222 i."""
    s = _plane_wave_pair_system()
    dx = O.transition_dipoles(s, [1.0, 0.0, 0.0])
    assert dx.shape == (1,)
    assert abs(dx[0] - 6.044850183796866j) <= 1e-13 * 6.05
    # the polarisation enters linearly: (1,1,1)/sqrt 3 picks Ga_x / sqrt 3
    d111 = O.transition_dipoles(s, np.ones(3) / math.sqrt(3.0))
    assert abs(d111[0] - 3.4899958808260794j) <= 1e-13 * 3.5
    # y: Gb belongs to a plane wave orthogonal to u_v, so nothing
    dy = O.transition_dipoles(s, [0.0, 1.0, 0.0])
    assert abs(dy[0]) <= 1e-13
    # the sign of the energy difference (e_c - e_v > 0): swapping the bands'
    # energies flips d
    s2 = dataclasses.replace(s, eps=np.array([[1.0, -1.0]]))
    assert abs(O.transition_dipoles(s2, [1.0, 0.0, 0.0])[0] + 6.044850183796866j) <= 1e-12


def _symmetric(s, W, tol=1e-14):
    """Hermiticity of every W(q) and the time-reversal relation of Sec. III.A
    (T = 1): W_{G,G'}(q) = conj(W_{t-G,t-G'}(qbar)) with -q = qbar + t."""
    n = np.array(s.kmesh)
    worst = 0.0
    for iq in range(s.nk):
        g = s.ng[iq]
        Wq = W[iq, :g, :g]
        worst = max(worst, np.abs(Wq - Wq.conj().T).max())
        iv = B.ktriplet(s.kmesh, iq)
        qb = (-iv) % n
        t = (-iv - qb) // n
        iqb = B.kindex(s.kmesh, qb)
        lut = {tuple(m): i for i, m in enumerate(s.gvec[iqb, : s.ng[iqb]])}
        perm = np.array([lut[tuple(t - m)] for m in s.gvec[iq, :g]])
        worst = max(worst, np.abs(Wq - np.conj(W[iqb][np.ix_(perm, perm)])).max())
    return worst <= tol * max(np.abs(W).max(), 1.0), worst


def test_orbit_direction_keeps_W_symmetric():
    """W + h D stays Hermitian and time-reversal symmetric along every
    direction the oracle's finite-difference pins use; a generic orbit touches
    four entries, one whose time-reversal image is its own transpose two."""
    s = B.make_system(B.cell_fcc(8.0), (8, 8, 8), (3, 2, 1), 1, 1, 2.0, seed=3)
    assert _symmetric(s, s.W)[0]
    rng = np.random.default_rng(4)
    h = 0.37 - 0.21j
    counts = []
    for iq in range(s.nk):
        g, gp = (int(x) for x in rng.integers(1, s.ng[iq], 2))
        if g == gp:
            gp = (g % (s.ng[iq] - 1)) + 1
        D = O.orbit_direction(s, iq, g, gp, h)
        ok, worst = _symmetric(s, s.W + D)
        assert ok, (iq, g, gp, worst)
        counts.append(int(np.count_nonzero(D)))
        iqb, perm = B.tr_partner(s, iq)
        if iqb != iq:
            assert counts[-1] == 4
    # q = 0 is its own partner (t = 0): the image of (G, G') is (-G, -G');
    # pick G' = -G so the image is the transposed entry and the orbit has two
    lut = {tuple(m): i for i, m in enumerate(s.gvec[0, : s.ng[0]])}
    g = 1
    gp = lut[tuple(-s.gvec[0, g])]
    D = O.orbit_direction(s, 0, g, gp, h)
    assert _symmetric(s, s.W + D)[0]
    assert np.count_nonzero(D) == 2
    # a single-entry change is not symmetric, so the check above can fail
    D1 = np.zeros_like(s.W)
    D1[1, 1, 2] = h
    assert not _symmetric(s, s.W + D1)[0]


def _direct_dft(x, grid):
    """Unnormalised DFT X(m) = sum_j x(j) exp(-2 pi i m.j / N) as three direct
    sums along the axes (no FFT)."""
    y = x.reshape(grid)
    for d, N in enumerate(grid):
        j = np.arange(N)
        F = np.exp(-2j * np.pi * np.outer(j, j) / N)  # [m][j]
        y = np.moveaxis(np.tensordot(F, np.moveaxis(y, d, 0), axes=(1, 0)), 0, d)
    return y


@pytest.mark.parametrize("grid", [(6, 6, 8), (8, 6, 6)])
def test_grad_matrix_equals_direct_dft_evaluation(grid):
    """<u_v|grad|u_c> = (i / N_r) sum_m G_m conj(U_v(m)) U_c(m) with U the
    unnormalised DFT, signed frequencies and the Nyquist planes removed,
    evaluated here with direct DFT sums against the oracle's library FFT."""
    s = B.make_system(B.cell_fcc(6.0), grid, (2, 1, 1), 2, 3, 0.5, seed=8)
    b = 2 * np.pi * np.linalg.inv(s.cell).T
    f = []
    for N in grid:
        m = np.arange(N)
        sf = np.where(m > N // 2, m - N, m).astype(np.float64)
        if N % 2 == 0:
            sf[N // 2] = 0.0
        f.append(sf)
    Gm = (f[0][:, None, None, None] * b[0] + f[1][None, :, None, None] * b[1]
          + f[2][None, None, :, None] * b[2])  # [m1][m2][m3][xyz]
    ref = np.zeros((s.nk, s.nv, s.nc, 3), dtype=np.complex128)
    for k in range(s.nk):
        U = [_direct_dft(s.u[k, n], grid) for n in range(s.nb)]
        for v in range(s.nv):
            for c in range(s.nc):
                p = np.conj(U[v]) * U[s.nv + c]
                ref[k, v, c] = 1j / s.nr * np.einsum("xyz,xyzd->d", p, Gm)
    got = O.grad_matrix(s)
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()
