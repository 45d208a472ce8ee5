"""Pins of the oracle's dipoles and spectrum.  CPU only."""
import dataclasses
import math

import numpy as np

import bse_synth as B
import oracle as O


def test_dipole_of_plane_waves():
    """u_v = e^{iGa.r}, u_c = (e^{iGa.r} + e^{iGb.r})/sqrt 2 on the grid:
    <u_v|grad|u_c> = i Ga / sqrt 2 (Gb contributes nothing, being orthogonal)."""
    s = B.make_system(B.cell_fcc(7.0), (8, 8, 8), (1, 1, 1), 1, 1, 1.0, seed=1)
    grid = np.array(s.grid)
    j = np.stack(np.meshgrid(*[np.arange(n) for n in grid], indexing="ij"), -1).reshape(-1, 3)
    ma, mb = np.array([1, -2, 0]), np.array([0, 1, 3])
    pw = lambda m: np.exp(2j * np.pi * (j @ (m / grid))) / math.sqrt(s.nr)
    u = np.zeros_like(s.u)
    u[0, 0] = pw(ma)
    u[0, 1] = (pw(ma) + pw(mb)) / math.sqrt(2)
    s2 = dataclasses.replace(s, u=u)
    D = O.grad_matrix(s2)[0, 0, 0]
    b = 2 * np.pi * np.linalg.inv(s.cell).T
    assert np.allclose(D, 1j * (ma @ b) / math.sqrt(2), atol=1e-13)


def test_dipole_drops_nyquist_plane():
    s = B.make_system(B.cell_sc(8.0), (8, 8, 8), (1, 1, 1), 1, 1, 1.0, seed=1)
    grid = np.array(s.grid)
    j = np.stack(np.meshgrid(*[np.arange(n) for n in grid], indexing="ij"), -1).reshape(-1, 3)
    pw = lambda m: np.exp(2j * np.pi * (j @ (np.array(m) / grid))) / math.sqrt(s.nr)
    u = np.zeros_like(s.u)
    u[0, 0] = pw([4, 1, 0])  # Nyquist along axis 1
    u[0, 1] = pw([4, 1, 0])
    D = O.grad_matrix(dataclasses.replace(s, u=u))[0, 0, 0]
    b = 2 * np.pi * np.linalg.inv(s.cell).T
    assert np.allclose(D, 1j * (np.array([0, 1, 0]) @ b), atol=1e-13)


def _solved():
    s = B.make_config(0)
    H = O.build_H(s)
    E, A = np.linalg.eigh(H)
    d = O.transition_dipoles(s, [1.0, 0.0, 0.0])
    return s, H, E, A, d


def test_oscillator_strength_sum_rules():
    s, H, E, A, d = _solved()
    t = A.T @ d
    assert abs(np.sum(np.abs(t) ** 2) - np.sum(np.abs(d) ** 2)) <= 1e-12 * np.sum(np.abs(d) ** 2)
    # t = A^T d (the spectral representation pairs A^S_l with n_S(0)), so the
    # first moment is the quadratic form of H at conj(d)
    lhs = np.sum(E * np.abs(t) ** 2)
    rhs = np.real(d @ H @ np.conj(d))
    assert abs(lhs - rhs) <= 1e-12 * abs(rhs)


def test_spectrum_integral_matches_truncated_lorentzians():
    s, H, E, A, d = _solved()
    Eh = E / O.HARTREE_EV
    eta = 0.1 / O.HARTREE_EV
    w = np.linspace(0, 10, 20001) / O.HARTREE_EV
    pref = 8 * np.pi / (s.nk * s.omega_cell)
    e2 = O.spectrum(Eh, A, d, pref, (w, eta))
    t2 = np.abs(A.T @ d) ** 2
    exact = pref * np.sum(t2 * (np.arctan((w[-1] - Eh) / eta) - np.arctan((w[0] - Eh) / eta)))
    trap = np.sum(0.5 * (e2[1:] + e2[:-1]) * np.diff(w))
    assert abs(trap - exact) <= 1e-6 * exact
    # first moment: integral of w * Lorentzian over [w0, w1]
    m1 = pref * np.sum(t2 * (Eh * (np.arctan((w[-1] - Eh) / eta) - np.arctan((w[0] - Eh) / eta))
                            + 0.5 * eta * np.log(((w[-1] - Eh) ** 2 + eta ** 2) / ((w[0] - Eh) ** 2 + eta ** 2))))
    trap1 = np.sum(0.5 * (w[1:] * e2[1:] + w[:-1] * e2[:-1]) * np.diff(w))
    assert abs(trap1 - m1) <= 1e-6 * abs(m1)


def test_zero_kernel_spectrum_is_independent_transitions():
    s = B.make_config(0)
    s0 = dataclasses.replace(s, W=np.zeros_like(s.W), vx=np.zeros_like(s.vx))
    H = O.build_H(s0)
    E, A = np.linalg.eigh(H)
    d = O.transition_dipoles(s0, [0.0, 1.0, 0.0])
    t2 = np.abs(A.T @ d) ** 2
    de = np.real(np.diag(H))
    # truncated f-sum: sum_l E_l |t_l|^2 = sum_S de_S |d_S|^2
    assert abs(np.sum(E * t2) - np.sum(de * np.abs(d) ** 2)) <= 1e-12 * np.sum(de * np.abs(d) ** 2)
