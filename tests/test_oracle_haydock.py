"""Pins of the oracle's Lanczos recurrence and continued fraction (the
resolvent of the appendix evaluated without eigenpairs).  CPU only."""
import numpy as np

import bse_synth as B
import oracle as O


def _herm(n, seed):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    return (X + X.conj().T) / 2, rng.standard_normal(n) + 1j * rng.standard_normal(n)


def test_tridiagonal_moments_equal_krylov_moments():
    """m steps reproduce the moments v^H H^p v / |v|^2 for p <= 2m - 1 exactly
    (Gauss quadrature of the recurrence): a dropped term, a wrong sign or a
    wrong index in the recurrence breaks the higher ones."""
    H, v = _herm(40, 1)
    m = 6
    a, b = O.lanczos(H, v, m)
    T = np.diag(a) + np.diag(b[:-1], 1) + np.diag(b[:-1], -1)
    vh = v / np.linalg.norm(v)
    x = vh.copy()
    e = np.zeros(m)
    e[0] = 1.0
    y = e.copy()
    for p in range(2 * m):
        mk = np.vdot(vh, x).real
        mt = y[0]
        assert abs(mk - mt) <= 1e-11 * max(abs(mk), 1.0) * 4.0 ** p, p
        x = H @ x
        y = T @ y


def test_full_recurrence_gives_exact_resolvent():
    """With m = n the continued fraction is v^H (z - H)^-1 v / |v|^2, the
    spectral sum over the eigenpairs (Eq. resolvent)."""
    H, v = _herm(12, 2)
    a, b = O.lanczos(H, v, 12)
    E, U = np.linalg.eigh(H)
    vh = v / np.linalg.norm(v)
    w = np.abs(U.conj().T @ vh) ** 2
    z = np.linspace(-5, 5, 41) + 0.3j
    exact = np.sum(w[None, :] / (z[:, None] - E[None, :]), axis=1)
    got = O.continued_fraction(a, b, z)
    assert np.abs(got - exact).max() <= 1e-10 * np.abs(exact).max()


def test_haydock_spectrum_converges_to_eigenpair_spectrum():
    """The tiny BSE case: the recurrence from conj(d) against the spectrum of
    the eigenpairs (the oracle's definition).  The broadened spectrum
    converges with the number of steps; past 1.5 N_S steps it agrees to
    rounding (without reorthogonalisation the recurrence keeps going after
    the Krylov space is exhausted, and the extra steps only add copies of
    converged eigenvalues with the right total weight); 24 steps are still
    visibly truncated."""
    s = B.make_config(0)
    H = O.build_H(s) / O.HARTREE_EV
    E, A = np.linalg.eigh(H)
    d = O.transition_dipoles(s, [1.0, 0.0, 0.0])
    pref = 8 * np.pi / (s.nk * s.omega_cell)
    w = (np.linspace(0.0, 10.0, 501) / O.HARTREE_EV, 0.1 / O.HARTREE_EV)
    ref = O.spectrum(E, A, d, pref, w)
    full = O.haydock_spectrum(H, d, pref, w, 2 * s.ns)
    assert np.abs(full - ref).max() <= 1e-12 * ref.max()
    short = O.haydock_spectrum(H, d, pref, w, 24)
    err = np.abs(short - ref).max()
    assert 1e-4 * ref.max() <= err <= 3e-2 * ref.max()
