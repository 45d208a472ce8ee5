"""The Haydock spectrum (Lanczos recurrence on the GPU, no eigenpairs) against
the oracle: its recurrence coefficients, the spectrum of the eigenpairs, and
at the full Si-like size the moments of the recurrence."""
import sys

import numpy as np
import pytest

import bse_synth as B
import oracle as O

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def test_haydock_matches_oracle_recurrence_and_spectrum():
    """24^3 Si-like case (N_S = 576), oracle H and dipoles: the first steps'
    coefficients against the oracle's recurrence (the later ones drift apart
    by rounding, as in any two implementations of the unreorthogonalised
    recurrence), and the converged spectrum (300 steps) against the spectrum
    of the eigenpairs, for three polarisations in one call."""
    import paper_1206_3518_amd as P
    import torch
    s = B.make_config(1)
    H = O.build_H(s)
    qs = ([1.0, 0.0, 0.0], [0.0, 1.0, 0.0], [0.0, 0.6, 0.8])
    d = np.stack([O.transition_dipoles(s, q) for q in qs])
    Hd = torch.from_numpy(H).cuda()
    dd = torch.from_numpy(d).cuda()
    niter = 300
    eps2, coef = P.bse_haydock_spectrum(Hd, dd, s.nk, s.omega_cell, niter, 1001, 0.0, 10.0, 0.1, want_coef=True)
    torch.cuda.synchronize()
    coef = coef.cpu().numpy()
    for p in range(len(qs)):
        a, b = O.lanczos(H, np.conj(d[p]), 20)
        ea = np.abs(coef[p, :20, 0] - a).max() / np.abs(a).max()
        eb = np.abs(coef[p, :20, 1] - b).max() / np.abs(b).max()
        _say(f"polarisation {p}: first 20 coefficients, rel. diff a {ea:.2e} b {eb:.2e}")
        assert ea <= 1e-10 and eb <= 1e-10
    E, A = np.linalg.eigh(H / O.HARTREE_EV)
    pref = 8 * np.pi / (s.nk * s.omega_cell)
    w = (np.linspace(0.0, 10.0, 1001) / O.HARTREE_EV, 0.1 / O.HARTREE_EV)
    ref = np.mean([O.spectrum(E, A, dq, pref, w) for dq in d], axis=0)
    got = eps2.cpu().numpy()
    err = np.abs(got - ref).max() / ref.max()
    _say(f"spectrum: rel. max diff {err:.2e} against the eigenpair spectrum (peak {ref.max():.3e})")
    assert err <= 1e-9


def test_haydock_polarisations_together_equal_one_by_one():
    import paper_1206_3518_amd as P
    import torch
    s = B.make_config(0)
    d = P.DeviceSystem(s)
    H = P.build_H(d)
    dd = P.bse_transition_dipoles(d, ([1.0, 0.0, 0.0], [0.0, 0.0, 1.0]))
    both = P.bse_haydock_spectrum(H, dd, s.nk, s.omega_cell, 64, 201, 0.0, 10.0, 0.1)
    one = [P.bse_haydock_spectrum(H, dd[p], s.nk, s.omega_cell, 64, 201, 0.0, 10.0, 0.1) for p in range(2)]
    torch.cuda.synchronize()
    assert (both - 0.5 * (one[0] + one[1])).abs().max().item() <= 1e-13 * both.abs().max().item()


def test_haydock_full_size_moments_and_eigenpair_spectrum():
    """Si-like 32^3 grid, 8^3 k mesh (N_S = 8192), GPU-built H: the tridiagonal
    of m steps reproduces the moments v^H H^p v for p < 2m (checked up to 7
    against repeated products with H), and 500 steps give the spectrum of the
    eigenpairs (GPU eigensolver) within 1e-6 of its peak."""
    import paper_1206_3518_amd as P
    import torch
    s = B.make_config(2)
    dev = P.DeviceSystem(s)
    H = P.build_H(dev)
    d = P.bse_transition_dipoles(dev, ([1.0, 0.0, 0.0],))
    niter = 500
    eps2, coef = P.bse_haydock_spectrum(H, d, s.nk, s.omega_cell, niter, 1001, 0.0, 10.0, 0.1, want_coef=True)
    torch.cuda.synchronize()
    a = coef[0, :, 0].cpu().numpy()
    b = coef[0, :, 1].cpu().numpy()
    m = 4
    T = np.diag(a[:m]) + np.diag(b[:m - 1], 1) + np.diag(b[:m - 1], -1)
    v = d[0].conj()
    v = v / torch.linalg.vector_norm(v)
    x = v.clone()
    e = np.zeros(m)
    e[0] = 1.0
    y = e.copy()
    scale = max(abs(a[:m]).max(), abs(b[:m]).max())
    for p in range(2 * m):
        mk = torch.vdot(v, x).real.item()
        _say(f"moment {p}: Krylov {mk:.15e}  tridiagonal {y[0]:.15e}")
        assert abs(mk - y[0]) <= 1e-12 * scale ** p * 4 ** p
        x = H @ x
        y = T @ y
    E, A = torch.linalg.eigh(H)
    ref = P.bse_spectrum(E, A, d, s.nk, s.omega_cell, 1001, 0.0, 10.0, 0.1)
    err = (eps2 - ref).abs().max().item() / ref.abs().max().item()
    _say(f"full size: Haydock ({niter} steps) vs eigenpair spectrum rel. max diff {err:.2e}")
    assert err <= 1e-6
