"""Pins of the oracle's gradient with respect to the pair densities: H built
from given densities reproduces build_H; directional derivatives of
L = Re sum conj(Gbar) H(densities) (exact for this real-linear L) match the
gradient for a Hermitian and a general Gbar; Euler identities of the bilinear
exchange and direct terms.  CPU only."""
import dataclasses

import numpy as np
import pytest

import bse_synth as B
import oracle as O


@pytest.fixture(scope="module")
def case():
    s = B.make_system(B.cell_fcc(7.0), (8, 8, 8), (2, 2, 1), 2, 2, 2.0, seed=31)
    X, rv, rc = O.densities(s)
    return s, X, rv, rc


def _gbars(s):
    H = O.build_H(s)
    _, x = np.linalg.eigh(H)
    rng = np.random.default_rng(4)
    return [np.outer(x[:, 0], np.conj(x[:, 0])),
            rng.normal(size=H.shape) + 1j * rng.normal(size=H.shape)]


def test_H_from_densities_is_build_H(case):
    s, X, rv, rc = case
    H = O.build_H(s)
    assert np.abs(O.H_from_densities(s, X, rv, rc) - H).max() <= 1e-13 * np.abs(H).max()


@pytest.mark.parametrize("which", ["X", "rv", "rc"])
def test_directional_derivatives(case, which):
    s, X, rv, rc = case
    rng = np.random.default_rng(5)
    for G in _gbars(s):
        grads = dict(zip(("X", "rv", "rc"), O.adjoint_densities(s, G, X, rv, rc)))
        base = {"X": X, "rv": rv, "rc": rc}
        arr = base[which]
        d = (rng.normal(size=arr.shape) + 1j * rng.normal(size=arr.shape)) * (np.abs(arr) > 0)

        def L(t):
            args = dict(base)
            args[which] = arr + t * d
            return np.real(np.sum(np.conj(G) * O.H_from_densities(s, args["X"], args["rv"], args["rc"])))

        h = 1e-2  # L is real-linear in each density set: the difference quotient is exact
        fd = (L(h) - L(-h)) / (2 * h)
        ad = np.real(np.sum(np.conj(grads[which]) * d))
        assert abs(fd - ad) <= 1e-9 * max(abs(ad), 1e-12), (which, fd, ad)


def test_euler_identities(case):
    s, X, rv, rc = case
    Hx = O.H_from_densities(dataclasses.replace(s, W=np.zeros_like(s.W), eps=np.zeros_like(s.eps)), X, rv, rc)
    vz = np.zeros_like(s.vx)
    Hd = O.H_from_densities(dataclasses.replace(s, vx=vz, eps=np.zeros_like(s.eps)), X, rv, rc)
    for G in _gbars(s):
        dX, drv, drc = O.adjoint_densities(s, G, X, rv, rc)
        Lx = np.real(np.sum(np.conj(G) * Hx))
        Ld = np.real(np.sum(np.conj(G) * Hd))
        assert abs(np.real(np.sum(np.conj(dX) * X)) - 2 * Lx) <= 1e-12 * abs(Lx) + 1e-15
        assert abs(np.real(np.sum(np.conj(drv) * rv)) - Ld) <= 1e-12 * abs(Ld) + 1e-15
        assert abs(np.real(np.sum(np.conj(drc) * rc)) - Ld) <= 1e-12 * abs(Ld) + 1e-15
