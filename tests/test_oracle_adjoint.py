"""Pins of the oracle adjoint: sum rules, the Euler identity of the linear W
dependence, and central finite differences along perturbations that keep W
Hermitian and time-reversal symmetric.  CPU only."""
import dataclasses

import numpy as np
import pytest

import bse_synth as B
import oracle as O


def _sys():
    return B.make_system(B.cell_fcc(7.0), (8, 8, 8), (2, 2, 1), 2, 2, 2.0, seed=31)


def _lowest(H):
    e, x = np.linalg.eigh(H)
    return e[0], x[:, 0], e[1] - e[0]


def test_hellmann_feynman_sum_rules():
    s = _sys()
    H = O.build_H(s)
    e0, x0, gap = _lowest(H)
    G = np.outer(x0, np.conj(x0))
    _, deps = O.adjoint(s, G)
    assert abs(deps[:, s.nv:].sum() - 1.0) < 1e-12
    assert abs(deps[:, : s.nv].sum() + 1.0) < 1e-12


def test_euler_identity_of_direct_term():
    s = _sys()
    H = O.build_H(s)
    H0 = O.build_H(dataclasses.replace(s, W=np.zeros_like(s.W)))
    e0, x0, _ = _lowest(H)
    G = np.outer(x0, np.conj(x0))
    dW, _ = O.adjoint(s, G)
    lhs = np.real(np.sum(np.conj(dW) * s.W))
    rhs = np.real(np.conj(x0) @ (H - H0) @ x0)
    assert abs(lhs - rhs) <= 1e-12 * max(abs(rhs), 1e-300)
    assert abs(rhs) > 1e-8


def test_finite_differences_along_symmetric_directions():
    s = _sys()
    H = O.build_H(s)
    e0, x0, gap = _lowest(H)
    assert gap > 1e-6
    G = np.outer(x0, np.conj(x0))
    dW, deps = O.adjoint(s, G)
    rng = np.random.default_rng(2)
    h = 1e-2  # H is linear in W and eps, so a large step is accurate
    for trial in range(6):
        iq = int(rng.integers(0, s.nk))
        g, gp = (int(x) for x in rng.integers(0, s.ng[iq], 2))
        z = (1.0 if trial % 2 == 0 else 1j) * s.W[iq, g, g].real
        D = O.orbit_direction(s, iq, g, gp, z)
        ad = np.real(np.sum(np.conj(dW) * D))
        ep = np.linalg.eigvalsh(O.build_H(dataclasses.replace(s, W=s.W + h * D)))[0]
        em = np.linalg.eigvalsh(O.build_H(dataclasses.replace(s, W=s.W - h * D)))[0]
        fd = (ep - em) / (2 * h)
        assert abs(fd - ad) <= 1e-6 * max(abs(ad), 1e-3 * np.abs(dW).max() * abs(z)), (trial, fd, ad)
    h = 1e-5  # E0 is not linear in eps: a step small against the gap
    for trial in range(4):
        k, b = int(rng.integers(0, s.nk)), int(rng.integers(0, s.nb))
        e = s.eps.copy()
        e[k, b] += h
        ep = np.linalg.eigvalsh(O.build_H(dataclasses.replace(s, eps=e)))[0]
        e[k, b] -= 2 * h
        em = np.linalg.eigvalsh(O.build_H(dataclasses.replace(s, eps=e)))[0]
        fd = (ep - em) / (2 * h)
        noise = 1e-14 * abs(e0) / h  # rounding of the eigenvalues through the step
        assert abs(fd - deps[k, b]) <= 1e-6 * abs(deps[k, b]) + noise


def test_restricted_q_matches_full():
    s = _sys()
    H = O.build_H(s)
    _, x0, _ = _lowest(H)
    G = np.outer(x0, np.conj(x0))
    dW, _ = O.adjoint(s, G)
    dW2, _ = O.adjoint(s, G, qs={1, 2})
    assert np.abs(dW2[1] - dW[1]).max() < 1e-15 and np.abs(dW2[2] - dW[2]).max() < 1e-15
    assert np.abs(dW2[0]).max() == 0.0


@pytest.mark.parametrize("kmesh,qexc", [((3, 1, 1), 1), ((2, 2, 1), 3)])
def test_adjoint_at_finite_exciton_momentum(kmesh, qexc):
    """At exciton momentum Q the map (W, eps) -> H of ``build_H_exciton`` is
    affine, so for any Gbar and any changes dW0, de0 of W and eps:
    Re <Gbar, H(W + dW0, eps + de0) - H(W, eps)> = Re <dL/dW, dW0> + <dL/de, de0>
    up to rounding.  The conduction energies enter at k + Q and the
    conduction densities pair (k + Q, k' + Q): an adjoint that credits the
    energies at k, or contracts the unshifted densities, fails it (the last
    two checks plant those mistakes)."""
    s = B.with_exciton_momentum(B.make_system(B.cell_fcc(7.0), (8, 8, 8), kmesh, 2, 2, 2.0, seed=33), qexc)
    rng = np.random.default_rng(8)
    Gbar = rng.standard_normal((s.ns, s.ns)) + 1j * rng.standard_normal((s.ns, s.ns))
    dW0 = np.zeros_like(s.W)
    for q in range(s.nk):
        ng = s.ng[q]
        dW0[q, :ng, :ng] = rng.standard_normal((ng, ng)) + 1j * rng.standard_normal((ng, ng))
    de0 = rng.standard_normal(s.eps.shape)
    H = O.build_H_exciton(s)
    H1 = O.build_H_exciton(dataclasses.replace(s, W=s.W + dW0, eps=s.eps + de0))
    lhs = np.real(np.sum(np.conj(Gbar) * (H1 - H)))
    dW, deps = O.adjoint(s, Gbar)
    rhs = np.real(np.sum(np.conj(dW) * dW0)) + np.sum(deps * de0)
    scale = np.abs(Gbar).sum() * np.abs(H1 - H).max()
    assert abs(lhs - rhs) <= 1e-12 * scale
    # the conduction energies credited at k instead of k + Q
    bad = deps.copy()
    dg = np.real(np.diag(Gbar)).reshape(s.nk, s.nv, s.nc)
    bad[:, s.nv:] = dg.sum(axis=1)
    assert abs(np.real(np.sum(np.conj(dW) * dW0)) + np.sum(bad * de0) - lhs) > 1e-6 * scale
    # the conduction densities of (k, k') instead of (k + Q, k' + Q)
    dWu, _ = O.adjoint(dataclasses.replace(s, qexc=0), Gbar)
    assert abs(np.real(np.sum(np.conj(dWu) * dW0)) + np.sum(deps * de0) - lhs) > 1e-6 * scale
