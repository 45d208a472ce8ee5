"""Pins of the screened interaction at every q unfolded from the irreducible q
points (Sec. III.A: q = T q_IBZ + G0, or -T q_IBZ + G0 with time reversal),
of the generator's irreducible points and maps, and of the oracle's
unfolding.  CPU only."""
import dataclasses

import numpy as np
import pytest

import bse_synth as B
import oracle as O


def _cart(sys, q, g):
    """Cartesian q + G (bohr^-1) of entry g of the sphere of q."""
    b = B.reciprocal(sys.cell)
    return B.q_vector(sys.cell, sys.kmesh, q) + sys.gvec[q, g] @ b


@pytest.mark.parametrize("cell,m,proper,want", [
    ("fcc", 4, False, 8), ("fcc", 8, False, 29), ("fcc", 8, True, 29),
    ("sc", 4, False, 10), ("sc", 8, True, 35)])
def test_irreducible_point_counts(cell, m, proper, want):
    """Gamma-centred m^3 meshes: 8 and 29 irreducible points for fcc at m = 4
    and 8; for sc the points 0 <= i3 <= i2 <= i1 <= m/2, C(m/2 + 3, 3) of them.
    The rotations with time reversal give the orbits of the full group."""
    c = B.cell_fcc(10.26) if cell == "fcc" else B.cell_sc(8.0)
    ops, reps, assign = B.irreducible_q(c, (m, m, m), proper)
    assert len(ops) == (24 if proper else 48)
    assert len(reps) == want
    assert all(a is not None for a in assign)


def test_assignments_hold_in_cartesian_coordinates():
    """Every q equals s T q_rep + G0 with T a Cartesian signed permutation of
    the axes (orthogonal, checked on the vectors themselves) and G0 a
    reciprocal-lattice vector."""
    for c, m in ((B.cell_fcc(10.26), 4), (B.cell_sc(8.0), 4), (B.cell_fcc(7.0), 3)):
        ops, reps, assign = B.irreducible_q(c, (m, m, m))
        b = B.reciprocal(c)
        for q, (rep, oi, s, g0) in enumerate(assign):
            R = b.T @ ops[oi] @ np.linalg.inv(b.T)          # Cartesian form of T
            assert np.allclose(R @ R.T, np.eye(3), atol=1e-12)
            assert np.allclose(np.abs(R), np.abs(np.rint(R)), atol=1e-12)
            lhs = B.q_vector(c, (m, m, m), q)
            rhs = s * (R @ B.q_vector(c, (m, m, m), rep)) + np.asarray(g0) @ b
            assert np.allclose(lhs, rhs, atol=1e-12)


def _chi(p):
    """A scalar of the cubic rotations that changes sign under inversion:
    x y z (x^2 - y^2)(y^2 - z^2)(z^2 - x^2)."""
    x, y, z = p[..., 0], p[..., 1], p[..., 2]
    return x * y * z * (x * x - y * y) * (y * y - z * z) * (z * z - x * x)


def _model_W(sys, q, alpha):
    """W_GG'(q) = a(|p|) delta_GG' + b(|p|) b(|p'|) (1 + i alpha (chi(p) - chi(p'))),
    p = q + G: Hermitian, invariant under the cubic rotations, and obeying
    time reversal W(-p, -p') = conj W(p, p'); with alpha != 0 not invariant
    under inversion."""
    ng = int(sys.ng[q])
    p = np.array([_cart(sys, q, g) for g in range(ng)])
    r2 = np.sum(p * p, axis=1)
    a = 4 * np.pi / (r2 + 0.3)
    bb = np.exp(-r2 / 5.0)
    ch = _chi(p)
    out = np.zeros((sys.ng_max, sys.ng_max), dtype=np.complex128)
    out[:ng, :ng] = np.diag(a) + np.outer(bb, bb) * (1 + 1j * alpha * (ch[:, None] - ch[None, :]))
    return out


def _unfold_model(sys, proper, alpha):
    reps, wsrc, wmap = B.point_group_maps(sys, proper)
    W_irr = np.array([_model_W(sys, q, alpha) for q in reps])
    got = O.unfold_W(W_irr, wsrc, wmap, sys.ng)
    want = np.array([_model_W(sys, q, alpha) for q in range(sys.nk)])
    return np.abs(got - want).max() / np.abs(want).max(), wsrc


@pytest.mark.parametrize("make", [lambda: B.make_config(1),
                                  lambda: B.make_system(B.cell_sc(8.0), (16, 16, 16), (4, 4, 4), 1, 1, 4.0, seed=3)],
                         ids=["fcc4", "sc4"])
def test_unfolding_reproduces_a_symmetric_model(make):
    """A model W with the symmetry of the rotations and of time reversal,
    evaluated directly at every q, equals its unfolding from the irreducible
    points: a wrong G0 sign, T in place of T^-1, or a dropped conjugation
    moves the rotated vectors or flips the odd part.  With the inversions in
    the group the same model fails (it lacks that symmetry): the check is not
    blind to the maps."""
    s = make()
    alpha = 1.0 / max(np.abs(_chi(np.array([_cart(s, q, g) for g in range(s.ng[q])]))).max() for q in range(s.nk))
    err, wsrc = _unfold_model(s, True, alpha)
    assert err <= 1e-13
    assert wsrc[:, 1].any() and not wsrc[:, 1].all()  # both relations in use
    err_real, _ = _unfold_model(s, False, 0.0)        # inversion-symmetric model, full group
    assert err_real <= 1e-13
    err_bad, _ = _unfold_model(s, False, alpha)
    assert err_bad > 1e-3


def test_unfolded_W_is_hermitian_time_reversal_symmetric_and_invariant():
    """The generator's symmetrised W, unfolded by the oracle from W_irr:
    Hermitian, W_{t-G,t-G'}(qbar) = conj W_GG'(q), equal to the generator's
    full W, W(q_IBZ) = W_irr, and invariant under every rotation of the group
    (not only the one the maps use)."""
    s0 = B.make_config(1)
    s = B.with_point_group_W(s0, proper=True)
    W = O.unfold_W(s.W_irr, s.wsrc, s.wmap, s.ng)
    assert np.array_equal(W, s.W)
    scale = np.abs(W).max()
    assert max(np.abs(W[q] - W[q].conj().T).max() for q in range(s.nk)) <= 1e-15 * scale
    for q in range(s.nk):
        qb, perm = B.tr_partner(s, q)
        ng = s.ng[q]
        assert np.abs(W[qb][np.ix_(perm[:ng], perm[:ng])] - np.conj(W[q][:ng, :ng])).max() <= 1e-15 * scale
    ops, reps, assign = B.irreducible_q(s.cell, s.kmesh, True)
    for i, q in enumerate(reps):
        assert np.array_equal(W[q], s.W_irr[i])
    n = np.array(s.kmesh)
    worst = 0.0
    for q in range(0, s.nk, 5):
        iq = np.array(B.ktriplet(s.kmesh, q))
        for M in ops:
            tm = M @ iq
            q2 = B.kindex(s.kmesh, tm % n)
            g0 = ((tm % n) - tm) // n
            Mi = np.rint(np.linalg.inv(M)).astype(int)
            pos = {tuple(m): g for g, m in enumerate(s.gvec[q, :s.ng[q]])}
            mp = [pos[tuple(int(x) for x in Mi @ (s.gvec[q2, g] + g0))] for g in range(s.ng[q2])]
            worst = max(worst, np.abs(W[q2][:s.ng[q2], :s.ng[q2]] - W[q][np.ix_(mp, mp)]).max())
    assert worst <= 1e-14 * scale


def test_hamiltonian_with_unfolded_W():
    """The symmetrised W changes H (it is not the generator's W), H stays
    Hermitian, and the oracle's H from its own unfolding equals that from
    the generator's full W."""
    s0 = B.make_system(B.cell_fcc(7.0), (16, 16, 16), (2, 2, 2), 2, 2, 3.0, seed=71)
    s = B.with_point_group_W(s0, proper=True)
    H = O.build_H(dataclasses.replace(s, W=O.unfold_W(s.W_irr, s.wsrc, s.wmap, s.ng)))
    H0 = O.build_H(s0)
    K = np.abs(H - np.diag(np.diag(H))).max()
    assert np.abs(H - H.conj().T).max() <= 1e-12 * K
    assert np.abs(H - O.build_H(s)).max() <= 1e-12 * K
    assert np.abs(H - H0).max() > 1e-3 * K


def test_fold_is_the_adjoint_of_the_unfolding():
    """For random dW at every q and a random change d of the irreducible
    matrices: Re <dW, unfold(d)> = Re <fold(dW), d>, the identity that makes
    fold(dL/dW) the gradient of L with respect to the irreducible matrices.
    A fold that forgets the conjugation of time-reversed images, or reads the
    map the wrong way round, fails it."""
    s = B.with_point_group_W(B.make_system(B.cell_fcc(7.0), (16, 16, 16), (3, 3, 3), 1, 1, 2.0, seed=74),
                             proper=True)
    rng = np.random.default_rng(9)
    nirr, ngm = len(s.W_irr), s.ng_max
    G = rng.standard_normal((s.nk, ngm, ngm)) + 1j * rng.standard_normal((s.nk, ngm, ngm))
    dlt = rng.standard_normal((nirr, ngm, ngm)) + 1j * rng.standard_normal((nirr, ngm, ngm))
    lhs = np.real(np.sum(np.conj(G) * O.unfold_W(dlt, s.wsrc, s.wmap, s.ng)))
    F = O.fold_dW(G, s.wsrc, s.wmap, s.ng, nirr, ngm)
    rhs = np.real(np.sum(np.conj(F) * dlt))
    assert abs(lhs - rhs) <= 1e-10 * abs(lhs)
    assert s.wsrc[:, 1].any()  # time-reversed images take part
    bad = O.fold_dW(G, np.column_stack([s.wsrc[:, 0], 0 * s.wsrc[:, 1]]), s.wmap, s.ng, nirr, ngm)
    assert abs(np.real(np.sum(np.conj(bad) * dlt)) - lhs) > 1e-3 * abs(lhs)
