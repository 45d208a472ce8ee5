"""The synthetic inputs have the structure the paper's quantities have."""
import numpy as np
import pytest

import bse_synth as B


@pytest.mark.parametrize("kw", [dict(kmesh=(2, 2, 2)), dict(kmesh=(3, 2, 1)), dict(kmesh=(4, 1, 1))])
def test_W_hermitian_positive_and_time_reversal(kw):
    s = B.make_system(B.cell_fcc(8.0), (8, 8, 8), kw["kmesh"], 1, 1, 2.0, seed=3)
    n = np.array(s.kmesh)
    for iq in range(s.nk):
        g = s.ng[iq]
        Wq = s.W[iq, :g, :g]
        assert np.abs(Wq - Wq.conj().T).max() < 1e-14
        assert np.linalg.eigvalsh(Wq).min() > -1e-12
        # Sec. III.A with T = 1: W_{G,G'}(q) = conj(W_{-G-G0,-G'-G0}(qbar))
        iv = B.ktriplet(s.kmesh, iq)
        qb = (-iv) % n
        t = (-iv - qb) // n
        iqb = B.kindex(s.kmesh, qb)
        lut = {tuple(m): i for i, m in enumerate(s.gvec[iqb, : s.ng[iqb]])}
        perm = np.array([lut[tuple(t - m)] for m in s.gvec[iq, :g]])
        assert np.abs(Wq - np.conj(s.W[iqb][np.ix_(perm, perm)])).max() < 1e-14


def test_wave_functions_orthonormal_and_energies_in_range():
    s = B.make_config(0)
    for k in range(s.nk):
        ov = s.u[k].conj() @ s.u[k].T
        assert np.abs(ov - np.eye(s.nb)).max() < 1e-13
    assert np.all((s.eps[:, : s.nv] >= -3) & (s.eps[:, : s.nv] <= 0))
    assert np.all((s.eps[:, s.nv:] >= 1) & (s.eps[:, s.nv:] <= 4))


def test_head_wings_and_exchange_kernel():
    s = B.make_config(0)
    assert s.W[0, 0, 0] == pytest.approx(4 * np.pi * 0.1 / s.omega_cell)
    assert np.all(s.W[0, 0, 1:] == 0) and np.all(s.W[0, 1:, 0] == 0)
    b = B.reciprocal(s.cell)
    G = s.gvec[0, 1: s.ng[0]] @ b
    assert np.allclose(s.vx[1: s.ng[0]], 4 * np.pi / np.sum(G * G, axis=1), rtol=1e-14)
    assert s.vx[0] == 0


def test_generation_is_deterministic():
    a = B.make_config(0)
    b = B.make_config(0)
    assert a.digest() == b.digest()
    c = B.make_config(0, seed=99)
    assert c.digest() != a.digest()


def test_slab_coulomb_truncation():
    p = np.array([[0.0, 0.0, 2 * np.pi / 30.0 * 2], [0.3, 0.0, 0.0]])
    v = B.coulomb(p, "slab", 30.0)
    assert abs(v[0]) < 1e-14  # even m3 at zero in-plane momentum
    assert v[1] == pytest.approx(4 * np.pi / 0.09 * (1 - np.exp(-0.3 * 15.0)))
