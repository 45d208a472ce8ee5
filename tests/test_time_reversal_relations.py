"""Time reversal of the inputs and of the pair densities (Sec. III.A: the
pair-density transformation, with T the identity combined with time
reversal), checked on the oracle's densities, each computed from its
definition.  For kbar the mesh point of -k and u_{kbar} = exp(-i K.r)
conj(u_k), the image of the pair (k, k') is (kbar, kbar') or (kbar', kbar):
  kbar <= kbar':  n_{a kbar, b kbar'}(G) = conj(n_{a k, b k'}(G'')), q + G'' = -(qbar + G)
  kbar >  kbar':  n_{a kbar', b kbar}(G) = n_{b k, a k'}(G)
which is what the GPU build relies on under BSE_TIME_REVERSAL."""
import numpy as np
import pytest

import bse_synth as B
import oracle as O


def _system(tr, kmesh=(3, 2, 1)):
    return B.make_system(B.cell_sc(10.0), (16, 16, 16), kmesh, 2, 2, 3.0, seed=77, time_reversal=tr)


def test_generator_obeys_time_reversal():
    s = _system(True, (4, 3, 1))
    for k in range(s.nk):
        kb, K = B.k_partner(s.kmesh, k)
        assert B.k_partner(s.kmesh, kb)[0] == k
        # -k = kbar - K on the mesh
        iv, ivb = B.ktriplet(s.kmesh, k), B.ktriplet(s.kmesh, kb)
        assert np.array_equal(-iv, ivb - K * np.array(s.kmesh))
        if kb != k:
            np.testing.assert_allclose(s.u[kb], B.u_partner(s.u[k], s.grid, K), rtol=0, atol=1e-14)
        np.testing.assert_allclose(s.u[k].conj() @ s.u[k].T, np.eye(s.nv + s.nc), atol=1e-12)
        np.testing.assert_array_equal(s.eps[k], s.eps[kb])


def _relation_errors(s):
    """Largest deviation from the two relations over every upper pair that
    touches no point that is its own partner, and the number of pairs of each
    kind (conjugate, exchanged, own image)."""
    _, rv, rc = O.densities(s)
    up = O.upper_pairs(s.nk)
    index = {p: i for i, p in enumerate(up)}
    kbar = [B.k_partner(s.kmesh, k)[0] for k in range(s.nk)]
    err, counts = 0.0, [0, 0, 0]
    for i, (ka, kb) in enumerate(up):
        x, y = kbar[ka], kbar[kb]
        if x == ka or y == kb:
            continue
        j = index[(min(x, y), max(x, y))]
        if j == i:
            counts[2] += 1
        iq_i, _ = O.fold(s.kmesh, ka, kb)
        iq_j, _ = O.fold(s.kmesh, min(x, y), max(x, y))
        ng = s.ng[iq_j]
        for rho in (rv, rc):
            if x <= y:
                qb, perm = B.tr_partner(s, iq_j)
                assert qb == iq_i and perm.min() >= 0
                want = np.conj(rho[i][:, :, perm])
                counts[0] += 1
            else:
                assert iq_i == iq_j
                want = np.swapaxes(rho[i], 0, 1)[:, :, :ng]
                counts[1] += 1
            err = max(err, float(np.abs(rho[j][:, :, :ng] - want).max()))
    return err, counts


def test_pair_density_images():
    s = _system(True)
    err, counts = _relation_errors(s)
    assert counts[0] > 0 and counts[1] > 0  # both kinds of image occur on this mesh
    assert err <= 1e-13, err


def test_images_fail_without_time_reversal():
    # the same relations do not hold for wave functions drawn independently at k and -k
    err, _ = _relation_errors(_system(False))
    assert err > 1e-3


@pytest.mark.parametrize("tr", [False, True])
def test_reversed_pair_conjugation(tr):
    """Without any symmetry of u: n_{ck,v'k'}(G) = conj(n_{v'k',ck}(G'')),
    G'' = t - G with -q = qbar + t (the sphere map of W), for every ordered
    pair, the diagonal ones included; the GPU's beyond-TDA coupling block
    gathers its (c, v') rows by it.  A plain conjugate on the same G fails."""
    s = _system(tr, (3, 2, 1))
    nv, nc = s.nv, s.nc
    worst, naive = 0.0, 0.0
    for ka in range(s.nk):
        for kb in range(s.nk):
            iq, _ = O.fold(s.kmesh, ka, kb)
            iqr, _ = O.fold(s.kmesh, kb, ka)
            qb, perm = B.tr_partner(s, iq)
            assert qb == iqr and perm.min() >= 0
            ng = s.ng[iq]
            items = [(ka, nv + c, kb, v) for c in range(nc) for v in range(nv)]
            rev = [(kb, v, ka, nv + c) for c in range(nc) for v in range(nv)]
            a = O.pair_density_items(s, items)[:, :ng]
            b = O.pair_density_items(s, rev)
            worst = max(worst, float(np.abs(a - np.conj(b[:, perm[:ng]])).max()))
            naive = max(naive, float(np.abs(a - np.conj(b[:, :ng])).max()))
    assert worst <= 1e-14, worst
    assert naive > 1e-3
