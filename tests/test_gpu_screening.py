"""Static RPA screening on the GPU (bse_screening) against the oracle's W, and
the Hamiltonian built from it against the oracle's H with the oracle's W."""
import dataclasses
import sys

import numpy as np
import pytest

import bse_synth as B
import oracle as O
from bars import fp64_h_bar

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _bse_part(s, W, nc_bse):
    """The BSE system of the first nc_bse empty bands with the given W."""
    nb = s.nv + nc_bse
    return dataclasses.replace(s, nc=nc_bse, u=np.ascontiguousarray(s.u[:, :nb]),
                               eps=np.ascontiguousarray(s.eps[:, :nb]), W=np.ascontiguousarray(W))


def _case(name):
    if name == "cubic":  # 16^3, 2 x 2 x 2 k, 2 occupied + 6 empty bands
        return B.make_system(B.cell_sc(10.0), (16, 16, 16), (2, 2, 2), 2, 6, 2.0, seed=61)
    if name == "fcc_odd":  # odd mesh, m0 = -1 on two axes
        return B.make_system(B.cell_fcc(7.5), (12, 12, 16), (3, 1, 2), 3, 5, 2.5, seed=62)
    if name == "hbn":  # long last axis: rotated pair-density frame, truncated Coulomb
        return B.make_system(B.cell_hex(B.A_HBN, B.C_HBN), (24, 24, 96), (3, 3, 1), 2, 4, 1.5,
                             coulomb_kind="slab", slab_L=B.C_HBN, seed=63)
    raise ValueError(name)


@pytest.mark.parametrize("name", ["cubic", "fcc_odd", "hbn"])
def test_screening_matches_oracle(name):
    import paper_1206_3518_amd as P
    import torch
    s = _case(name)
    vq = B.coulomb_table(s)
    head = s.head
    d = P.DeviceSystem(s)
    W = P.bse_screening(d, vq, head)
    torch.cuda.synchronize()
    Wg = W.cpu().numpy()
    ref = O.screened_interaction(s, vq, head)
    err = np.abs(Wg - ref).max()
    scale = np.abs(ref).max()
    _say(f"{name}: ng_max {s.ng_max}, nv {s.nv} nc {s.nc}: max|dW| {err:.3e} (max|W| {scale:.3e})")
    assert err <= 1e-11 * scale
    # the H built from the GPU's W against the oracle's H with the oracle's W
    sb = _bse_part(s, Wg, 2)
    db = P.DeviceSystem(sb)
    H = P.build_H(db).cpu().numpy()
    Href = O.build_H(_bse_part(s, ref, 2))
    dh = np.abs(H - Href).max()
    _say(f"{name}: H from the screened W, max|dH| vs oracle {dh:.3e} eV")
    assert dh <= fp64_h_bar(Href) + 1e-11 * np.abs(Href - np.diag(np.diag(Href))).max()


def test_screening_in_chunks_and_validated_build():
    """Chunks of q (small budget) give the same W; the W passes the build's
    Hermiticity and time-reversal scan (BSE_VALIDATE) for time-reversal
    symmetric wave functions."""
    import paper_1206_3518_amd as P
    import torch
    s = B.make_system(B.cell_sc(10.0), (16, 16, 16), (4, 3, 1), 2, 4, 2.0, seed=64, time_reversal=True)
    vq = B.coulomb_table(s)
    d = P.DeviceSystem(s)
    W1 = P.bse_screening(d, vq, s.head)
    P.bse_set_chunk_budget(1 << 20)
    try:
        W2 = P.bse_screening(d, vq, s.head)
        torch.cuda.synchronize()
    finally:
        P.bse_set_chunk_budget(0)
    assert torch.equal(W1, W2)
    sb = _bse_part(s, W1.cpu().numpy(), 3)
    db = P.DeviceSystem(sb)
    P.bse_build_H([db], P.BSE_FP64, P.BSE_VALIDATE)
    torch.cuda.synchronize()
