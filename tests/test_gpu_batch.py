"""Batches of independent systems of uneven size built by one launch per stage
(static and persistent work-queue dispatch), against single-system builds and
the CPU oracle."""
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


def _ragged_cubic():
    # same 16^3 grid, different cells, k meshes, band counts and spheres
    return [
        B.make_system(B.cell_sc(10.0), (16, 16, 16), (2, 2, 2), 2, 2, 3.0, seed=41),
        B.make_system(B.cell_fcc(9.0), (16, 16, 16), (3, 1, 1), 1, 3, 2.0, seed=42),
        B.make_system(B.cell_sc(9.5), (16, 16, 16), (2, 2, 1), 3, 1, 4.0, seed=43),
    ]


def _hbn_small():
    # h-BN-like cells on the 24 x 24 x 96 grid with the slab Coulomb kernel;
    # small spheres and meshes so that the oracle finishes in seconds
    return B.make_hbn_batch(7, nsys=3, ecut=1.5, nv=2, nc=2, meshes=[2, 3, 1])


@pytest.mark.parametrize("persist", [False, True])
def test_batch_equals_single_builds_and_oracle(persist):
    import paper_1206_3518_amd as P
    import torch
    systems = _ragged_cubic()
    devs = [P.DeviceSystem(s) for s in systems]
    _say(f"batch of {len(devs)} (persistent={persist}): ns = {[s.ns for s in systems]}")
    single = []
    for d in devs:
        P.bse_build_H([d], P.BSE_FP64, 0)
        single.append(d.H.clone())
    flags = P.BSE_PERSISTENT if persist else 0
    for d in devs:
        d.H.zero_()
    P.bse_build_H(devs, P.BSE_FP64, flags)
    torch.cuda.synchronize()
    for i, (d, s, h1) in enumerate(zip(devs, systems, single)):
        assert torch.equal(d.H, h1), f"system {i}: batch differs from its single build"
        ref = O.build_H(s)
        err = np.abs(d.H.cpu().numpy() - ref).max()
        _say(f"  system {i}: max|dH| vs oracle = {err:.3e}")
        assert err <= fp64_h_bar(ref)


def test_hbn_batch_fp64_and_split_fp32():
    import paper_1206_3518_amd as P
    import torch
    systems = _hbn_small()
    devs = [P.DeviceSystem(s) for s in systems]
    _say(f"h-BN batch: grid {systems[0].grid}, meshes {[s.kmesh for s in systems]}, "
         f"ng_max {[s.ng_max for s in systems]}")
    ws = P.workspace(max(P.bse_workspace_size(devs, p) for p in (P.BSE_FP64, P.BSE_SPLIT_FP32)))
    P.bse_build_H(devs, P.BSE_FP64, P.BSE_PERSISTENT, ws)
    torch.cuda.synchronize()
    H64 = [d.H.clone() for d in devs]
    for i, (s, h) in enumerate(zip(systems, H64)):
        ref = O.build_H(s)
        err = np.abs(h.cpu().numpy() - ref).max()
        _say(f"  system {i}: FP64 max|dH| vs oracle = {err:.3e}")
        assert err <= fp64_h_bar(ref)
    P.bse_build_H(devs, P.BSE_SPLIT_FP32, P.BSE_PERSISTENT, ws)
    torch.cuda.synchronize()
    for i, (d, h) in enumerate(zip(devs, H64)):
        K = h - torch.diag(torch.diag(h))
        dH = (d.H - h).abs().max().item()
        _say(f"  system {i}: split-FP32 max|dH| = {dH:.3e} eV (kernel {K.abs().max().item():.3e})")
        assert dH <= 1e-4 and dH <= 1e-3 * K.abs().max().item()
        e = torch.linalg.eigvalsh(d.H)[:10]
        e64 = torch.linalg.eigvalsh(h)[:10]
        assert (e - e64).abs().max().item() <= 1e-4


def test_batch_rejects_mixed_grids_and_unknown_flags():
    import paper_1206_3518_amd as P
    a = B.make_system(B.cell_sc(10.0), (16, 16, 16), (1, 1, 1), 1, 1, 2.0, seed=1)
    b = B.make_system(B.cell_sc(10.0), (16, 12, 12), (1, 1, 1), 1, 1, 2.0, seed=2)
    da, db = P.DeviceSystem(a), P.DeviceSystem(b)
    ws = P.workspace(1 << 20)
    with pytest.raises(P.BseError) as e:
        P.bse_build_H([da, db], P.BSE_FP64, 0, ws)
    assert e.value.code == -2  # BSE_ERR_SHAPE
    with pytest.raises(P.BseError) as e:
        P.bse_build_H([da], P.BSE_FP64, 64, ws)
    assert e.value.code == -1  # BSE_ERR_INVALID_ARG


def test_validate_flag():
    import paper_1206_3518_amd as P
    import torch
    s = B.make_system(B.cell_sc(10.0), (16, 16, 16), (3, 1, 1), 2, 2, 3.0, seed=61)
    d = P.DeviceSystem(s)
    ws = P.workspace(P.bse_workspace_size([d]))
    P.bse_build_H([d], P.BSE_FP64, 0, ws)
    torch.cuda.synchronize()
    ref = d.H.clone()
    d.H.zero_()
    P.bse_build_H([d], P.BSE_FP64, P.BSE_VALIDATE, ws)  # valid inputs: same H
    torch.cuda.synchronize()
    assert torch.equal(d.H, ref)
    # a NaN in the wave functions
    keep = d.u[1, 0, 5].clone()
    d.u[1, 0, 5] = complex(float("nan"), 0.0)
    with pytest.raises(P.BseError) as e:
        P.bse_build_H([d], P.BSE_FP64, P.BSE_VALIDATE, ws)
    assert e.value.code == -6 and "u" in str(e.value)
    d.u[1, 0, 5] = keep
    # W(q) made non-Hermitian in one entry
    W0 = d.W.clone()
    d.W[1, 2, 3] += 1e-3 * d.W.abs().max()
    with pytest.raises(P.BseError) as e:
        P.bse_build_H([d], P.BSE_FP64, P.BSE_VALIDATE, ws)
    assert e.value.code == -5 and "Hermitian" in str(e.value)
    # a Hermitian change at one q that breaks time reversal (on the 3 x 1 x 1
    # mesh q = 1 and q = 2 are each other's partners)
    d.W.copy_(W0)
    z = 1e-3 * d.W.abs().max().item()
    d.W[1, 2, 3] += z
    d.W[1, 3, 2] += z
    with pytest.raises(P.BseError) as e:
        P.bse_build_H([d], P.BSE_FP64, P.BSE_VALIDATE, ws)
    assert e.value.code == -5 and "time reversal" in str(e.value)
    d.W.copy_(W0)
    P.bse_build_H([d], P.BSE_FP64, P.BSE_VALIDATE, ws)
    torch.cuda.synchronize()
    assert torch.equal(d.H, ref)
