"""The h-BN-like batch at its real shape (24 x 24 x 96 grid, 9 Ha, ~779 plane
waves, 4 + 4 bands, k meshes n x n x 1): three members of the 16-system
batch (n = 12, 9, 6, generated exactly as in the whole batch) built together,
against oracle blocks sampled from each, in FP64 and the mixed precisions."""
import sys

import numpy as np
import pytest

import bse_synth as B
import oracle as O

pytestmark = pytest.mark.gpu

MEMBERS = (3, 2, 4)  # n = 12, 9, 6 in the batch of seed 1209


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def batch():
    systems = B.make_hbn_batch(1206 + 3, only=MEMBERS)
    assert [s.kmesh[0] for s in systems] == [12, 9, 6]
    rng = np.random.default_rng(7)
    blocks, refs = [], []
    for s in systems:
        nk = s.nk
        bl = [(0, 0), (0, nk - 1), (nk - 1, 0), (nk // 2, nk // 2 + 1)]
        bl += [tuple(int(x) for x in rng.integers(0, nk, 2)) for _ in range(3)]
        blocks.append(bl)
        refs.append(O.build_blocks(s, bl))
    return systems, blocks, refs


def _blocks_of(h, s, bl):
    nt = s.nv * s.nc
    return [h[a * nt:(a + 1) * nt, b * nt:(b + 1) * nt].cpu().numpy() for a, b in bl]


def test_hbn_real_shape_fp64_against_oracle(batch):
    import paper_1206_3518_amd as P
    import torch
    systems, blocks, refs = batch
    _say(f"h-BN members {MEMBERS}: ng_max {[s.ng_max for s in systems]}, NS {[s.ns for s in systems]}")
    devs = [P.DeviceSystem(s) for s in systems]
    ws = P.workspace(P.bse_workspace_size(devs))
    for flags in (0, P.BSE_PERSISTENT):
        P.bse_build_H(devs, P.BSE_FP64, flags, ws)
        torch.cuda.synchronize()
        for s, d, bl, ref in zip(systems, devs, blocks, refs):
            kmax = max(np.abs(r - np.diag(np.diag(r))).max() for r in ref)
            for (a, b), g, r in zip(bl, _blocks_of(d.H, s, bl), ref):
                err = np.abs(g - r).max()
                assert err <= 1e-10 * kmax + 2.0 ** -50 * np.abs(r).max(), (s.name, a, b, err)
            _say(f"  {s.name} flags {flags}: {len(bl)} blocks within the FP64 bar (max|K| {kmax:.3e} eV)")


@pytest.mark.parametrize("mode", ["split_fp32", "bf16x3", "bf16x3+fp32_pairdens"])
def test_hbn_real_shape_mixed_against_oracle(batch, mode):
    import paper_1206_3518_amd as P
    import torch
    systems, blocks, refs = batch
    devs = [P.DeviceSystem(s) for s in systems]
    prec = P.PRECISIONS[mode.split("+")[0]]
    flags = P.BSE_FP32_PAIRDENS if "fp32" in mode else 0
    ws = P.workspace(P.bse_workspace_size(devs, prec, flags))
    P.bse_build_H(devs, prec, flags, ws)
    torch.cuda.synchronize()
    for s, d, bl, ref in zip(systems, devs, blocks, refs):
        kmax = max(np.abs(r - np.diag(np.diag(r))).max() for r in ref)
        err = max(np.abs(g - r).max() for g, r in zip(_blocks_of(d.H, s, bl), ref))
        _say(f"  {s.name} {mode}: max|dH| {err:.3e} eV = {err / kmax:.2e} of max|K|")
        assert err <= 1e-4 and err <= 1e-3 * kmax
