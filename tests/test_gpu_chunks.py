"""Builds whose k pairs are processed in many chunks (a small per-chunk budget)
against the oracle and against the one-chunk build of the same inputs."""
import sys

import numpy as np
import pytest

import bse_synth as B
import oracle as O
from bars import fp64_h_bar

pytestmark = pytest.mark.gpu

SMALL = 2 << 20  # bytes of per-pair arrays per chunk: tens of chunks at these shapes


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _build(P, devs, prec, flags, budget):
    import torch
    P.bse_set_chunk_budget(budget)
    try:
        ws = P.workspace(P.bse_workspace_size(devs, prec, flags))
        for d in devs:
            d.H.fill_(float("nan"))
        P.bse_build_H(devs, prec, flags, ws)
        torch.cuda.synchronize()
        return [d.H.clone() for d in devs], ws.numel()
    finally:
        P.bse_set_chunk_budget(0)


@pytest.mark.parametrize("prec", ["fp64", "bf16x3"])
def test_many_chunks_equal_one_chunk(prec):
    """H does not depend on the chunking: every output element is summed in
    the same order whichever chunk its pair falls in."""
    import paper_1206_3518_amd as P
    import torch
    systems = [B.make_config(1),  # batches share (N2, N3)
               B.make_system(B.cell_fcc(7.5), (20, 24, 24), (3, 1, 2), 3, 2, 3.0, seed=21)]
    devs = [P.DeviceSystem(s) for s in systems]
    p = P.PRECISIONS[prec]
    one, n1 = _build(P, devs, p, 0, 0)
    many, n2 = _build(P, devs, p, 0, SMALL)
    _say(f"{prec}: workspace {n1 / 1e6:.1f} MB in one chunk, {n2 / 1e6:.1f} MB with a {SMALL >> 20} MB budget")
    assert n2 < n1
    for a, b in zip(one, many):
        assert torch.equal(a, b)
    if prec == "fp64":
        for s, h in zip(systems, many):
            ref = O.build_H(s)
            assert np.abs(h.cpu().numpy() - ref).max() <= fp64_h_bar(ref)


def test_many_chunks_time_reversal_and_persistent():
    """Time-reversal images are gathered inside the chunk of the pair they come
    from; persistent dispatch per chunk."""
    import paper_1206_3518_amd as P
    import torch
    s = B.make_system(B.cell_sc(10.0), (16, 16, 16), (4, 3, 2), 2, 2, 3.0, seed=85, time_reversal=True)
    d = P.DeviceSystem(s)
    ref = O.build_H(s)
    for flags in (P.BSE_TIME_REVERSAL, P.BSE_TIME_REVERSAL | P.BSE_PERSISTENT, P.BSE_PERSISTENT):
        (h,), _ = _build(P, [d], P.BSE_FP64, flags, SMALL // 8)
        err = np.abs(h.cpu().numpy() - ref).max()
        _say(f"flags {flags}: max|dH| vs oracle {err:.3e}")
        assert err <= fp64_h_bar(ref)


def test_many_chunks_backward():
    """The adjoint accumulates dW over the chunks; the density gradients are
    written per pair."""
    import paper_1206_3518_amd as P
    import torch
    s = B.make_system(B.cell_sc(10.0), (16, 16, 16), (3, 2, 2), 2, 2, 3.0, seed=87)
    d = P.DeviceSystem(s)
    g = torch.Generator().manual_seed(4)
    G = torch.complex(torch.randn(s.ns, s.ns, generator=g, dtype=torch.float64),
                      torch.randn(s.ns, s.ns, generator=g, dtype=torch.float64)).to(d.device)
    for prec in ("fp64", "split_fp32"):
        ref = [x.clone() for x in P.bse_build_H_backward(d, G, precision=prec, flags=P.BSE_PROJECT_DW,
                                                         want_densities=True)]
        P.bse_set_chunk_budget(SMALL // 8)
        try:
            got = P.bse_build_H_backward(d, G, precision=prec, flags=P.BSE_PROJECT_DW, want_densities=True)
            torch.cuda.synchronize()
        finally:
            P.bse_set_chunk_budget(0)
        for name, a, b in zip(("dW", "deps", "dX", "drho_vv", "drho_cc"), got, ref):
            err = (a - b).abs().max().item()
            scale = b.abs().max().item()
            _say(f"  {prec} {name}: max diff {err:.3e} (max {scale:.3e})")
            assert err <= (1e-12 if prec == "fp64" else 1e-6) * scale, name
