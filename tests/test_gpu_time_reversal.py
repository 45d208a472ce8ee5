"""BSE_TIME_REVERSAL: pair densities of time-reversal images gathered instead
of transformed.  The GPU build under the flag is compared with the oracle
(which computes every density from its definition) and with the GPU build
without the flag, on inputs that obey time reversal: cubic meshes with and
without time-reversal-invariant points, a ragged batch, and h-BN-like cells
on the rotated 24 x 24 x 96 frame."""
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


def _cubic_tr():
    return [
        B.make_system(B.cell_sc(10.0), (16, 16, 16), (3, 2, 1), 2, 2, 3.0, seed=81, time_reversal=True),
        B.make_system(B.cell_fcc(9.0), (16, 16, 16), (2, 2, 2), 1, 3, 2.0, seed=82, time_reversal=True),
        B.make_system(B.cell_sc(9.5), (16, 16, 16), (4, 3, 1), 3, 1, 3.0, seed=83, time_reversal=True),
    ]


@pytest.mark.parametrize("persist", [False, True])
def test_tr_build_matches_oracle_and_full_build(persist):
    import paper_1206_3518_amd as P
    import torch
    systems = _cubic_tr()
    devs = [P.DeviceSystem(s) for s in systems]
    ws = P.workspace(P.bse_workspace_size(devs))
    base = P.BSE_PERSISTENT if persist else 0
    P.bse_build_H(devs, P.BSE_FP64, base, ws)
    torch.cuda.synchronize()
    full = [d.H.clone() for d in devs]
    for d in devs:
        d.H.fill_(float("nan"))
    P.bse_build_H(devs, P.BSE_FP64, base | P.BSE_TIME_REVERSAL | P.BSE_VALIDATE, ws)
    torch.cuda.synchronize()
    for i, (d, s, h) in enumerate(zip(devs, systems, full)):
        ref = O.build_H(s)
        scale = max(np.abs(ref).max(), 1.0)
        err = np.abs(d.H.cpu().numpy() - ref).max()
        dfull = (d.H - h).abs().max().item()
        _say(f"  system {i} kmesh {s.kmesh}: max|dH| vs oracle {err:.3e}, vs full build {dfull:.3e}")
        assert err <= 1e-12 * scale
        assert dfull <= 1e-13 * scale


def test_tr_hbn_rotated_frame_and_split_fp32():
    import paper_1206_3518_amd as P
    import torch
    systems = B.make_hbn_batch(7, nsys=3, ecut=1.5, nv=2, nc=2, meshes=[2, 3, 1])
    systems = [B.make_system(B.cell_hex(B.A_HBN, B.C_HBN), s.grid, s.kmesh, s.nv, s.nc, s.ecut,
                             coulomb_kind="slab", slab_L=B.C_HBN, seed=90 + i, time_reversal=True)
               for i, s in enumerate(systems)]
    devs = [P.DeviceSystem(s) for s in systems]
    ws = P.workspace(max(P.bse_workspace_size(devs, p) for p in (P.BSE_FP64, P.BSE_SPLIT_FP32)))
    for prec, tol in ((P.BSE_FP64, 1e-12), (P.BSE_SPLIT_FP32, None)):
        P.bse_build_H(devs, prec, 0, ws)
        torch.cuda.synchronize()
        full = [d.H.clone() for d in devs]
        P.bse_build_H(devs, prec, P.BSE_TIME_REVERSAL, ws)
        torch.cuda.synchronize()
        for i, (d, s, h) in enumerate(zip(devs, systems, full)):
            dfull = (d.H - h).abs().max().item()
            K = h - torch.diag(torch.diag(h))
            _say(f"  h-BN {i} precision {prec}: max|dH| vs full build {dfull:.3e} (kernel {K.abs().max().item():.3e})")
            if tol is not None:
                ref = O.build_H(s)
                err = np.abs(d.H.cpu().numpy() - ref).max()
                assert err <= tol * max(np.abs(ref).max(), 1.0)
                assert dfull <= 1e-13 * max(np.abs(ref).max(), 1.0)
            else:
                assert dfull <= 1e-4 and dfull <= 1e-3 * K.abs().max().item()


def test_tr_validate_rejects_inputs_without_time_reversal():
    import paper_1206_3518_amd as P
    import torch
    s = B.make_system(B.cell_sc(10.0), (16, 16, 16), (3, 1, 1), 2, 2, 3.0, seed=84)  # u drawn independently
    d = P.DeviceSystem(s)
    ws = P.workspace(P.bse_workspace_size([d]))
    with pytest.raises(P.BseError) as e:
        P.bse_build_H([d], P.BSE_FP64, P.BSE_TIME_REVERSAL | P.BSE_VALIDATE, ws)
    assert e.value.code == -8 and "time reversal" in str(e.value)
    # the same inputs build without the flag
    P.bse_build_H([d], P.BSE_FP64, P.BSE_VALIDATE, ws)
    torch.cuda.synchronize()
    ref = O.build_H(s)
    assert np.abs(d.H.cpu().numpy() - ref).max() <= fp64_h_bar(ref)


def test_tr_full_size_si():
    """Si-like 32^3 grid, 8^3 k mesh, 4+4 bands (H 8192 x 8192) with
    time-reversal-symmetric inputs, in the launch configuration the benchmark
    times: the whole H against the general build, and oracle blocks at k pairs
    whose densities were gathered (and at their images, which were computed)."""
    import paper_1206_3518_amd as P
    import torch
    s = B.make_config(2, time_reversal=True)
    d = P.DeviceSystem(s)
    ws = P.workspace(P.bse_workspace_size([d]))
    _say(f"full size, time reversal: NS = {s.ns}")
    P.bse_build_H([d], P.BSE_FP64, 0, ws)
    torch.cuda.synchronize()
    Hg = d.H.clone()
    d.H.fill_(float("nan"))
    P.bse_build_H([d], P.BSE_FP64, P.BSE_TIME_REVERSAL, ws)
    torch.cuda.synchronize()
    scale = Hg.abs().max().item()
    diff = (d.H - Hg).abs().max().item()
    _say(f"  max|dH| vs general build {diff:.3e} (max|H| {scale:.3e})")
    assert diff <= 1e-13 * scale
    nk, nt = s.nk, s.nv * s.nc
    kbar = [B.k_partner(s.kmesh, k)[0] for k in range(nk)]
    rng = np.random.default_rng(11)
    blocks = []
    for ka, kb in [(1, 2), (3, 200), (77, 77)] + [tuple(sorted(int(x) for x in rng.integers(0, nk, 2)))
                                                  for _ in range(3)]:
        x, y = kbar[ka], kbar[kb]
        blocks += [(ka, kb), (min(x, y), max(x, y))]
    ref = O.build_blocks(s, blocks)
    kmax = max(np.abs(r - np.diag(np.diag(r))).max() for r in ref)
    for (ka, kb), r in zip(blocks, ref):
        g = d.H[ka * nt:(ka + 1) * nt, kb * nt:(kb + 1) * nt].cpu().numpy()
        assert np.abs(g - r).max() <= 1e-10 * kmax + 2.0 ** -50 * np.abs(r).max(), (ka, kb)


def test_tr_backward_matches_general_backward():
    """The adjoint recomputes the pair densities; under BSE_TIME_REVERSAL the
    image pairs are gathered there too, with the same gradients."""
    import paper_1206_3518_amd as P
    import torch
    s = B.make_system(B.cell_sc(10.0), (16, 16, 16), (4, 3, 1), 2, 2, 3.0, seed=85, time_reversal=True)
    d = P.DeviceSystem(s)
    g = torch.Generator().manual_seed(3)
    G = torch.complex(torch.randn(s.ns, s.ns, generator=g, dtype=torch.float64),
                      torch.randn(s.ns, s.ns, generator=g, dtype=torch.float64)).to(d.device)
    ws = P.workspace(P.bse_workspace_size([d], P.BSE_FP64, P.BSE_PROJECT_DW))
    for flags in (0, P.BSE_PROJECT_DW):
        ref = P.bse_build_H_backward(d, G, flags=flags, ws=ws, want_densities=True)
        ref = [x.clone() for x in ref]
        got = P.bse_build_H_backward(d, G, flags=flags | P.BSE_TIME_REVERSAL, ws=ws, want_densities=True)
        torch.cuda.synchronize()
        for name, a, b in zip(("dW", "deps", "dX", "drho_vv", "drho_cc"), got, ref):
            err = (a - b).abs().max().item()
            _say(f"  flags {flags}: {name} max diff {err:.3e} (max {b.abs().max().item():.3e})")
            assert err <= 1e-12 * max(b.abs().max().item(), 1e-30), name
