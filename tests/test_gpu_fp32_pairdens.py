"""BSE_FP32_PAIRDENS: the valence-valence and conduction-conduction pair
densities of the mixed-precision modes transformed in FP32.  Checked against
the FP64 build to the mixed-precision bar (max |dH| <= 1e-4 eV and <= 1e-3 of
the largest kernel element, lowest exciton energies within 1e-4 eV)."""
import sys

import numpy as np
import pytest

import bse_synth as B
from bars import fp64_h_bar

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _check(devs, H64, tag):
    import torch
    for i, (d, h) in enumerate(zip(devs, H64)):
        K = h - torch.diag(torch.diag(h))
        kmax = K.abs().max().item()
        dH = (d.H - h).abs().max().item()
        dE = (torch.linalg.eigvalsh(d.H)[:10] - torch.linalg.eigvalsh(h)[:10]).abs().max().item()
        _say(f"  {tag} system {i}: max|dH| {dH:.3e} eV = {dH / kmax:.2e} of max|K|, lowest-10 dE {dE:.2e} eV")
        assert dH <= 1e-4 and dH <= 1e-3 * kmax
        assert dE <= 1e-4


def _run(systems, flags=0, tr_inputs=False):
    import paper_1206_3518_amd as P
    import torch
    devs = [P.DeviceSystem(s) for s in systems]
    ws = P.workspace(max(P.bse_workspace_size(devs, p, f) for p, f in
                         ((P.BSE_FP64, 0), (P.BSE_SPLIT_FP32, P.BSE_FP32_PAIRDENS), (P.BSE_BF16X3, P.BSE_FP32_PAIRDENS))))
    P.bse_build_H(devs, P.BSE_FP64, flags, ws)
    torch.cuda.synchronize()
    H64 = [d.H.clone() for d in devs]
    for prec, name in ((P.BSE_SPLIT_FP32, "split-FP32"), (P.BSE_BF16X3, "BF16x3")):
        for d in devs:
            d.H.fill_(float("nan"))
        P.bse_build_H(devs, prec, flags | P.BSE_FP32_PAIRDENS, ws)
        torch.cuda.synchronize()
        _check(devs, H64, name + " + FP32 densities")


def test_fp32_pairdens_ragged_cubic_batch():
    _run([
        B.make_system(B.cell_sc(10.0), (16, 16, 16), (2, 2, 2), 2, 2, 3.0, seed=41),
        B.make_system(B.cell_fcc(9.0), (16, 16, 16), (3, 1, 1), 1, 3, 2.0, seed=42),
        B.make_system(B.cell_sc(9.5), (16, 16, 16), (2, 2, 1), 3, 1, 4.0, seed=43),
    ])


def test_fp32_pairdens_hbn_rotated_persistent():
    import paper_1206_3518_amd as P
    _run(B.make_hbn_batch(7, nsys=3, ecut=1.5, nv=2, nc=2, meshes=[2, 3, 1]), flags=P.BSE_PERSISTENT)


def test_fp32_pairdens_with_time_reversal():
    import paper_1206_3518_amd as P
    _run([B.make_system(B.cell_sc(10.0), (16, 16, 16), (4, 3, 1), 2, 2, 3.0, seed=86, time_reversal=True)],
         flags=P.BSE_TIME_REVERSAL)


def test_fp32_pairdens_full_size_si():
    """Si-like 32^3 grid, 8^3 k mesh, 4+4 bands (H 8192 x 8192), in the launch
    configuration the benchmark times."""
    _run([B.make_config(2)])


def test_fp32_pairdens_needs_mixed_precision():
    import paper_1206_3518_amd as P
    s = B.make_system(B.cell_sc(10.0), (16, 16, 16), (1, 1, 1), 1, 1, 2.0, seed=1)
    d = P.DeviceSystem(s)
    ws = P.workspace(P.bse_workspace_size([d], P.BSE_FP64, P.BSE_FP32_PAIRDENS))
    with pytest.raises(P.BseError) as e:
        P.bse_build_H([d], P.BSE_FP64, P.BSE_FP32_PAIRDENS, ws)
    assert e.value.code == -1 and "mixed" in str(e.value)


def test_fp32_pairdens_backward():
    """The adjoint with FP32 recomputed densities against the one with FP64
    densities (same split-FP32 dW contraction): within 1e-4 of each output's
    largest entry; FP32 densities need a mixed precision here too."""
    import paper_1206_3518_amd as P
    import torch
    s = B.make_system(B.cell_sc(10.0), (16, 16, 16), (3, 2, 1), 2, 2, 3.0, seed=87)
    d = P.DeviceSystem(s)
    g = torch.Generator().manual_seed(4)
    G = torch.complex(torch.randn(s.ns, s.ns, generator=g, dtype=torch.float64),
                      torch.randn(s.ns, s.ns, generator=g, dtype=torch.float64)).to(d.device)
    ws = P.workspace(P.bse_workspace_size([d], P.BSE_SPLIT_FP32, P.BSE_FP32_PAIRDENS))
    ref = [x.clone() for x in P.bse_build_H_backward(d, G, precision=P.BSE_SPLIT_FP32, ws=ws, want_densities=True)]
    got = P.bse_build_H_backward(d, G, precision=P.BSE_SPLIT_FP32, flags=P.BSE_FP32_PAIRDENS, ws=ws,
                                 want_densities=True)
    torch.cuda.synchronize()
    for name, a, b in zip(("dW", "deps", "dX", "drho_vv", "drho_cc"), got, ref):
        err = (a - b).abs().max().item()
        scale = b.abs().max().item()
        _say(f"  {name}: max diff {err:.3e} (max {scale:.3e})")
        assert err <= 1e-4 * scale, name
    with pytest.raises(P.BseError):
        P.bse_build_H_backward(d, G, precision=P.BSE_FP64, flags=P.BSE_FP32_PAIRDENS, ws=ws)


@pytest.mark.parametrize("case", ["planes_18", "planes_17", "wide_window"])
def test_fp32_pairdens_corner_cases(case):
    """Plane counts that four planes per step do not divide (18, 17), and a
    window of more than 16 kept rows along the first in-plane axis (the two-
    planes-per-step kernel).  The FP32 densities alone (BF16x3 with FP64
    densities as reference) move H by far less than the mixed bar."""
    import paper_1206_3518_amd as P
    import torch
    if case == "planes_18":
        s = B.make_system(B.cell_sc(10.0), (18, 16, 16), (2, 2, 1), 2, 2, 3.0, seed=88)
    elif case == "planes_17":
        s = B.make_system(B.cell_sc(10.0), (17, 16, 16), (3, 1, 1), 2, 1, 3.0, seed=89)
    else:
        s = B.make_system(np.diag([10.0, 20.0, 10.0]), (16, 32, 32), (1, 2, 1), 1, 2, 3.0, seed=90)
    d = P.DeviceSystem(s)
    ws = P.workspace(max(P.bse_workspace_size([d], p, f) for p, f in
                         ((P.BSE_FP64, 0), (P.BSE_SPLIT_FP32, 0), (P.BSE_BF16X3, 0),
                          (P.BSE_SPLIT_FP32, P.BSE_FP32_PAIRDENS), (P.BSE_BF16X3, P.BSE_FP32_PAIRDENS))))
    P.bse_build_H([d], P.BSE_FP64, 0, ws)
    torch.cuda.synchronize()
    h64 = d.H.clone()
    P.bse_build_H([d], P.BSE_BF16X3, 0, ws)
    torch.cuda.synchronize()
    hbf = d.H.clone()
    d.H.fill_(float("nan"))
    P.bse_build_H([d], P.BSE_BF16X3, P.BSE_FP32_PAIRDENS, ws)
    torch.cuda.synchronize()
    kmax = (h64 - torch.diag(torch.diag(h64))).abs().max().item()
    d32 = (d.H - hbf).abs().max().item()
    _say(f"  {case}: FP32 densities move H by {d32:.3e} eV = {d32 / kmax:.2e} of max|K|")
    assert d32 <= 1e-5 * kmax
    _check([d], [h64], case)


def test_mixed_modes_on_bandlimited_wave_functions():
    """Band-limited wave functions (plane waves up to E_cut/4) give a kernel
    ~1000x larger than white noise at the same shapes: the FP64 build against
    the oracle, and every mixed mode against the FP64 build, at the 24^3
    Si-like shape."""
    import paper_1206_3518_amd as P
    import torch
    import oracle as O
    s = B.make_config(1, wf="bandlimited", wf_ecut=1.5)
    d = P.DeviceSystem(s)
    ws = P.workspace(max(P.bse_workspace_size([d], p, f) for p, f in
                         ((P.BSE_FP64, 0), (P.BSE_SPLIT_FP32, 0), (P.BSE_BF16X3, 0),
                          (P.BSE_SPLIT_FP32, P.BSE_FP32_PAIRDENS), (P.BSE_BF16X3, P.BSE_FP32_PAIRDENS))))
    P.bse_build_H([d], P.BSE_FP64, 0, ws)
    torch.cuda.synchronize()
    h64 = d.H.clone()
    ref = O.build_H(s)
    err = np.abs(h64.cpu().numpy() - ref).max()
    kmax = np.abs(ref - np.diag(np.diag(ref))).max()
    _say(f"  band-limited: max|K| {kmax:.3e} eV, FP64 vs oracle {err:.3e} eV")
    assert err <= fp64_h_bar(ref)
    for prec, flags, name in ((P.BSE_SPLIT_FP32, 0, "split-FP32"), (P.BSE_BF16X3, 0, "BF16x3"),
                              (P.BSE_SPLIT_FP32, P.BSE_FP32_PAIRDENS, "split-FP32 + FP32 densities"),
                              (P.BSE_BF16X3, P.BSE_FP32_PAIRDENS, "BF16x3 + FP32 densities")):
        P.bse_build_H([d], prec, flags, ws)
        torch.cuda.synchronize()
        _check([d], [h64], name)
