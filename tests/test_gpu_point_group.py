"""The HIP build with W given at the irreducible q points only (Sec. III.A,
unfolded inside the library through the caller's sphere maps) against the
build with W at every q and against the oracle on the unfolded W."""
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


def _fcc2():
    return B.make_system(B.cell_fcc(7.0), (16, 16, 16), (2, 2, 2), 2, 3, 3.0, seed=72)


def _hex6():
    return B.make_system(B.cell_hex(B.A_HBN, B.C_HBN), (12, 12, 40), (6, 6, 1), 2, 2, 4.0, seed=76)


CASES = [("fcc2-O", _fcc2, True), ("hex6-D6", _hex6, True), ("si24-O", lambda: B.make_config(1), True),
         ("si24-Oh", lambda: B.make_config(1), False)]


@pytest.mark.parametrize("name,make,proper", CASES, ids=[c[0] for c in CASES])
def test_irreducible_W_equals_the_full_W_build(name, make, proper):
    """Every precision: the maps read the same values the unfolded W holds, so
    the build is bit-identical to the one from W at every q."""
    import paper_1206_3518_amd as P
    import torch
    s = B.with_point_group_W(make(), proper=proper)
    for prec in ("fp64", "split_fp32", "bf16x3"):
        a = P.build_H(P.DeviceSystem(s), prec).clone()
        d = P.DeviceSystem(s, irreducible_W=True)
        b = P.build_H(d, prec)
        torch.cuda.synchronize()
        _say(f"{name} {prec}: {d.nirr} of {s.nk} W matrices; equal {torch.equal(a, b)}")
        assert d.W.shape[0] == len(s.W_irr) < s.nk
        assert torch.equal(a, b)


@pytest.mark.parametrize("name,make,proper", CASES[:3], ids=[c[0] for c in CASES[:3]])
def test_irreducible_W_matches_oracle(name, make, proper):
    """FP64 parity with the oracle on W unfolded by the oracle itself."""
    import dataclasses

    import paper_1206_3518_amd as P
    import torch
    s = B.with_point_group_W(make(), proper=proper)
    ref_sys = dataclasses.replace(s, W=O.unfold_W(s.W_irr, s.wsrc, s.wmap, s.ng))
    H = P.build_H(P.DeviceSystem(s, irreducible_W=True), "fp64")
    torch.cuda.synchronize()
    Hc = H.cpu().numpy()
    nk, nt = s.nk, s.nv * s.nc
    if nk <= 8:
        ref = O.build_H(ref_sys)
        err, bar = np.abs(Hc - ref).max(), fp64_h_bar(ref)
    else:
        rng = np.random.default_rng(5)
        blocks = [(0, 0), (0, nk - 1), (nk - 1, nk - 1), (3, 17)]
        blocks += [tuple(sorted(int(x) for x in rng.integers(0, nk, 2))) for _ in range(6)]
        ref = O.build_blocks(ref_sys, blocks)
        kmax = max(np.abs(r - np.diag(np.diag(r))).max() for r in ref)
        bar = 1e-10 * kmax + 2.0 ** -50 * max(np.abs(r).max() for r in ref)
        err = max(np.abs(Hc[a * nt:(a + 1) * nt, b * nt:(b + 1) * nt] - r).max() for (a, b), r in zip(blocks, ref))
    _say(f"{name}: max|H - H_oracle| {err:.3e} eV (bar {bar:.3e})")
    assert err <= bar


def test_irreducible_W_with_time_reversal_chunks_and_batch():
    """BSE_TIME_REVERSAL and many chunks give the same H as the plain build;
    a batch mixing a system with W at every q and one with W at the
    irreducible points equals their single builds."""
    import paper_1206_3518_amd as P
    import torch
    s = B.with_point_group_W(B.make_config(1, time_reversal=True), proper=True)
    d = P.DeviceSystem(s, irreducible_W=True)
    P.bse_build_H([d], P.BSE_FP64, 0)
    one = d.H.clone()
    P.bse_build_H([d], P.BSE_FP64, P.BSE_TIME_REVERSAL | P.BSE_VALIDATE)
    torch.cuda.synchronize()
    tr_err = (d.H - one).abs().max().item()
    try:
        P.bse_set_chunk_budget(64 << 20)
        d.H.zero_()
        P.bse_build_H([d], P.BSE_FP64, 0)
        torch.cuda.synchronize()
        assert torch.equal(d.H, one)
    finally:
        P.bse_set_chunk_budget(0)
    e = P.DeviceSystem(B.make_system(B.cell_fcc(B.A_SI), (24, 24, 24), (2, 2, 2), 3, 3, 6.0, seed=62))
    P.bse_build_H([e], P.BSE_FP64, 0)
    single = e.H.clone()
    d.H.zero_()
    e.H.zero_()
    P.bse_build_H([e, d], P.BSE_FP64, 0)
    torch.cuda.synchronize()
    _say(f"time reversal: max|dH| {tr_err:.3e} eV")
    assert tr_err <= 1e-10 * one.abs().max().item()
    assert torch.equal(d.H, one) and torch.equal(e.H, single)


def test_irreducible_W_validation():
    """BSE_VALIDATE accepts the irreducible matrices and catches a
    non-Hermitian one."""
    import paper_1206_3518_amd as P
    s = B.with_point_group_W(_fcc2(), proper=True)
    d = P.DeviceSystem(s, irreducible_W=True)
    P.bse_build_H([d], P.BSE_FP64, P.BSE_VALIDATE)
    d.W[1, 2, 3] += 0.5
    with pytest.raises(P.BseError) as ei:
        P.bse_build_H([d], P.BSE_FP64, P.BSE_VALIDATE)
    assert "Hermitian" in str(ei.value)


def test_screening_at_the_irreducible_points():
    """bse_screening with the maps computes W at the irreducible q points only:
    matrix i equals the oracle's W at that point and the full screening's W
    there; the H built from those matrices through the maps matches the
    oracle's H on W unfolded by the oracle from its own matrices."""
    import dataclasses

    import paper_1206_3518_amd as P
    import torch
    s0 = B.make_system(B.cell_fcc(7.0), (16, 16, 16), (2, 2, 2), 2, 6, 2.0, seed=73)
    s = B.with_point_group_W(s0, proper=True)
    reps, _, _ = B.point_group_maps(s0, proper=True)
    vq = B.coulomb_table(s)
    d = P.DeviceSystem(s, irreducible_W=True)
    Wi = P.bse_screening(d, vq, s.head)
    Wf = P.bse_screening(P.DeviceSystem(s), vq, s.head)
    torch.cuda.synchronize()
    assert Wi.shape[0] == len(reps) < s.nk
    # the full screening gathers its empty x occupied densities from the partner
    # q's transforms, the irreducible one transforms both orders: equal to rounding
    dfull = max((Wi[i] - Wf[q]).abs().max().item() for i, q in enumerate(reps))
    ref = O.screened_interaction(s, vq, s.head)
    err = max(np.abs(Wi[i].cpu().numpy() - ref[q]).max() for i, q in enumerate(reps))
    scale = np.abs(ref).max()
    _say(f"irreducible screening: {len(reps)} of {s.nk} q; max|dW| {err:.3e} (max|W| {scale:.3e}); "
         f"max|dW| against the full screening there {dfull:.3e}")
    assert err <= 1e-11 * scale
    assert dfull <= 1e-12 * scale
    # few q: the row sums are split into slices and reduced in order, the same
    # in any chunking
    try:
        P.bse_set_chunk_budget(1 << 20)
        Wc = P.bse_screening(d, vq, s.head)
        torch.cuda.synchronize()
    finally:
        P.bse_set_chunk_budget(0)
    assert torch.equal(Wc, Wi)
    # the BSE of the first 2 empty bands on those matrices
    nb = s.nv + 2
    cut = dict(nc=2, u=np.ascontiguousarray(s.u[:, :nb]), eps=np.ascontiguousarray(s.eps[:, :nb]))
    sg = dataclasses.replace(s, W_irr=Wi.cpu().numpy(), **cut)
    H = P.build_H(P.DeviceSystem(sg, irreducible_W=True)).cpu().numpy()
    W_or = O.unfold_W(np.array([ref[q] for q in reps]), s.wsrc, s.wmap, s.ng)
    Href = O.build_H(dataclasses.replace(s, W=W_or, **cut))
    dh = np.abs(H - Href).max()
    _say(f"H from the irreducible screened W: max|dH| vs oracle {dh:.3e} eV")
    assert dh <= fp64_h_bar(Href) + 1e-11 * np.abs(Href - np.diag(np.diag(Href))).max()


def test_irreducible_W_at_finite_momentum_and_beyond_tda():
    """The mapped W loader in the other builds that run the direct term: at
    finite exciton momentum, and in the coupling block of the beyond-TDA
    matrix, W through the maps gives the same matrix as W at every q."""
    import paper_1206_3518_amd as P
    import torch
    s = B.with_point_group_W(_fcc2(), proper=True)
    sq = B.with_exciton_momentum(s, 3)
    a = P.build_H(P.DeviceSystem(sq), "fp64").clone()
    b = P.build_H(P.DeviceSystem(sq, irreducible_W=True), "fp64")
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    f1 = P.bse_build_H_full(P.DeviceSystem(s)).clone()
    f2 = P.bse_build_H_full(P.DeviceSystem(s, irreducible_W=True))
    torch.cuda.synchronize()
    _say(f"finite Q and beyond-TDA with irreducible W: equal {torch.equal(a, b)}, {torch.equal(f1, f2)}")
    assert torch.equal(f1, f2)


@pytest.mark.parametrize("make", [
    lambda: B.make_system(B.cell_fcc(7.0), (16, 16, 16), (3, 3, 3), 2, 2, 2.0, seed=75),
    lambda: B.make_system(B.cell_hex(B.A_HBN, B.C_HBN), (12, 12, 40), (3, 3, 1), 2, 2, 3.0, seed=79)],
    ids=["fcc3-O", "hex3-D6"])
def test_backward_with_irreducible_W(make):
    """The adjoint with W given at the irreducible points: dL/dW of the nirr
    matrices equals the oracle's adjoint at every q folded by the oracle
    (the adjoint of the unfolding), and the fold of the GPU's own full-W
    backward; dL/de is unchanged."""
    import paper_1206_3518_amd as P
    import torch
    s = B.with_point_group_W(make(), proper=True)
    assert s.wsrc[:, 1].any()
    d = P.DeviceSystem(s, irreducible_W=True)
    H = P.build_H(d).cpu().numpy()
    e, x = np.linalg.eigh(H)
    G = np.outer(x[:, 0], np.conj(x[:, 0]))
    dG = torch.from_numpy(G).cuda()
    dWi, depsi = P.bse_build_H_backward(d, dG)
    dWf, depsf = P.bse_build_H_backward(P.DeviceSystem(s), dG)
    torch.cuda.synchronize()
    dWi, depsi, dWf, depsf = dWi.cpu().numpy(), depsi.cpu().numpy(), dWf.cpu().numpy(), depsf.cpu().numpy()
    nirr, ngm = len(s.W_irr), s.ng_max
    assert dWi.shape == (nirr, ngm, ngm)
    rW, reps = O.adjoint(s, G)
    ref = O.fold_dW(rW, s.wsrc, s.wmap, s.ng, nirr, ngm)
    scale = np.abs(ref).max()
    err = np.abs(dWi - ref).max()
    own = np.abs(dWi - O.fold_dW(dWf, s.wsrc, s.wmap, s.ng, nirr, ngm)).max()
    _say(f"backward with irreducible W: {nirr} of {s.nk} matrices; max|dW - oracle| {err:.3e} "
         f"(max {scale:.3e}); against the folded full-W backward {own:.3e}")
    assert err <= 1e-10 * scale
    assert own <= 1e-12 * scale
    assert np.array_equal(depsi, depsf) and np.abs(depsi - reps).max() <= 1e-12
