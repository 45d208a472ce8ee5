"""Split-FP32 and BF16x3 contractions vs the FP64 oracle."""
import sys

import numpy as np
import pytest

import bse_synth as B
import oracle as O

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("prec", ["split_fp32", "bf16x3"])
@pytest.mark.parametrize("case", ["cfg0", "cfg1", "ragged", "wide_bands"])
def test_mixed_H_within_tolerance(prec, case):
    import paper_1206_3518_amd as P
    import torch
    if case == "wide_bands":  # nv * nc = 81: k blocks span up to three exchange tiles
        s = B.make_system(B.cell_sc(8.0), (16, 16, 16), (4, 1, 1), 9, 9, 1.5, seed=32)
    elif case == "cfg0":
        s = B.make_config(0)
    elif case == "cfg1":
        s = B.make_config(1)
    else:
        s = B.make_system(B.cell_fcc(7.5), (10, 12, 16), (3, 1, 2), 3, 2, 3.0, seed=21)
    H = P.build_H(s, prec)
    torch.cuda.synchronize()
    H = H.cpu().numpy()
    Href = O.build_H(s)
    K = Href - np.diag(np.diag(Href))
    err = np.abs(H - Href).max()
    kscale = np.abs(K).max()
    e = np.linalg.eigvalsh(H)[:10]
    er = np.linalg.eigvalsh(Href)[:10]
    _say(f"{case} {prec}: max|dH| = {err:.3e} eV, max|K| = {kscale:.3e} eV, rel {err / kscale:.3e}, "
         f"max|dE| = {np.abs(e - er).max():.3e} eV")
    assert err <= 1e-4
    assert err <= 1e-3 * kscale
    assert np.abs(e - er).max() <= 1e-4
    # the diagonal transition energies are FP64: only kernel-sized deviations
    d = np.abs(np.diag(H) - np.diag(Href)).max()
    assert d <= 1e-3 * kscale


@pytest.mark.parametrize("prec", ["split_fp32", "bf16x3"])
def test_mixed_full_size_blocks(prec):
    import paper_1206_3518_amd as P
    import torch
    s = B.make_config(2)
    H = P.build_H(s, prec)
    torch.cuda.synchronize()
    nk, nt = s.nk, s.nv * s.nc
    blocks = [(0, 0), (3, 3), (0, nk - 1), (200, 17), (511, 510), (44, 300)]
    ref = O.build_blocks(s, blocks)
    worst = 0.0
    for (ka, kb), r in zip(blocks, ref):
        g = H[ka * nt:(ka + 1) * nt, kb * nt:(kb + 1) * nt].cpu().numpy()
        k = r - (np.diag(np.diag(r)) if ka == kb else 0)
        worst = max(worst, np.abs(g - r).max() / max(np.abs(k).max(), 1e-300))
        assert np.abs(g - r).max() <= 1e-4
    _say(f"full size {prec}: worst block error relative to kernel {worst:.3e}")
    assert worst <= 1e-3
