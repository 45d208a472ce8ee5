"""Adjoint kernels for the pair-density gradients (dL/dn_{vk,ck}, dL/drho_vv',
dL/drho_cc') against the oracle, for a Hermitian and a general dL/dH, and at
the full Si 32^3 size on the whole exchange gradient and sampled pairs."""
import sys

import numpy as np
import pytest

import bse_synth as B
import oracle as O

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _cmp(tag, got, ref):
    err = np.abs(got - ref).max()
    scale = np.abs(ref).max()
    _say(f"  {tag}: max err {err:.3e} (scale {scale:.3e})")
    assert err <= 1e-12 * scale


@pytest.mark.parametrize("case", ["cfg0", "ragged", "hbn"])
def test_density_gradients_match_oracle(case):
    import paper_1206_3518_amd as P
    import torch
    if case == "cfg0":
        s = B.make_config(0)
    elif case == "hbn":  # rotated pair-density frame
        s = B.make_hbn_batch(5, nsys=1, ecut=1.5, nv=2, nc=2, meshes=[2])[0]
    else:
        s = B.make_system(B.cell_fcc(7.5), (10, 12, 16), (3, 1, 2), 3, 2, 3.0, seed=21)
    d = P.DeviceSystem(s)
    H = O.build_H(s)
    _, x = np.linalg.eigh(H)
    rng = np.random.default_rng(9)
    X, rv, rc = O.densities(s)
    for tag, G in (("hermitian", np.outer(x[:, 0], np.conj(x[:, 0]))),
                   ("general", rng.normal(size=H.shape) + 1j * rng.normal(size=H.shape))):
        _say(f"{case} {tag}: ns {s.ns}, pairs {s.nk * (s.nk + 1) // 2}")
        dW, deps, dX, drv, drc = P.bse_build_H_backward(d, torch.from_numpy(G).cuda(), want_densities=True)
        torch.cuda.synchronize()
        rX, rrv, rrc = O.adjoint_densities(s, G, X, rv, rc)
        _cmp("dX", dX.cpu().numpy(), rX)
        _cmp("drho_vv", drv.cpu().numpy(), rrv)
        _cmp("drho_cc", drc.cpu().numpy(), rrc)


def test_density_gradients_full_size_sampled():
    import paper_1206_3518_amd as P
    import torch
    s = B.make_config(2)
    d = P.DeviceSystem(s)
    P.bse_build_H([d], P.BSE_FP64, 0)
    e, V = torch.linalg.eigh(d.H)
    x = V[:, 0]
    G = torch.outer(x, x.conj())
    dW, deps, dX, drv, drc = P.bse_build_H_backward(d, G, want_dW=False, want_deps=False, want_densities=True)
    torch.cuda.synchronize()
    Gn = G.cpu().numpy()
    npairs = s.nk * (s.nk + 1) // 2
    # pairs among the k points that carry most of the exciton, plus random ones
    w = (np.abs(x.cpu().numpy()) ** 2).reshape(s.nk, -1).sum(axis=1)
    k1, k2 = (int(k) for k in np.argsort(w)[-2:])
    lex = lambda a, b: a * s.nk - a * (a - 1) // 2 + (b - a)
    rng = np.random.default_rng(3)
    pairs = sorted({lex(k1, k1), lex(k2, k2), lex(min(k1, k2), max(k1, k2)), 0, npairs - 1,
                    *(int(p) for p in rng.choice(npairs, size=3, replace=False))})
    Xo, rvo, rco = O.densities(s, pairs=pairs)
    rX, rrv, rrc = O.adjoint_densities(s, Gn, Xo, rvo, rco, pairs=pairs)
    _say(f"full size: ns {s.ns}, sampled pairs {pairs}")
    _cmp("dX (all S)", dX.cpu().numpy(), rX)
    _cmp("drho_vv (sampled)", drv[pairs].cpu().numpy(), rrv)
    _cmp("drho_cc (sampled)", drc[pairs].cpu().numpy(), rrc)
    assert np.abs(rrv).max() > 1e-3 * np.abs(rX).max()  # the sample sees the exciton
