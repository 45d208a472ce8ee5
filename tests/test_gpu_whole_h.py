"""The whole Si-like Hamiltonian (32^3 grid, 8^3 k mesh, 4 + 4 bands,
N_S = 8192) against the oracle's, from the committed record of one full
oracle run (tests/golden/si32_whole_h.json, written by make_si32_whole_h.py
with the oracle alone): the ten lowest exciton energies, and H times a fixed
probe vector on one row per k point."""
import json
import os
import sys

import numpy as np
import pytest

import bse_synth as B

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "si32_whole_h.json")
PHI = 0.6180339887498949


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def case():
    g = json.load(open(GOLD))
    s = B.make_config(2)
    # the generator's factorisations round differently between machines: the
    # inputs must agree with the record's to rounding, not bit for bit
    f = g["inputs_fingerprint"]
    for key, got in (("u_sum", [s.u.sum().real, s.u.sum().imag]), ("W_sum", [s.W.sum().real, s.W.sum().imag])):
        assert np.allclose(got, f[key], rtol=1e-10, atol=1e-10 * f[key.replace("_sum", "_abs_sum")]
                           if key == "W_sum" else 1e-9), key
    assert abs(np.sum(np.abs(s.u) ** 4) - f["u_abs4_sum"]) <= 1e-10 * f["u_abs4_sum"]
    assert abs(np.abs(s.W).sum() - f["W_abs_sum"]) <= 1e-10 * f["W_abs_sum"]
    assert abs(s.eps.sum() - f["eps_sum"]) <= 1e-12 * abs(f["eps_sum"])
    assert abs(s.vx.sum() - f["vx_sum"]) <= 1e-12 * abs(f["vx_sum"])
    return s, g


def _probe(ns):
    x = np.arange(ns, dtype=np.float64)
    return np.exp(2j * np.pi * np.mod(x * PHI, 1.0))


@pytest.mark.parametrize("mode", ["fp64", "bf16x3+fp32_pairdens"])
def test_whole_h_against_oracle_record(case, mode):
    import paper_1206_3518_amd as P
    import torch
    s, g = case
    prec = P.PRECISIONS[mode.split("+")[0]]
    flags = P.BSE_FP32_PAIRDENS if "fp32_pairdens" in mode else 0
    d = P.DeviceSystem(s)
    ws = P.workspace(P.bse_workspace_size([d], prec, flags))
    P.bse_build_H([d], prec, flags, ws)
    torch.cuda.synchronize()
    del ws
    E = torch.linalg.eigvalsh(d.H)[:10].cpu().numpy()
    Eg = np.array(g["lowest_exciton_eV"])
    dE = np.abs(E - Eg)
    kmax = g["max_abs_K_eV"]
    w = torch.from_numpy(_probe(s.ns)).to(d.device)
    rows = torch.tensor(g["rows"], device=d.device)
    Hw = (d.H[rows] @ w).cpu().numpy()
    ref = np.array(g["Hw_re"]) + 1j * np.array(g["Hw_im"])
    dHw = np.abs(Hw - ref).max()
    _say(f"{mode}: lowest-10 |dE| max {dE.max():.3e} eV (rel {np.max(dE / np.abs(Eg)):.2e}); "
         f"|d(Hw)| max {dHw:.3e} eV on {len(rows)} rows; max|K| {kmax:.3e} eV")
    if mode == "fp64":
        assert np.all(dE <= 1e-6 * np.abs(Eg))
        # each probed row sums 8192 entries of unit-modulus weight: the FP64
        # bar of H (1e-10 max|K| plus 4 ulp of the diagonal) times sqrt(N_S)
        assert dHw <= 1e-10 * kmax * np.sqrt(s.ns) + 2.0 ** -50 * g["max_abs_H_eV"] * 4
    else:
        assert dE.max() <= 1e-4
        assert dHw <= 1e-3 * kmax * np.sqrt(s.ns)
