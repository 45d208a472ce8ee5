"""Writes si32_whole_h.json: the oracle's whole Hamiltonian for the Si-like
32^3 workload (fcc a = 10.26 bohr, 8x8x8 k mesh, 4 + 4 bands, ecut 8 Ha,
N_S = 8192), reduced to numbers a GPU test can compare against:

* the ten lowest exciton energies (FP64 eigensolve of the oracle's H),
* max |H| and max |K| with K = H - diag(H),
* (H w)_S on 512 sampled rows S for a fixed unimodular probe vector
  w_S' = exp(2 pi i frac(S' phi)), phi the golden ratio, and ||H w||.

Every one of the 512^2 (k, k') blocks is computed on its own by the oracle
(direct sums, Sec. II.B-II.C), on all host cores: about 40 minutes on 8.
Calls only the oracle and the seeded input generator.

The seeded inputs agree between machines only to rounding (the QR and
Cholesky factorisations of the generator round differently), so the record
also holds sums over the inputs that a test compares to 1e-10 instead of a
bitwise digest.

    python tests/golden/make_si32_whole_h.py                 # everything
    python tests/golden/make_si32_whole_h.py --fingerprint   # only the input sums
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import bse_synth as B  # noqa: E402
import oracle as O  # noqa: E402

PHI = 0.6180339887498949


def probe(ns):
    s = np.arange(ns, dtype=np.float64)
    return np.exp(2j * np.pi * np.mod(s * PHI, 1.0))


def sample_rows(nk, nt):
    return [k * nt + (7 * k) % nt for k in range(nk)]


def fingerprint(s):
    """Sums over the inputs, equal between machines to rounding."""
    return {"u_sum": [float(s.u.sum().real), float(s.u.sum().imag)],
            "u_abs4_sum": float(np.sum(np.abs(s.u) ** 4)),
            "W_sum": [float(s.W.sum().real), float(s.W.sum().imag)],
            "W_abs_sum": float(np.abs(s.W).sum()),
            "eps_sum": float(s.eps.sum()), "vx_sum": float(s.vx.sum())}


def main():
    path = os.path.join(HERE, "si32_whole_h.json")
    if "--fingerprint" in sys.argv:
        s = B.make_config(2)
        out = json.load(open(path))
        out["inputs_fingerprint"] = fingerprint(s)
        with open(path, "w") as f:
            json.dump(out, f, indent=1)
        print(f"updated the input sums of {path}")
        return
    t0 = time.perf_counter()
    s = B.make_config(2)
    H = O.build_H(s)
    t_build = time.perf_counter() - t0
    K = H - np.diag(np.diag(H))
    herm = float(np.abs(H - H.conj().T).max())
    E = np.linalg.eigvalsh(H)[:10]
    w = probe(s.ns)
    Hw = H @ w
    rows = sample_rows(s.nk, s.nv * s.nc)
    out = {
        "workload": s.name, "inputs_digest": s.digest(), "inputs_fingerprint": fingerprint(s), "ns": s.ns,
        "oracle_threads": O.num_threads(), "oracle_build_s": t_build,
        "lowest_exciton_eV": E.tolist(),
        "max_abs_H_eV": float(np.abs(H).max()), "max_abs_K_eV": float(np.abs(K).max()),
        "max_abs_H_minus_H_dagger_eV": herm,
        "probe": "w_S = exp(2 pi i frac(S * 0.6180339887498949))",
        "norm_Hw": float(np.linalg.norm(Hw)),
        "rows": rows, "Hw_re": Hw[rows].real.tolist(), "Hw_im": Hw[rows].imag.tolist(),
    }
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(f"wrote {path}: build {t_build:.0f} s, E0 = {E[0]:.12f} eV, herm {herm:.2e}")


if __name__ == "__main__":
    main()
