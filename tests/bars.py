"""Tolerances shared by the GPU parity tests."""
import numpy as np


def fp64_h_bar(ref):
    """Bar for an FP64 GPU H against the oracle's: 1e-10 of the kernel
    K = H - diag(H) (the two sides sum in different orders: FFT against direct
    DFT sums, GEMM blocking against loops) plus 4 ulp of the largest element,
    for the eV-sized transition energies on the diagonal."""
    ref = np.asarray(ref)
    kmax = np.abs(ref - np.diag(np.diag(ref))).max() if ref.ndim == 2 and ref.shape[0] == ref.shape[1] else 0.0
    return 1e-10 * kmax + 2.0 ** -50 * np.abs(ref).max()
