"""bse_spectrum_noalloc (static device scratch, no workspace) against
bse_spectrum on the same inputs, two calls in a row with the second smaller,
through the C ABI."""
import numpy as np
import pytest


pytestmark = pytest.mark.gpu


def _inputs(ns, nlam, nq, seed):
    import torch
    rng = np.random.default_rng(seed)
    E = np.sort(rng.uniform(1.0, 8.0, nlam))
    A = rng.standard_normal((ns, nlam)) + 1j * rng.standard_normal((ns, nlam))
    d = rng.standard_normal((nq, ns)) + 1j * rng.standard_normal((nq, ns))
    return [torch.from_numpy(np.ascontiguousarray(x)).cuda() for x in (E, A, d)]


def test_noalloc_spectrum_matches_workspace_spectrum():
    import paper_1206_3518_amd as P
    import torch
    nk, omega = 64, 270.0
    for ns, nlam, nq, nw in ((900, 700, 3, 1001), (200, 130, 1, 301)):
        E, A, d = _inputs(ns, nlam, nq, ns)
        ref = P.bse_spectrum(E, A, d, nk, omega, nw, 0.0, 10.0, 0.1)
        out = torch.full((nw,), float("nan"), dtype=torch.float64, device=A.device)
        got = P.bse_spectrum_noalloc(E, A, d, nk, omega, nw, 0.0, 10.0, 0.1, eps2=out)
        torch.cuda.synchronize()
        err = (got - ref).abs().max().item()
        print(f"ns {ns} nlam {nlam} nq {nq}: max diff {err:.3e} (max {ref.abs().max().item():.3e})", flush=True)
        assert torch.equal(got, ref)


def test_noalloc_spectrum_rejects_too_many_excitons():
    """Above the static scratch's size the call is refused on the host; nothing
    is enqueued (the pointers are never touched)."""
    import ctypes
    import paper_1206_3518_amd as P
    n = P.NOALLOC_MAX_NLAM + 1
    fake = ctypes.c_void_p(0x1000)
    rc = P.lib().bse_spectrum_noalloc(n, n, fake, fake, fake, 1, 1, 1.0, 11, 0.0, 1.0, 0.1, fake, None)
    assert rc == -3 and "BSE_NOALLOC_MAX_NLAM" in P.bse_last_error()
