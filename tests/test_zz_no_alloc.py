"""GPU: the allocation-free FP64 product (gabi_matvec_noalloc) against the
context product gabi_matvec_dev at GABI_FP64 on the same surfaces (Section
2.2, eqs. (eqdbef1)/(eqdbef2)).

Two calls in a row, the second on a smaller surface, so the second reuses
(and must fully rewrite) the scratch the first left behind: the first is
large enough that the allocation-free product takes several passes while
the context takes one (equal to rounding, within the FP64 parity bound
1e-10 of the other product tests); the second takes the symmetric scheme
in one pass in both (the context's tuned scheme from N = 8,192 on) and is
bitwise equal.  Sizes beyond the scratch are rejected with an error.
"""
import sys

import numpy as np
import pytest

from paper_1301_5885_amd import gabi
from paper_1301_5885_amd.synth import icosphere

pytestmark = pytest.mark.gpu
EPS1, EPS2, KAPPA = 1.0, 80.0, 0.1257


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def relmax(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def elements_dev(torch, V, F):
    """(cx, cy, cz, area) per element, then (nx, ny, nz, 0), on the device."""
    el = gabi.mesh_elements(V, F)
    n = el["cx"].shape[0]
    host = np.zeros((2, n, 4))
    host[0] = np.stack([el["cx"], el["cy"], el["cz"], el["area"]], axis=1)
    host[1, :, :3] = np.stack([el["nx"], el["ny"], el["nz"]], axis=1)
    return torch.tensor(host.reshape(-1), dtype=torch.float64, device="cuda")


def test_noalloc_product_matches_context_product():
    import torch
    ctx = gabi.Context(0)
    ctx.set_params(EPS1, EPS2, KAPPA)
    nc = gabi.Context(0)
    nc.set_params(EPS1, EPS2, KAPPA)
    try:
        # nu = 50: N = 50,000 (196 blocks, ragged); nu = 21: N = 8,820 (35
        # blocks, ragged), where the context's tuned decomposition is the
        # symmetric scheme in one pass, as the allocation-free product's
        for k, (nu, R) in enumerate(((50, 32.0), (21, 13.0))):
            V, F = icosphere(nu, R)
            n = len(F)
            log(f"[noalloc] call {k + 1}: N={n}")
            ctx.set_surface_mesh(V, F)
            u = torch.tensor(np.random.default_rng(100 + k).normal(size=2 * n),
                             dtype=torch.float64, device="cuda")
            y_ref = torch.empty_like(u)
            ctx.matvec_dev(u, y_ref, gabi.FP64)
            elem = elements_dev(torch, V, F)
            y = torch.full_like(u, float("nan"))
            nc.matvec_noalloc(elem, u, y)
            torch.cuda.synchronize()
            a, b = y.cpu().numpy(), y_ref.cpu().numpy()
            log(f"    rel {rel(a, b):.2e} max {relmax(a, b):.2e} "
                f"bitwise {np.array_equal(a, b)}")
            assert np.all(np.isfinite(a))
            assert rel(a, b) <= 1e-10 and relmax(a, b) <= 1e-10
            if k == 1:
                assert np.array_equal(a, b)
    finally:
        ctx.close()
        nc.close()


def test_noalloc_rejects_sizes_beyond_its_scratch():
    import torch
    nc = gabi.Context(0)
    nc.set_params(EPS1, EPS2, KAPPA)
    try:
        n = 65537
        elem = torch.zeros(8 * n, dtype=torch.float64, device="cuda")
        u = torch.zeros(2 * n, dtype=torch.float64, device="cuda")
        y = torch.zeros_like(u)
        with pytest.raises(gabi.GabiError) as e:
            nc.matvec_noalloc(elem, u, y)
        assert "65536" in str(e.value)
    finally:
        nc.close()
