"""GPU: products and solves under decompositions other than the tuned table.

The decomposition (rows per thread, source splits, 64-source tail splits,
or the symmetric scheme that evaluates each unordered pair once) changes only
the order in which a row's terms are added and which shared quantities feed
them, so every decomposition must meet the same bars against the oracle: FP64 product
<= 1e-10, FP32-pair product within fp32_tol, and batched results bitwise
equal to the same request alone under that decomposition.  Each test sets the
whole table before creating its contexts and restores it afterwards.
"""
import numpy as np
import pytest

import oracle
from paper_1301_5885_amd import gabi

from test_gpu_parity import (CASES, EPS1, EPS2, KAPPA, fp32_tol, load, log, rel, relmax,
                             star_problem)

pytestmark = pytest.mark.gpu

# (scheme, rows per thread, target workgroups, tail pieces)
LAYOUTS = {
    "one_row_tail16": (gabi.SCHEME_SPLIT, 1, 8192, 16),
    "two_rows_tail5": (gabi.SCHEME_SPLIT, 2, 2048, 5),
    "coarse_no_tail": (gabi.SCHEME_SPLIT, 2, 64, 0),
    "all_tail": (gabi.SCHEME_SPLIT, 1, 1, 4096),   # every split is a 64-source piece
    "symmetric": (gabi.SCHEME_SYMMETRIC, 1, 1, 0),
    "symmetric_band3": (gabi.SCHEME_SYMMETRIC, 1, 1, 3),   # pairs with J - I <= 3 halved
}


@pytest.fixture
def layout(request):
    saved = {(p, b): gabi.tune_get(p, b) for p in (gabi.FP64, gabi.FP32_PAIR) for b in range(40)}
    for p in (gabi.FP64, gabi.FP32_PAIR):
        for b in range(40):
            gabi.tune_set(p, b, *LAYOUTS[request.param])
    yield request.param
    for (p, b), e in saved.items():
        gabi.tune_set(p, b, *e)


@pytest.mark.parametrize("layout", list(LAYOUTS), indirect=True)
@pytest.mark.parametrize("name", ["tetra_4", "ico_80", "born_1280", "star_1620_ragged",
                                  "star_4500_ragged", "star_10580_ragged_r2"])
def test_products_under_layout(layout, name):
    V, F, pos, q = CASES[name]()
    log(f"[layout {layout}] {name} N={len(F)}")
    with gabi.Context(0) as ctx:
        el = load(ctx, V, F, pos, q)
        u = np.random.default_rng(len(F) + 11).normal(size=2 * el.n)
        ref = oracle.matvec(el, u, EPS1, EPS2, KAPPA)
        y64 = ctx.matvec(u, gabi.FP64)
        y32 = ctx.matvec(u, gabi.FP32_PAIR)
        log(f"    fp64 {rel(y64, ref):.3e} max {relmax(y64, ref):.3e}; fp32 {rel(y32, ref):.3e}")
        assert rel(y64, ref) <= 1e-10 and relmax(y64, ref) <= 1e-10
        assert rel(y32, ref) <= fp32_tol(el)
        assert np.array_equal(ctx.matvec(u, gabi.FP32_PAIR), y32)


@pytest.mark.parametrize("layout", ["one_row_tail16", "all_tail", "symmetric", "symmetric_band3"],
                         indirect=True)
def test_batch_bitwise_alone_under_layout(layout):
    probs = [star_problem(9, 12.0, 40, 7), star_problem(15, 16.0, 110, 8),
             star_problem(11, 13.0, 60, 21)]
    ref = []
    with gabi.Context(0) as c:
        for V, F, pos, q in probs:
            c.set_surface_mesh(V, F)
            c.set_charges(pos, q)
            c.set_params(EPS1, EPS2, KAPPA)
            u, info = c.solve(tol=1e-8, mode=gabi.SOLVE_MIXED_IR)
            ref.append((u, c.energy()))
    reqs = [gabi.Request.from_mesh(V, F, pos, q, kappa=KAPPA, tag=i, want_solution=True)
            for i, (V, F, pos, q) in enumerate(probs)]
    res = gabi.batch_solve(reqs, tol=1e-8, mode=gabi.SOLVE_MIXED_IR)
    for (u, E), r, req in zip(ref, res, reqs):
        assert r["status"] == gabi.OK
        assert r["energy"] == E
        assert np.array_equal(req.u, u)
