"""GPU: products taken in several passes (a small partial-sum budget).

The symmetric product keeps one partial sum per row and round, at most
`budget / (2N x 8 bytes)` (FP64) or `/ (2N x 4 bytes)` (FP32 pair) of them
at a time: with a small budget a product runs as several passes whose sums
are folded into an FP64 accumulator.  The result must still match the
oracle's product (Section 2.2, eqs. (eqdbef1)/(eqdbef2)) to the tolerances
of test_gpu_parity.py, agree with the single-pass product to rounding, and
stay bitwise the same alone and in a batch whose molecules take different
numbers of passes.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_1301_5885_amd import gabi
from paper_1301_5885_amd.synth import charges_in_star, config_problem, star_surface
from test_gpu_parity import fp32_tol, rel, relmax
from test_gpu_batch import alone, requests

pytestmark = pytest.mark.gpu
EPS1, EPS2, KAPPA = 1.0, 80.0, 0.1257


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def star(nu, R, nc, seed, kappa=KAPPA):
    rng = np.random.default_rng(seed)
    V, F, shape = star_surface(nu, R, rng)
    pos = charges_in_star(rng, shape, nc, 0.8)
    return V, F, pos, rng.normal(0.0, 0.5, nc), kappa


@pytest.fixture
def budget():
    base = gabi.get_part_budget()
    yield gabi.set_part_budget
    gabi.set_part_budget(base)


CASES = {
    "star_4500_ragged": lambda: star(15, 16.0, 110, 8),       # 18 blocks
    "star_10580_ragged": lambda: star(23, 22.0, 260, 9),      # 42 blocks
    "kirkwood_20480": lambda: (lambda p: (p.V, p.F, p.pos, p.q, KAPPA))(
        config_problem("kirkwood")),                           # 80 blocks
}


@pytest.mark.parametrize("slots", [1, 5, 13])
@pytest.mark.parametrize("name", sorted(CASES))
def test_multipass_product_matches_oracle(budget, name, slots):
    V, F, pos, q, kappa = CASES[name]()
    n = len(F)
    budget(slots * 2 * n * 8)  # `slots` FP64 slots per row, twice as many FP32
    log(f"[passes] {name} N={n} FP64 slots {slots}")
    el = oracle.mesh_elements(V, F)
    rng = np.random.default_rng(n + slots)
    u = rng.normal(size=2 * el.n)
    y_ref = oracle.matvec(el, u, EPS1, EPS2, kappa)
    with gabi.Context(0) as ctx:
        ctx.set_surface_mesh(V, F)
        ctx.set_charges(pos, q)
        ctx.set_params(EPS1, EPS2, kappa)
        y64 = ctx.matvec(u, gabi.FP64)
        y32 = ctx.matvec(u, gabi.FP32_PAIR)
    log(f"    fp64 {rel(y64, y_ref):.2e} fp32 {rel(y32, y_ref):.2e}")
    assert rel(y64, y_ref) <= 1e-10 and relmax(y64, y_ref) <= 1e-10
    assert rel(y32, y_ref) <= fp32_tol(el)


def test_multipass_agrees_with_one_pass(budget):
    V, F, pos, q, kappa = CASES["star_10580_ragged"]()
    n = len(F)
    u = np.random.default_rng(1).normal(size=2 * n)
    out = {}
    for key, b in (("one", 1 << 30), ("many", 4 * 2 * n * 8)):
        budget(b)
        with gabi.Context(0) as ctx:
            ctx.set_surface_mesh(V, F)
            ctx.set_charges(pos, q)
            ctx.set_params(EPS1, EPS2, kappa)
            out[key] = (ctx.matvec(u, gabi.FP64), ctx.matvec(u, gabi.FP32_PAIR),
                        ctx.matvec(u, gabi.FP64))
    one, many = out["one"], out["many"]
    assert np.array_equal(many[0], many[2])          # repeatable bit for bit
    assert rel(many[0], one[0]) <= 1e-14
    assert rel(many[1], one[1]) <= 1e-6


@pytest.mark.parametrize("mode", [gabi.SOLVE_FP64, gabi.SOLVE_MIXED_IR])
def test_multipass_batch_is_bitwise_alone(budget, mode):
    """Molecules of 6, 18 and 42 blocks under a budget of 8 FP64 slots of the
    largest: 1, 2-3 and 6 passes; the batch runs as many launches as its
    largest member needs."""
    probs = [star(10, 9.0, 20, 40, 0.1), star(15, 16.0, 80, 41, 0.0),
             star(23, 22.0, 150, 42, 0.3)]
    budget(8 * 2 * 10580 * 8)
    log(f"[passes batch] mode={mode}")
    ref = alone(probs, tol=1e-8, mode=mode)
    reqs = requests(probs)
    res = gabi.batch_solve(reqs, tol=1e-8, mode=mode)
    for (u, E, info), r, req in zip(ref, res, reqs):
        assert r["status"] == gabi.OK
        assert r["info"]["iterations"] == info["iterations"]
        assert r["energy"] == E
        assert np.array_equal(req.u, u)


def test_multipass_solve_matches_oracle(budget):
    V, F, pos, q, kappa = CASES["star_4500_ragged"]()
    budget(3 * 2 * len(F) * 8)
    el = oracle.mesh_elements(V, F)
    _, E_ref, _ = oracle.solve(el, pos, q, EPS1, EPS2, kappa, tol=1e-12, maxit=1000)
    with gabi.Context(0) as ctx:
        ctx.set_surface_mesh(V, F)
        ctx.set_charges(pos, q)
        ctx.set_params(EPS1, EPS2, kappa)
        for mode, tol in ((gabi.SOLVE_FP64, 1e-7), (gabi.SOLVE_MIXED_IR, 1e-6)):
            _, info = ctx.solve(tol=1e-8, mode=mode)
            E = ctx.energy()
            log(f"    mode {mode}: E {E:.10f} oracle {E_ref:.10f} {info}")
            assert info["converged"]
            assert abs(E / E_ref - 1) <= tol
