"""Pins for the treecode oracle (CPU only).

The treecode approximates the product of Section 2.2 (eqs. (eqdbef1),
(eqdbef2)); its oracle is pinned against the direct-sum oracle (itself
pinned in test_oracle.py) and against properties of its own parts:
theta -> 0 reproduces the direct sum, the error falls as the interpolation
degree rises and as theta falls, barycentric interpolation reproduces
polynomials of its degree exactly, the modified weights conserve the total
weight (the Lagrange basis sums to one), and the tree partitions the
elements.
"""
import math

import numpy as np
import pytest

import oracle
import oracle.treecode as tc
from paper_1301_5885_amd.synth import icosphere, star_surface

EPS1, EPS2, KAPPA = 1.0, 80.0, 0.1257


@pytest.fixture(scope="module")
def sphere():
    V, F = icosphere(16, 10.0)           # N = 5120
    el = oracle.mesh_elements(V, F)
    u = np.random.default_rng(0).normal(size=2 * el.n)
    return el, u, oracle.matvec(el, u, EPS1, EPS2, KAPPA)


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def test_theta_zero_is_the_direct_sum(sphere):
    el, u, yd = sphere
    y, st = tc.matvec(el, u, EPS1, EPS2, KAPPA, theta=0.0, degree=4, leaf=128, stats=True)
    assert st.far_entries == 0
    assert st.near_pairs == el.n * el.n           # every pair, the self terms skipped inside
    assert rel(y, yd) < 1e-14


def test_error_falls_with_degree(sphere):
    el, u, yd = sphere
    errs = []
    for deg in (2, 3, 4, 5, 6):
        y, st = tc.matvec(el, u, EPS1, EPS2, KAPPA, theta=0.8, degree=deg, leaf=64,
                          stats=True)
        assert st.far_entries > 0
        errs.append(rel(y, yd))
    assert all(b < a for a, b in zip(errs, errs[1:])), errs
    # about a factor 3-7 per degree on this mesh
    assert errs[-1] < 3e-6 and errs[0] > 1e-4


def test_error_falls_with_theta(sphere):
    el, u, yd = sphere
    errs = [rel(tc.matvec(el, u, EPS1, EPS2, KAPPA, theta=t, degree=3, leaf=64), yd)
            for t in (0.9, 0.7, 0.5)]
    assert errs[1] < errs[0] and errs[2] < errs[1], errs


def test_kappa_zero_and_star_surface():
    """Coulomb case (K1 = K4 = 0) and an uneven surface."""
    rng = np.random.default_rng(3)
    V, F, _ = star_surface(16, 12.0, rng)
    el = oracle.mesh_elements(V, F)
    u = rng.normal(size=2 * el.n)
    for kappa in (0.0, 0.3):
        yd = oracle.matvec(el, u, EPS1, EPS2, kappa)
        y = tc.matvec(el, u, EPS1, EPS2, kappa, theta=0.7, degree=7, leaf=64)
        assert rel(y, yd) < 1e-6


@pytest.mark.parametrize("n", [1, 3, 6])
def test_barycentric_interpolation_reproduces_polynomials(n):
    s = tc.cheb_points(np.array([-1.3, 0.2, 5.0]), np.array([2.0, 0.9, 7.5]), n)
    b = tc.bary_weights(n)
    rng = np.random.default_rng(n)
    coef = rng.normal(size=n + 1)
    for d in range(3):
        y = rng.uniform(s[d].min(), s[d].max(), 40)
        y[0] = s[d][0]                       # a node exactly
        L = tc.lagrange_1d(y, s[d], b)
        assert np.allclose(L.sum(axis=1), 1.0, atol=1e-13)
        p = lambda x: np.polyval(coef, x)
        assert np.allclose(L @ p(s[d]), p(y), rtol=1e-11, atol=1e-11)
        assert L[0, 0] == 1.0 and np.all(L[0, 1:] == 0.0)


def test_modified_weights_conserve_the_total(sphere):
    el, u, _ = sphere
    pts = el.centroids
    root = tc.build_tree(pts, 64)
    w_s = el.area * u[el.n:]
    w_m = (el.area * u[:el.n])[:, None] * el.normals
    node = root.children[0]
    P, Ws, Wm = tc.proxies(node, pts, w_s, w_m, 4)
    assert P.shape == (125, 3)
    assert math.isclose(Ws.sum(), w_s[node.idx].sum(), rel_tol=1e-11, abs_tol=1e-12)
    assert np.allclose(Wm.sum(axis=0), w_m[node.idx].sum(axis=0), rtol=1e-11, atol=1e-12)
    # proxies lie in the cluster's box
    assert np.all(P >= node.lo - 1e-12) and np.all(P <= node.hi + 1e-12)


def test_tree_partitions_the_elements(sphere):
    el, _, _ = sphere
    pts = el.centroids
    root = tc.build_tree(pts, 100)
    lv = tc.leaves(root)
    allidx = np.concatenate([l.idx for l in lv])
    assert np.array_equal(np.sort(allidx), np.arange(el.n))
    assert all(l.idx.size <= 100 for l in lv)
    for l in lv:
        p = pts[l.idx]
        assert np.all(p >= l.lo) and np.all(p <= l.hi)
