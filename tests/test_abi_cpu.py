"""C-ABI checks that need no GPU: the library loads, exports every entry
point declared in include/gabi.h, and its host-only utilities agree with
the oracle."""
import os
import re
import subprocess

import numpy as np
import pytest

import oracle
from paper_1301_5885_amd import gabi
from paper_1301_5885_amd.synth import icosphere, star_surface

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gabi.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gabi_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_binding_exports():
    assert declared_functions() == sorted(gabi.EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = gabi.load()
    for name in declared_functions():
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", gabi.LIB_PATH],
                         capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r"\bT (gabi_\w+)", out))
    assert set(declared_functions()) <= exported


def test_library_is_gfx950():
    """The library built here embeds a gfx950 code object (bundle id)."""
    blob = open(gabi.LIB_PATH, "rb").read()
    assert b"amdgcn-amd-amdhsa--gfx950" in blob


def test_default_opts():
    o = gabi.default_opts()
    assert (o.restart, o.maxit, o.tol, o.mode) == (20, 100, 1e-6, gabi.SOLVE_FP64)
    assert o.inner_tol == 3e-6


@pytest.mark.parametrize("kind", ["sphere", "star"])
def test_mesh_elements_match_oracle(kind):
    if kind == "sphere":
        V, F = icosphere(6, 3.0)
    else:
        V, F, _ = star_surface(6, 10.0, np.random.default_rng(1))
    got = gabi.mesh_elements(V, F)
    ref = oracle.mesh_elements(V, F)
    for k in ("cx", "cy", "cz", "nx", "ny", "nz", "area"):
        assert np.allclose(got[k], getattr(ref, k), rtol=1e-15, atol=1e-15), k


def test_mesh_elements_rejects_bad_meshes():
    V, F = icosphere(2, 1.0)
    bad = F.copy()
    bad[3, 1] = len(V)          # index out of range
    with pytest.raises(gabi.GabiError) as e:
        gabi.mesh_elements(V, bad)
    assert e.value.code == gabi.EMESH
    deg = F.copy()
    deg[0, 2] = deg[0, 1]       # zero-area triangle
    with pytest.raises(gabi.GabiError) as e:
        gabi.mesh_elements(V, deg)
    assert e.value.code == gabi.EMESH


def test_create_without_device_fails_cleanly():
    """With no GPU visible, gabi_create reports GABI_EDEVICE (no crash, no
    fallback); with a GPU it succeeds."""
    try:
        ctx = gabi.Context(0)
    except gabi.GabiError as e:
        assert e.code == gabi.EDEVICE
    else:
        ctx.close()


def test_tuning_table_set_get_and_validation():
    """The decomposition table is host state: entries read back as set, and
    out-of-range entries are rejected without changing the table."""
    before = gabi.tune_get(gabi.FP32_PAIR, 14)
    try:
        gabi.tune_set(gabi.FP32_PAIR, 14, gabi.SCHEME_SPLIT, 2, 3000, 17)
        assert gabi.tune_get(gabi.FP32_PAIR, 14) == (gabi.SCHEME_SPLIT, 2, 3000, 17)
        for bad in [(0, 3, 100, 0), (0, 1, 0, 0), (0, 1, 1 << 21, 0), (0, 1, 100, -1),
                    (0, 1, 100, 5000), (2, 1, 100, 0), (gabi.SCHEME_SYMMETRIC, 2, 1, 0)]:
            with pytest.raises(gabi.GabiError) as e:
                gabi.tune_set(gabi.FP32_PAIR, 14, *bad)
            assert e.value.code == gabi.EINVAL
        with pytest.raises(gabi.GabiError):
            gabi.tune_set(gabi.FP64, 40, gabi.SCHEME_SPLIT, 1, 100, 0)
        assert gabi.tune_get(gabi.FP32_PAIR, 14) == (gabi.SCHEME_SPLIT, 2, 3000, 17)
    finally:
        gabi.tune_set(gabi.FP32_PAIR, 14, *before)


def test_footprint_follows_the_decomposition():
    """More splits mean a larger partial-sum buffer, so a larger footprint."""
    b = (20480).bit_length() - 1
    saved = [gabi.tune_get(p, b) for p in (gabi.FP64, gabi.FP32_PAIR)]
    try:
        for p in (gabi.FP64, gabi.FP32_PAIR):
            gabi.tune_set(p, b, gabi.SCHEME_SPLIT, 1, 64, 0)
        small = gabi.solve_footprint(20480, 200, 10)
        for p in (gabi.FP64, gabi.FP32_PAIR):
            gabi.tune_set(p, b, gabi.SCHEME_SPLIT, 1, 8192, 64)
        large = gabi.solve_footprint(20480, 200, 10)
        # 80 row blocks: one split of all 80 tiles, against 64 one-tile splits
        # of the first 16384 sources and 64 tail splits of the last 4096
        assert large - small == (128 - 1) * 2 * 20480 * 8
        # symmetric: one partial per 256-source block (80), FP64 for both
        # precisions' buffer since the FP64 sums are the larger
        for p in (gabi.FP64, gabi.FP32_PAIR):
            gabi.tune_set(p, b, gabi.SCHEME_SYMMETRIC, 1, 1, 0)
        sym = gabi.solve_footprint(20480, 200, 10)
        assert sym - small == (80 - 1) * 2 * 20480 * 8
        # tail_pieces does not change the symmetric scheme
        for p in (gabi.FP64, gabi.FP32_PAIR):
            gabi.tune_set(p, b, gabi.SCHEME_SYMMETRIC, 1, 1, 16)
        assert gabi.solve_footprint(20480, 200, 10) == sym
        # a budget of 20 FP64 slots: 4 passes of 20 rounds, 20 slots per row
        # and an FP64 accumulator of 2N
        budget = gabi.get_part_budget()
        try:
            gabi.set_part_budget(20 * 2 * 20480 * 8)
            assert gabi.solve_footprint(20480, 200, 10) - small == \
                (20 - 1) * 2 * 20480 * 8 + 2 * 20480 * 8
        finally:
            gabi.set_part_budget(budget)
    finally:
        for p, e in zip((gabi.FP64, gabi.FP32_PAIR), saved):
            gabi.tune_set(p, b, *e)


@pytest.mark.parametrize("theta,degree,leaf", [(0.7, 4, 64), (0.5, 6, 128), (0.8, 2, 256),
                                               (0.0, 3, 100)])
def test_tree_plan_matches_the_treecode_oracle(theta, degree, leaf):
    """The library's host tree builder and interaction lists (tree.hip) and
    the oracle's own implementation of the same rules give the same tree:
    leaves, proxy clusters, list entries and pair counts agree exactly."""
    import oracle.treecode as tc
    rng = np.random.default_rng(5)
    V, F, _ = star_surface(12, 9.0, rng)
    el = oracle.mesh_elements(V, F)
    got = gabi.tree_plan(el.centroids, theta, degree, leaf)
    _, st = tc.matvec(el, rng.normal(size=2 * el.n), theta=theta, degree=degree, leaf=leaf,
                      stats=True)
    assert got["leaves"] == st.leaves
    assert got["clusters_with_proxies"] == st.clusters_with_proxies
    assert got["far_entries"] == st.far_entries and got["near_entries"] == st.near_entries
    assert got["far_pairs"] == st.far_pairs and got["near_pairs"] == st.near_pairs


def test_tree_plan_rejects_bad_options():
    c = np.random.default_rng(0).normal(size=(50, 3))
    for bad in [dict(theta=1.0), dict(theta=-0.1), dict(degree=0), dict(degree=9),
                dict(leaf_size=0), dict(leaf_size=257)]:
        kw = dict(theta=0.5, degree=3, leaf_size=16)
        kw.update(bad)
        with pytest.raises(gabi.GabiError):
            gabi.tree_plan(c, **kw)


def test_part_budget_bounds_the_footprint():
    """The partial-sum budget bounds a molecule's device memory: at the
    default budget a 327,680-element solve holds well under 1 GB, and the
    footprint grows about linearly in N beyond the size where the budget
    binds."""
    base = gabi.get_part_budget()
    assert base == 512 << 20
    f_large = gabi.solve_footprint(327680, 5000, 10)
    assert f_large < 1 << 30
    f_2x = gabi.solve_footprint(4 * 327680, 5000, 10)
    assert f_2x < 4 * f_large * 1.05   # linear, not quadratic
    try:
        gabi.set_part_budget(1 << 20)
        assert gabi.solve_footprint(327680, 5000, 10) < f_large
    finally:
        gabi.set_part_budget(base)
    with pytest.raises(gabi.GabiError):
        gabi.set_part_budget(0)
