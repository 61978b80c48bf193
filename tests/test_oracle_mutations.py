"""The oracle's pins catch plausible mistakes (CPU only).

Each case plants one mistake in a temporary copy of oracle/oracle.c -- a
dropped term, a wrong sign, a wrong index, a transposed operand -- builds it
with gcc, and checks that at least one independent pin fails on it, while
the unmodified source passes them all.
"""
import ctypes as C
import math
import os
import subprocess

import numpy as np
import pytest

import oracle
from closed_forms import born_energy, born_surface, sphere_kernel_integrals
from paper_1301_5885_amd.synth import icosphere

SRC = os.path.join(os.path.dirname(oracle.__file__), "oracle.c")

MUTANTS = {
    "K1_sign": ("K[0] = g.G0 - g.Gk;", "K[0] = g.G0 + g.Gk;"),
    "K2_drop_eps": ("K[1] = eps * g.dGk_dny - g.dG0_dny;",
                    "K[1] = g.dGk_dny - g.dG0_dny;"),
    "K3_inverse_eps": ("K[2] = g.dG0_dnx - g.dGk_dnx / eps;",
                       "K[2] = g.dG0_dnx - g.dGk_dnx * eps;"),
    "second_derivative_sign": ("double d2r = (-nn + ux * uy / (r * r)) / r;",
                               "double d2r = (nn + ux * uy / (r * r)) / r;"),
    "normal_swapped": ("double drdnx = ux / r;", "double drdnx = uy / r;"),
    "matvec_transposed_operand": (
        "s_top += area[j] * (K[0] * u[n + j] + K[1] * u[j]);",
        "s_top += area[j] * (K[0] * u[j] + K[1] * u[n + j]);"),
    "matvec_target_area": (
        "s_bot += area[j] * (K[2] * u[n + j] + K[3] * u[j]);",
        "s_bot += area[i] * (K[2] * u[n + j] + K[3] * u[j]);"),
    "diagonal_swapped": ("y[i] = 0.5 * (1.0 + eps) * u[i] - s_top;",
                         "y[i] = 0.5 * (1.0 + 1.0 / eps) * u[i] - s_top;"),
    "rhs_sign": ("s2 += q[k] * g.dG0_dnx;", "s2 -= q[k] * g.dG0_dnx;"),
    "energy_transposed": (
        "s += area[j] * (K[0] * u[n + j] + K[1] * u[j]);\n        }\n        phi_reac[k] = s;",
        "s += area[j] * (K[0] * u[j] + K[1] * u[n + j]);\n        }\n        phi_reac[k] = s;"),
    "givens_sign": ("H[(i + 1) * m + j] = -sn[i] * a + cs[i] * c;",
                    "H[(i + 1) * m + j] = sn[i] * a + cs[i] * c;"),
    "mgs_skips_last": ("for (int64_t i = 0; i <= j; ++i) {\n                double *vi",
                       "for (int64_t i = 0; i < j; ++i) {\n                double *vi"),
    # the sampled-row product (sole checker of the largest products)
    "rows_diagonal_swapped": (
        "out[r] = bottom ? 0.5 * (1.0 + 1.0 / eps) * u[n + i] - s\n"
        "                        : 0.5 * (1.0 + eps) * u[i] - s;",
        "out[r] = bottom ? 0.5 * (1.0 + eps) * u[n + i] - s\n"
        "                        : 0.5 * (1.0 + 1.0 / eps) * u[i] - s;"),
    "rows_bottom_transposed": (
        "s += area[j] * (K[2] * u[n + j] + K[3] * u[j]);",
        "s += area[j] * (K[2] * u[j] + K[3] * u[n + j]);"),
    "rows_index_shift": ("int64_t i = row < n ? row : row - n;",
                         "int64_t i = row < n ? row : row - n + 1;"),
}


def _build(tmp_path, name, text):
    src = tmp_path / f"{name}.c"
    src.write_text(text)
    so = tmp_path / f"lib{name}.so"
    subprocess.run(["gcc", "-O1", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                    "-o", str(so), str(src), "-lm"], check=True)
    lib = C.CDLL(str(so))
    oracle._declare(lib)
    return lib


def _pins():
    """Quick independent pins; returns the names of those that fail."""
    failed = []
    a, kap, eps = 2.0, 0.1257, 80.0
    V, F = icosphere(4, a)
    el = oracle.mesh_elements(V, F)
    n = el.n
    # sphere integrals of K1..K4 through the product
    ref = np.array(sphere_kernel_integrals(a, kap, eps))
    y1 = oracle.matvec(el, np.r_[np.ones(n), np.zeros(n)], 1.0, eps, kap)
    y2 = oracle.matvec(el, np.r_[np.zeros(n), np.ones(n)], 1.0, eps, kap)
    got = np.array([(-y2[:n]).mean(), (0.5 * (1 + eps) - y1[:n]).mean(),
                    (0.5 * (1 + 1 / eps) - y2[n:]).mean(), (-y1[n:]).mean()])
    if np.any(np.abs(got - ref) > 0.12 * np.maximum(np.abs(ref), 1e-2)):
        failed.append("sphere_integrals")
    # Gauss's law for the source term of a central charge
    b = oracle.rhs(el, np.zeros((1, 3)), [1.0])
    if abs(np.dot(el.area, b[n:]) + 1.0) > 0.05:
        failed.append("gauss")
    # Born energy
    u, E, info = oracle.solve(el, np.zeros((1, 3)), [1.0], 1.0, eps, kap, tol=1e-10)
    if not info["converged"] or abs(E / born_energy(a, 1.0, 1.0, eps, kap) - 1) > 0.08:
        failed.append("born")
    # dense LU
    rng = np.random.default_rng(0)
    bb = rng.normal(size=2 * n)
    A = oracle.assemble(el, 1.0, eps, kap)
    ulu = np.linalg.solve(A, bb)
    ug, _ = oracle.gmres(el, bb, 1.0, eps, kap, tol=1e-12, maxit=300)
    if np.linalg.norm(ug - ulu) > 1e-9 * np.linalg.norm(ulu):
        failed.append("dense_lu")
    # swap symmetry of K1, K4 at one pair and the explicit A factor of K2
    x, y = np.array([0.3, 0.1, -0.2]), np.array([1.1, -0.4, 0.5])
    nx_, ny_ = np.array([0.0, 0.6, 0.8]), np.array([0.8, 0.0, -0.6])
    K = oracle.pair_kernels(x, nx_, y, ny_, kap, eps)
    Ks = oracle.pair_kernels(y, ny_, x, nx_, kap, eps)
    r = np.linalg.norm(x - y)
    A_ = math.exp(-kap * r) * (1 + kap * r)
    k2 = (eps * A_ - 1) * np.dot(x - y, ny_) / (4 * math.pi * r ** 3)
    if abs(K[0] - Ks[0]) > 1e-14 * abs(K[0]) or abs(K[3] - Ks[3]) > 1e-12 * abs(K[3]) \
            or abs(K[1] - k2) > 1e-12 * abs(k2):
        failed.append("pair_identities")
    # sampled rows of the product: the Born surface values (the continuous
    # solution) satisfy the discrete equations to O(h) at every row, and the
    # rows of the upper and lower halves differ in diagonal and kernels
    phi_b, psi_b = born_surface(a, 1.0, 1.0, eps, kap)
    ub = np.r_[np.full(n, phi_b), np.full(n, psi_b)]
    rows = np.array([0, 7, n - 1, n, n + 7, 2 * n - 1])
    yr = oracle.matvec_rows(el, ub, rows, 1.0, eps, kap)
    bb0 = oracle.rhs(el, np.zeros((1, 3)), [1.0])
    scale = np.abs(bb0[rows])
    if np.any(np.abs(yr - bb0[rows]) > 0.1 * scale):
        failed.append("rows_born_residual")
    # the sampled rows against the whole product (itself pinned above) on a
    # random vector, all 2N rows
    ur = np.random.default_rng(3).normal(size=2 * n)
    if not np.array_equal(oracle.matvec_rows(el, ur, np.arange(2 * n), 1.0, eps, kap),
                          oracle.matvec(el, ur, 1.0, eps, kap)):
        failed.append("rows_vs_product")
    return failed


@pytest.fixture
def swap_lib():
    saved = oracle._load()
    yield lambda lib: setattr(oracle, "_lib", lib)
    oracle._lib = saved


def test_unmodified_oracle_passes_quick_pins(tmp_path, swap_lib):
    swap_lib(_build(tmp_path, "orig", open(SRC).read()))
    assert _pins() == []


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(tmp_path, swap_lib, name):
    old, new = MUTANTS[name]
    text = open(SRC).read()
    assert text.count(old) == 1, f"mutation site for {name} not unique"
    swap_lib(_build(tmp_path, name, text.replace(old, new)))
    assert _pins(), f"planted mistake {name} passed every pin"
