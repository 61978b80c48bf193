"""FP64 CPU oracle for the boundary-integral Poisson-Boltzmann hot path.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the smoke check and by
the benchmark's CPU-baseline leg, never by the library.  It shares no code
with the HIP path.  The arithmetic lives in ``oracle.c`` (plain C, FP64,
OpenMP over output rows); this module compiles it with gcc and marshals
numpy arrays.  ``dense_solve`` adds the exact solution of the assembled
system by LAPACK LU (numpy.linalg.solve) for small N.

Functions and the passage of arXiv:1301.5885 each follows:
  mesh_elements       Section 2.2 (flat triangles, centroid collocation)
  greens/pair_kernels Section 2.1, eqs. (eq_potential), (Eq_Ls)
  rhs                 Section 2.1, eq. (Eq_Ss); Section 2.2
  matvec/matvec_rows  Section 2.2, eqs. (eqdbef1), (eqdbef2)
  assemble/dense_solve  the same operator as an explicit matrix
  gmres               Section 2.2 and 2.4: restarted GMRES, x0 = 0
  energy/reaction_potential  Section 2.3, eq. (solvation_energy)
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

COULOMB = 332.0716  # kcal A / (mol e^2)


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc into oracle/liboracle.so."""
    if not force and os.path.exists(_LIB) and \
            os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + f".tmp{os.getpid()}"
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
           "-o", tmp, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build(force=False)
        _lib = C.CDLL(_LIB)
        _declare(_lib)
    return _lib


# Timing-only build of the same source with the flags of the CPU-baseline
# plan (-O3 -march=native; -ffp-contract=off keeps every product and sum as
# written, so its results are bitwise those of the default build).
_NATIVE = os.path.join(_HERE, "liboracle_native.so")
NATIVE_FLAGS = ["-O3", "-march=native", "-ffp-contract=off"]


def use_native_build(enable: bool = True) -> None:
    """Route later oracle calls to the timing build (enable) or back to the
    default build.  For timing runs only."""
    global _lib
    if not enable:
        _lib = None
        _load()
        return
    tmp = _NATIVE + f".tmp{os.getpid()}"
    subprocess.run(["gcc", *NATIVE_FLAGS, "-fopenmp", "-fPIC", "-shared", "-std=c11",
                    "-o", tmp, _SRC, "-lm"], check=True)
    os.replace(tmp, _NATIVE)
    lib = C.CDLL(_NATIVE)
    _declare(lib)
    _lib = lib


_dp = C.POINTER(C.c_double)
_i64 = C.c_int64


class GmresInfo(C.Structure):
    _fields_ = [("iterations", C.c_int64), ("matvecs", C.c_int64),
                ("restarts", C.c_int64), ("rel_residual", C.c_double),
                ("converged", C.c_int64)]


def _declare(lib):
    el = [_i64] + [_dp] * 6
    lib.oracle_mesh_elements.argtypes = [_i64, _dp, _i64, C.POINTER(C.c_int32)] + [_dp] * 7
    lib.oracle_pair_kernels.argtypes = [_dp, _dp, _dp, _dp, C.c_double, C.c_double, _dp]
    lib.oracle_greens.argtypes = [_dp, _dp, _dp, _dp, C.c_double, _dp]
    lib.oracle_rhs.argtypes = el + [_i64, _dp, _dp, _dp, _dp, C.c_double, _dp]
    ops = el + [_dp, C.c_double, C.c_double, C.c_double]
    lib.oracle_matvec.argtypes = ops + [_dp, _dp]
    lib.oracle_matvec_rows.argtypes = ops + [_dp, _i64, C.POINTER(C.c_int64), _dp]
    lib.oracle_assemble.argtypes = ops + [_dp]
    lib.oracle_gmres.argtypes = ops + [_dp, _i64, C.c_double, _i64, _dp,
                                       C.POINTER(GmresInfo)]
    lib.oracle_gmres.restype = C.c_int
    lib.oracle_reaction_potential.argtypes = ops + [_dp, _i64, _dp, _dp, _dp, _dp]
    lib.oracle_energy.argtypes = ops + [_dp, _i64, _dp, _dp, _dp, _dp]
    lib.oracle_energy.restype = C.c_double
    lib.oracle_num_threads.restype = C.c_int
    lib.oracle_set_num_threads.argtypes = [C.c_int]


def num_threads() -> int:
    """Threads the oracle's OpenMP loops use."""
    return int(_load().oracle_num_threads())


def set_num_threads(t: int) -> None:
    """Threads of later OpenMP loops (timing runs only; no effect on results)."""
    _load().oracle_set_num_threads(int(t))


def _p(a):
    return a.ctypes.data_as(_dp)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


@dataclass
class Elements:
    """Flat-triangle element data: centroids, unit normals, areas (SoA)."""
    cx: np.ndarray
    cy: np.ndarray
    cz: np.ndarray
    nx: np.ndarray
    ny: np.ndarray
    nz: np.ndarray
    area: np.ndarray

    @property
    def n(self) -> int:
        return int(self.cx.shape[0])

    def args(self):
        return [_i64(self.n)] + [_p(a) for a in (self.cx, self.cy, self.cz,
                                                 self.nx, self.ny, self.nz)]

    @property
    def centroids(self):
        return np.stack([self.cx, self.cy, self.cz], axis=1)

    @property
    def normals(self):
        return np.stack([self.nx, self.ny, self.nz], axis=1)

    @staticmethod
    def from_arrays(c, nrm, area) -> "Elements":
        c, nrm = _f64(c), _f64(nrm)
        return Elements(*(np.ascontiguousarray(c[:, k]) for k in range(3)),
                        *(np.ascontiguousarray(nrm[:, k]) for k in range(3)),
                        _f64(area))


def mesh_elements(V, F) -> Elements:
    lib = _load()
    V = _f64(V)
    F = np.ascontiguousarray(F, dtype=np.int32)
    n = F.shape[0]
    out = [np.empty(n) for _ in range(7)]
    lib.oracle_mesh_elements(_i64(V.shape[0]), _p(V), _i64(n),
                             F.ctypes.data_as(C.POINTER(C.c_int32)),
                             *[_p(a) for a in out])
    return Elements(*out)


def pair_kernels(x, nux, y, nuy, kappa, eps):
    """(K1, K2, K3, K4) at one target/source pair, eps = eps2/eps1."""
    lib = _load()
    a = [_f64(v) for v in (x, nux, y, nuy)]
    K = np.empty(4)
    lib.oracle_pair_kernels(*[_p(v) for v in a], C.c_double(kappa),
                            C.c_double(eps), _p(K))
    return K


def greens(x, nux, y, nuy, kappa):
    """(G0, Gk, dG0/dnu_y, dGk/dnu_y, dG0/dnu_x, dGk/dnu_x, d2G0, d2Gk)."""
    lib = _load()
    a = [_f64(v) for v in (x, nux, y, nuy)]
    out = np.empty(8)
    lib.oracle_greens(*[_p(v) for v in a], C.c_double(kappa), _p(out))
    return out


def _charges(pos, q):
    pos = _f64(pos).reshape(-1, 3)
    return ([np.ascontiguousarray(pos[:, k]) for k in range(3)], _f64(q))


def rhs(el: Elements, pos, q, eps1: float = 1.0) -> np.ndarray:
    lib = _load()
    (px, py, pz), q = _charges(pos, q)
    b = np.empty(2 * el.n)
    lib.oracle_rhs(*el.args(), _i64(q.shape[0]), _p(px), _p(py), _p(pz),
                   _p(q), C.c_double(eps1), _p(b))
    return b


def _ops(el, eps1, eps2, kappa):
    return el.args() + [_p(el.area), C.c_double(eps1), C.c_double(eps2),
                        C.c_double(kappa)]


def matvec(el: Elements, u, eps1=1.0, eps2=80.0, kappa=0.1257) -> np.ndarray:
    lib = _load()
    u = _f64(u)
    assert u.shape == (2 * el.n,)
    y = np.empty(2 * el.n)
    lib.oracle_matvec(*_ops(el, eps1, eps2, kappa), _p(u), _p(y))
    return y


def matvec_rows(el: Elements, u, rows, eps1=1.0, eps2=80.0,
                kappa=0.1257) -> np.ndarray:
    lib = _load()
    u = _f64(u)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    out = np.empty(rows.shape[0])
    lib.oracle_matvec_rows(*_ops(el, eps1, eps2, kappa), _p(u),
                           _i64(rows.shape[0]),
                           rows.ctypes.data_as(C.POINTER(C.c_int64)), _p(out))
    return out


def assemble(el: Elements, eps1=1.0, eps2=80.0, kappa=0.1257) -> np.ndarray:
    lib = _load()
    A = np.empty((2 * el.n, 2 * el.n))
    lib.oracle_assemble(*_ops(el, eps1, eps2, kappa), _p(A))
    return A


def dense_solve(el: Elements, b, eps1=1.0, eps2=80.0, kappa=0.1257):
    """Exact solution of A u = b by LU on the assembled matrix."""
    return np.linalg.solve(assemble(el, eps1, eps2, kappa), _f64(b))


def gmres(el: Elements, b, eps1=1.0, eps2=80.0, kappa=0.1257, restart=10,
          tol=1e-6, maxit=100, x0=None):
    """Restarted GMRES(restart).  Returns (u, info dict)."""
    lib = _load()
    b = _f64(b)
    x = np.zeros(2 * el.n) if x0 is None else _f64(x0).copy()
    info = GmresInfo()
    rc = lib.oracle_gmres(*_ops(el, eps1, eps2, kappa), _p(b), _i64(restart),
                          C.c_double(tol), _i64(maxit), _p(x), C.byref(info))
    if rc < 0:
        raise MemoryError("oracle_gmres allocation failed")
    return x, {"iterations": info.iterations, "matvecs": info.matvecs,
               "restarts": info.restarts, "rel_residual": info.rel_residual,
               "converged": bool(info.converged)}


def reaction_potential(el: Elements, u, pos, eps1=1.0, eps2=80.0,
                       kappa=0.1257) -> np.ndarray:
    lib = _load()
    (px, py, pz), _ = _charges(pos, np.zeros(len(np.atleast_2d(pos))))
    out = np.empty(px.shape[0])
    lib.oracle_reaction_potential(*_ops(el, eps1, eps2, kappa), _p(_f64(u)),
                                  _i64(px.shape[0]), _p(px), _p(py), _p(pz),
                                  _p(out))
    return out


def energy(el: Elements, u, pos, q, eps1=1.0, eps2=80.0,
           kappa=0.1257) -> float:
    """Electrostatic solvation energy in kcal/mol."""
    lib = _load()
    (px, py, pz), q = _charges(pos, q)
    return float(lib.oracle_energy(*_ops(el, eps1, eps2, kappa), _p(_f64(u)),
                                   _i64(q.shape[0]), _p(px), _p(py), _p(pz),
                                   _p(q)))


def solve(el: Elements, pos, q, eps1=1.0, eps2=80.0, kappa=0.1257,
          restart=10, tol=1e-6, maxit=100):
    """rhs -> GMRES -> energy.  Returns (u, E_kcal_per_mol, info)."""
    b = rhs(el, pos, q, eps1)
    u, info = gmres(el, b, eps1, eps2, kappa, restart, tol, maxit)
    return u, energy(el, u, pos, q, eps1, eps2, kappa), info
