"""Seeded synthetic inputs: triangulated closed surfaces and point charges.

This module only *generates* inputs (vertex/face meshes, charge positions and
values, per-request parameters).  It holds none of the solver's arithmetic:
no centroid/normal/area conversion, no kernels, no sums.  Both the HIP path
and the CPU oracle receive the arrays produced here.

Stand-ins for the paper's workloads (Section 3): the paper triangulates
molecular surfaces with MSMS and places CHARMM22 partial charges on PDB atoms;
neither the program nor the structures are available, so closed surfaces are
generated directly:

* ``icosphere(nu, R)`` -- frequency-``nu`` geodesic sphere: each icosahedron
  face is cut into ``nu**2`` triangles on a barycentric grid and every vertex
  is projected to radius ``R``.  ``N = 20 nu^2`` faces, ``10 nu^2 + 2``
  vertices, ``30 nu^2`` edges (Euler's polyhedron formula of Section 2.2).
* ``star_surface(nu, R, rng)`` -- the geodesic sphere displaced radially by
  ``r(u) = R (1 + 0.15 sum_{l=1..6} sum_m a_lm Y_lm(u))`` with
  ``a_lm ~ N(0, 1/l^2)`` (redrawn while ``min r < 0.5 R``), a rough,
  non-spherical but star-shaped (hence embedded) surface.

Faces are listed counter-clockwise seen from outside, so the right-hand
normal points out of the molecule.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "icosphere", "star_surface", "star_radius", "charges_in_ball",
    "charges_in_star", "Problem", "config_problem", "serving_requests",
    "CONFIG_NAMES",
]


# --------------------------------------------------------------------------
# geodesic sphere
# --------------------------------------------------------------------------
def _icosahedron():
    p = (1.0 + math.sqrt(5.0)) / 2.0
    v = np.array([
        [-1, p, 0], [1, p, 0], [-1, -p, 0], [1, -p, 0],
        [0, -1, p], [0, 1, p], [0, -1, -p], [0, 1, -p],
        [p, 0, -1], [p, 0, 1], [-p, 0, -1], [-p, 0, 1],
    ], dtype=np.float64)
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    f = np.array([
        [0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11],
        [1, 5, 9], [5, 11, 4], [11, 10, 2], [10, 7, 6], [7, 1, 8],
        [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9],
        [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1],
    ], dtype=np.int64)
    return v, f


def icosphere(nu: int, radius: float = 1.0):
    """Frequency-``nu`` geodesic sphere of radius ``radius``.

    Returns ``(V, F)``: ``V`` float64 (nv, 3), ``F`` int32 (20 nu^2, 3),
    counter-clockwise seen from outside.  Vertices shared between icosahedron
    faces are keyed by their integer barycentric weights on the icosahedron
    vertices, so every shared vertex is generated exactly once and from the
    same arithmetic.
    """
    nu = int(nu)
    if nu < 1:
        raise ValueError("nu must be >= 1")
    iv, ifc = _icosahedron()
    index = {}
    verts = []

    def vid(weights):
        key = tuple(sorted((int(a), int(w)) for a, w in weights if w))
        got = index.get(key)
        if got is None:
            p = np.zeros(3)
            for a, w in key:
                p = p + (w / nu) * iv[a]
            got = len(verts)
            index[key] = got
            verts.append(p)
        return got

    faces = []
    for a, b, c in ifc:
        # grid point (i, j): weights (nu-i-j) on a, i on b, j on c
        g = {}
        for i in range(nu + 1):
            for j in range(nu + 1 - i):
                g[(i, j)] = vid(((a, nu - i - j), (b, i), (c, j)))
        for i in range(nu):
            for j in range(nu - i):
                faces.append((g[(i, j)], g[(i + 1, j)], g[(i, j + 1)]))
                if i + j < nu - 1:
                    faces.append((g[(i + 1, j)], g[(i + 1, j + 1)], g[(i, j + 1)]))
    V = np.array(verts, dtype=np.float64)
    V *= radius / np.linalg.norm(V, axis=1, keepdims=True)
    F = np.array(faces, dtype=np.int32)
    # orient every face counter-clockwise seen from outside
    e1 = V[F[:, 1]] - V[F[:, 0]]
    e2 = V[F[:, 2]] - V[F[:, 0]]
    flip = np.einsum("ij,ij->i", np.cross(e1, e2), V[F].mean(axis=1)) < 0
    F[flip] = F[flip][:, [0, 2, 1]]
    return V, F


# --------------------------------------------------------------------------
# star-shaped surface
# --------------------------------------------------------------------------
def _real_sph_harm(l: int, m: int, u: np.ndarray) -> np.ndarray:
    """Real orthonormal spherical harmonic Y_lm at unit vectors ``u``."""
    from scipy.special import sph_harm_y
    theta = np.arccos(np.clip(u[:, 2], -1.0, 1.0))
    phi = np.arctan2(u[:, 1], u[:, 0])
    y = sph_harm_y(l, abs(m), theta, phi)
    if m > 0:
        return math.sqrt(2.0) * (-1) ** m * y.real
    if m < 0:
        return math.sqrt(2.0) * (-1) ** m * y.imag
    return y.real


@dataclass
class StarShape:
    radius: float
    coeffs: dict = field(default_factory=dict)   # (l, m) -> a_lm
    amplitude: float = 0.15
    lmax: int = 6


def star_radius(shape: StarShape, u: np.ndarray) -> np.ndarray:
    """r(u) = R (1 + amp * sum a_lm Y_lm(u)) at unit vectors u (k, 3)."""
    s = np.zeros(len(u))
    for (l, m), a in shape.coeffs.items():
        s += a * _real_sph_harm(l, m, u)
    return shape.radius * (1.0 + shape.amplitude * s)


def _draw_star(radius: float, rng: np.random.Generator, probe: np.ndarray,
               lmax: int = 6, amplitude: float = 0.15) -> StarShape:
    while True:
        coeffs = {}
        for l in range(1, lmax + 1):
            for m in range(-l, l + 1):
                coeffs[(l, m)] = rng.normal(0.0, 1.0 / l)
        shape = StarShape(radius, coeffs, amplitude, lmax)
        if star_radius(shape, probe).min() >= 0.5 * radius:
            return shape


def star_surface(nu: int, radius: float, rng: np.random.Generator):
    """Radially displaced geodesic sphere.  Returns ``(V, F, shape)``."""
    V, F = icosphere(nu, 1.0)
    shape = _draw_star(radius, rng, V)
    return V * star_radius(shape, V)[:, None], F, shape


# --------------------------------------------------------------------------
# charges
# --------------------------------------------------------------------------
def _unit_vectors(rng, k):
    g = rng.normal(size=(k, 3))
    return g / np.linalg.norm(g, axis=1, keepdims=True)


def charges_in_ball(rng, nc: int, rmax: float):
    """``nc`` positions uniform in the ball of radius ``rmax`` (k, 3)."""
    u = _unit_vectors(rng, nc)
    s = rng.random(nc) ** (1.0 / 3.0)
    return u * (rmax * s)[:, None]


def charges_in_star(rng, shape: StarShape, nc: int, frac: float = 0.8):
    u = _unit_vectors(rng, nc)
    s = rng.random(nc) ** (1.0 / 3.0)
    return u * (frac * s * star_radius(shape, u))[:, None]


# --------------------------------------------------------------------------
# named workloads
# --------------------------------------------------------------------------
@dataclass
class Problem:
    name: str
    V: np.ndarray           # (nv, 3) float64 vertices
    F: np.ndarray           # (n, 3) int32 faces, CCW from outside
    pos: np.ndarray         # (nc, 3) float64 charge positions
    q: np.ndarray           # (nc,) float64 charges in units of e
    eps1: float = 1.0
    eps2: float = 80.0
    kappa: float = 0.1257   # inverse Debye length, 1/Angstrom
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.F.shape[0])

    @property
    def nc(self) -> int:
        return int(self.q.shape[0])


CONFIG_NAMES = ("born", "kirkwood", "star", "large")


def config_problem(name: str, nu: int | None = None) -> Problem:
    """The four single-solve workloads, optionally at a smaller frequency.

    born      sphere R=2, nu=8 (N=1280), one +1 charge at the centre
    kirkwood  sphere R=20, nu=32 (N=20480), 200 charges uniform in r<=18,
              Q uniform on {-1,+1} (seed 2)
    star      star surface R=30, nu=64 (N=81920), 2000 charges inside 0.8 r,
              Q ~ N(0, 0.5^2) (seed 3)
    large     sphere R=40, nu=128 (N=327680), 5000 charges in r<=36,
              Q ~ N(0, 0.5^2) (seed 4)
    eps1=1, eps2=80, kappa=0.1257 / Angstrom for all four.
    """
    if name == "born":
        V, F = icosphere(nu or 8, 2.0)
        return Problem(name, V, F, np.zeros((1, 3)), np.ones(1),
                       meta={"nu": nu or 8, "R": 2.0})
    if name == "kirkwood":
        rng = np.random.default_rng(2)
        V, F = icosphere(nu or 32, 20.0)
        pos = charges_in_ball(rng, 200, 18.0)
        q = np.where(rng.random(200) < 0.5, -1.0, 1.0)
        return Problem(name, V, F, pos, q, meta={"nu": nu or 32, "R": 20.0})
    if name == "star":
        rng = np.random.default_rng(3)
        V, F, shape = star_surface(nu or 64, 30.0, rng)
        pos = charges_in_star(rng, shape, 2000, 0.8)
        q = rng.normal(0.0, 0.5, 2000)
        return Problem(name, V, F, pos, q, meta={"nu": nu or 64, "R": 30.0})
    if name == "large":
        rng = np.random.default_rng(4)
        V, F = icosphere(nu or 128, 40.0)
        pos = charges_in_ball(rng, 5000, 36.0)
        q = rng.normal(0.0, 0.5, 5000)
        return Problem(name, V, F, pos, q, meta={"nu": nu or 128, "R": 40.0})
    raise KeyError(name)


def serving_requests(count: int = 512, nmin: int = 1280, nmax: int = 81920,
                     base_seed: int = 5000):
    """Per-request workloads for the serving mix.

    N_target log-uniform in [nmin, nmax] -> nu = round(sqrt(N/20)) clipped to
    [8, 64], N = 20 nu^2, R = sqrt(N / (16 pi)) (about 4 elements per square
    Angstrom), Nc = N / 40 charges with Q ~ N(0, 0.5^2) inside 0.8 r,
    kappa ~ U[0, 0.3].  Request i uses seed base_seed + i.  Returns a list of
    lazily built problems: ``(nu, kappa, build)`` where ``build()`` makes the
    Problem.
    """
    out = []
    for i in range(count):
        rng = np.random.default_rng(base_seed + i)
        nt = math.exp(rng.uniform(math.log(nmin), math.log(nmax)))
        nu = int(min(64, max(8, round(math.sqrt(nt / 20.0)))))
        kappa = float(rng.uniform(0.0, 0.3))
        seed = int(rng.integers(0, 2**31 - 1))

        def build(nu=nu, kappa=kappa, seed=seed, i=i):
            r = np.random.default_rng(seed)
            n = 20 * nu * nu
            R = math.sqrt(n / (16.0 * math.pi))
            V, F, shape = star_surface(nu, R, r)
            nc = n // 40
            pos = charges_in_star(r, shape, nc, 0.8)
            q = r.normal(0.0, 0.5, nc)
            return Problem(f"req{i}", V, F, pos, q, kappa=kappa,
                           meta={"nu": nu, "R": R})
        out.append((nu, kappa, build))
    return out
