"""Treecode approximation of the boundary-integral product -- TEST
INFRASTRUCTURE ONLY (imported by tests/ and the benchmark's CPU leg; shares
no code with the HIP library).

Geng & Jacob (arXiv:1301.5885) evaluate the product of Section 2.2, eqs.
(eqdbef1)/(eqdbef2), by direct summation and name tree codes, O(N log N),
as the way to larger surfaces (Section 1; Section 4).  The treecode here is
the barycentric Lagrange treecode (BLTC) of L. Wang, R. Krasny and
S. Tlupova, "A kernel-independent treecode based on barycentric Lagrange
interpolation", Commun. Comput. Phys. 28 (2020), in its particle-cluster
form with target batches:

* tree: the element centroids are split recursively.  A node holds the
  minimal box of its points; a node with more than `leaf` points is cut at
  the box midpoint in every dimension whose extent is at least 1/sqrt(2) of
  the largest (2, 4 or 8 children; a point with coordinate >= the midpoint
  goes to the upper half); empty children are dropped, the others kept in
  the order of their bit codes (bit t set when the point is in the upper half
  of the t-th cut dimension, dimensions in x, y, z order).  Leaves are the
  target batches.  Centre = box centre, radius = half the box diagonal.
* proxies: a cluster with more than (n+1)^3 points carries the tensor
  Chebyshev points of the second kind of its box, s = mid + hw cos(k pi/n),
  k = 0..n per dimension (hw = the box half-width, raised to 1e-6 of the
  largest half-width of the box where a dimension is flat), and modified
  weights W_k = sum_{j in C} L_k(y_j) w_j for the weights w_j = (s_j, m_j)
  of its elements; L_k is the product of the 1-D barycentric Lagrange bases
  l_k(y) = [b_k/(y - s_k)] / sum_l [b_l/(y - s_l)], b_k = (-1)^k (halved at
  k = 0, n), with l_k = 1 and the others 0 where y = s_k.
* interactions: for batch B every cluster C is visited from the root: if
  (r_B + r_C) < theta R (R = centre distance; compared squared, as
  (r_B + r_C)^2 < theta^2 R^2) then C acts through its proxies if it has
  more than (n+1)^3 points, else through all its points directly; otherwise
  a leaf acts directly and an inner node hands over to its children.
* the product: y_i = (1+eps)/2 phi_i - top_i, y_{N+i} = (1+1/eps)/2 psi_i -
  bot_i with the near (direct, self term skipped) and far (proxy) sums.

"parity unpinned" does not apply: the pins are the direct-sum oracle (theta
-> 0 gives it exactly up to summation order; the error falls with n and as
theta decreases) and the exactness of the interpolation on polynomials.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

from . import Elements

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "treecode.c")
_LIB = os.path.join(_HERE, "liboracle_tree.so")
_lib = None
_dp = C.POINTER(C.c_double)
_i64p = C.POINTER(C.c_int64)


def build(force: bool = True) -> str:
    """Compile treecode.c with oracle.c into oracle/liboracle_tree.so."""
    if not force and os.path.exists(_LIB) and all(
            os.path.getmtime(_LIB) >= os.path.getmtime(p)
            for p in (_SRC, os.path.join(_HERE, "oracle.c"))):
        return _LIB
    tmp = _LIB + f".tmp{os.getpid()}"
    subprocess.run(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-o", tmp,
                    _SRC, os.path.join(_HERE, "oracle.c"), "-lm"], check=True)
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build(force=False)
        lib = C.CDLL(_LIB)
        lib.oracle_general_sums.argtypes = [C.c_int64, _dp, _dp, _i64p, C.c_int64, _dp, _dp,
                                            _dp, _i64p, C.c_double, C.c_double, _dp, _dp]
        lib.oracle_general_sums.restype = None
        _lib = lib
    return _lib


def general_sums(tx, tn, ys, s, m, kappa, eps, skip=None, sid=None):
    """(top, bot) at targets (tx, tn) from generalised sources (ys, s, m)."""
    lib = _load()
    f = lambda a: np.ascontiguousarray(a, dtype=np.float64)
    tx, tn, ys, s, m = f(tx), f(tn), f(ys), f(s), f(m)
    nt, ns = tx.shape[0], ys.shape[0]
    top, bot = np.empty(nt), np.empty(nt)
    sk = None if skip is None else np.ascontiguousarray(skip, dtype=np.int64)
    si = None if sid is None else np.ascontiguousarray(sid, dtype=np.int64)
    p = lambda a: a.ctypes.data_as(_dp)
    lib.oracle_general_sums(nt, p(tx), p(tn), None if sk is None else sk.ctypes.data_as(_i64p),
                            ns, p(ys), p(s), p(m),
                            None if si is None else si.ctypes.data_as(_i64p),
                            float(kappa), float(eps), p(top), p(bot))
    return top, bot


# ---------------------------------------------------------------- the tree
@dataclass
class Node:
    idx: np.ndarray            # element indices, increasing
    lo: np.ndarray
    hi: np.ndarray
    children: list = field(default_factory=list)

    @property
    def centre(self):
        return (self.lo + self.hi) / 2.0

    @property
    def radius(self):
        h = (self.hi - self.lo) / 2.0
        return math.sqrt(h[0] * h[0] + h[1] * h[1] + h[2] * h[2])


def build_tree(pts, leaf):
    """Recursive bisection of the points (rules in the module docstring)."""
    def make(idx):
        p = pts[idx]
        node = Node(idx, p.min(axis=0), p.max(axis=0))
        ext = node.hi - node.lo
        L = float(ext.max())
        if idx.size <= leaf or L == 0.0:
            return node
        dims = [d for d in range(3) if ext[d] >= L / math.sqrt(2.0)]
        mid = (node.lo + node.hi) / 2.0
        code = np.zeros(idx.size, dtype=np.int64)
        for t, d in enumerate(dims):
            code |= (p[:, d] >= mid[d]).astype(np.int64) << t
        for c in range(1 << len(dims)):
            sub = idx[code == c]
            if sub.size:
                node.children.append(make(sub))
        return node
    return make(np.arange(pts.shape[0]))


def leaves(node):
    if not node.children:
        return [node]
    out = []
    for c in node.children:
        out += leaves(c)
    return out


# ----------------------------------------------------- interpolation parts
def cheb_points(lo, hi, n):
    """Per-dimension Chebyshev points of the second kind of the box."""
    hw = (hi - lo) / 2.0
    big = float(hw.max())
    hw = np.maximum(hw, 1e-6 * big)
    mid = (lo + hi) / 2.0
    c = np.cos(np.arange(n + 1) * math.pi / n)
    return [mid[d] + hw[d] * c for d in range(3)]


def bary_weights(n):
    b = np.array([(-1.0) ** k for k in range(n + 1)])
    b[0] *= 0.5
    b[n] *= 0.5
    return b


def lagrange_1d(y, s, b):
    """l_k(y) for all k (rows: points y, columns: nodes s)."""
    y = np.asarray(y, dtype=np.float64)
    out = np.empty((y.size, s.size))
    for a, yy in enumerate(y):
        diff = yy - s
        hit = np.nonzero(diff == 0.0)[0]
        if hit.size:
            out[a] = 0.0
            out[a, hit[0]] = 1.0
        else:
            q = b / diff
            out[a] = q / q.sum()
    return out


def proxies(node, pts, w_s, w_m, n):
    """Proxy points (P, 3) and modified weights (P,), (P, 3) of a cluster;
    k = (k1 (n+1) + k2)(n+1) + k3 for nodes k1 in x, k2 in y, k3 in z."""
    sx, sy, sz = cheb_points(node.lo, node.hi, n)
    b = bary_weights(n)
    p = pts[node.idx]
    lx, ly, lz = (lagrange_1d(p[:, 0], sx, b), lagrange_1d(p[:, 1], sy, b),
                  lagrange_1d(p[:, 2], sz, b))
    # L[j, k1, k2, k3] = lx[j,k1] ly[j,k2] lz[j,k3]
    L = lx[:, :, None, None] * ly[:, None, :, None] * lz[:, None, None, :]
    L = L.reshape(p.shape[0], -1)
    Ws = L.T @ w_s[node.idx]
    Wm = L.T @ w_m[node.idx]
    X, Y, Z = np.meshgrid(sx, sy, sz, indexing="ij")
    P = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    return P, Ws, Wm


def interaction_lists(root, batch, theta, n):
    """(far clusters, near nodes) of one batch, in visiting order."""
    P = (n + 1) ** 3
    far, near = [], []
    cb, rb = batch.centre, batch.radius
    th2 = theta * theta

    def visit(c):
        d = cb - c.centre
        R2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2]
        rr = rb + c.radius
        if rr * rr < th2 * R2:
            (far if c.idx.size > P else near).append(c)
        elif not c.children:
            near.append(c)
        else:
            for ch in c.children:
                visit(ch)
    visit(root)
    return far, near


@dataclass
class TreeStats:
    leaves: int
    clusters_with_proxies: int
    far_entries: int
    near_entries: int
    far_pairs: int
    near_pairs: int


def matvec(el: Elements, u, eps1=1.0, eps2=80.0, kappa=0.1257, theta=0.7, degree=5,
           leaf=256, stats=False):
    """Treecode approximation of A u (same output layout as oracle.matvec)."""

    n_el = el.n
    eps = eps2 / eps1
    u = np.asarray(u, dtype=np.float64)
    phi, psi = u[:n_el], u[n_el:]
    pts = el.centroids
    nrm = el.normals
    w_s = el.area * psi
    w_m = (el.area * phi)[:, None] * nrm
    root = build_tree(pts, leaf)
    batches = leaves(root)
    cache = {}
    top = np.empty(n_el)
    bot = np.empty(n_el)
    nf = nn = fp = np_ = 0
    for B in batches:
        far, near = interaction_lists(root, B, theta, degree)
        ys, s, m, sid = [], [], [], []
        for c in near:
            ys.append(pts[c.idx])
            s.append(w_s[c.idx])
            m.append(w_m[c.idx])
            sid.append(c.idx)
            np_ += c.idx.size * B.idx.size
        for c in far:
            key = id(c)
            if key not in cache:
                cache[key] = proxies(c, pts, w_s, w_m, degree)
            Pp, Ws, Wm = cache[key]
            ys.append(Pp)
            s.append(Ws)
            m.append(Wm)
            sid.append(np.full(Pp.shape[0], -1, dtype=np.int64))
            fp += Pp.shape[0] * B.idx.size
        nf += len(far)
        nn += len(near)
        t, b = general_sums(pts[B.idx], nrm[B.idx], np.concatenate(ys), np.concatenate(s),
                            np.concatenate(m), kappa, eps, skip=B.idx,
                            sid=np.concatenate(sid))
        top[B.idx] = t
        bot[B.idx] = b
    y = np.empty(2 * n_el)
    y[:n_el] = 0.5 * (1.0 + eps) * phi - top
    y[n_el:] = 0.5 * (1.0 + 1.0 / eps) * psi - bot
    if stats:
        return y, TreeStats(len(batches), len(cache), nf, nn, fp, np_)
    return y
