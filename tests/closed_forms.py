"""Closed-form references used to pin the CPU oracle (test helpers).

Nothing here is the boundary-integral method itself; these are independent
analytic results that the discrete method must approach as the mesh is
refined (Section 3.1 of arXiv:1301.5885 measures error against such
solutions):

* Born ion: a point charge at the centre of a dielectric sphere.
* Kirkwood's spherical-harmonic series for charges inside a sphere with a
  screened exterior (the analytic reference of Section 3.2).  The paper does
  not print the series; it is derived here from the interface conditions
  (eq1)-(radiation): inside, Coulomb plus sum_n B_n r^n P_n; outside,
  C_n k_n(kappa r) P_n; continuity of phi and eps dphi/dr at r = a gives
      B_n = [eps1 (n+1) + eps2 g_n] / [eps1 n - eps2 g_n],
      g_n = z k_n'(z) / k_n(z), z = kappa a,
  with k_n the modified spherical Bessel function of the second kind.
* Integrals of the kernels over a sphere of radius a for a point on it,
  with the chord rho as variable: dS = 2 pi rho drho on [0, 2a],
  (x-y).nu_y = -rho^2/(2a), (x-y).nu_x = rho^2/(2a), nu_x.nu_y = 1 - rho^2/(2a^2).

Units follow the oracle: charges in e, potentials carry 1/(4 pi), energies in
kcal/mol via 4 pi * 332.0716.
"""
from __future__ import annotations

import math

import numpy as np

COULOMB = 332.0716
FOURPI = 4.0 * math.pi


# ------------------------------------------------------------------ Born
def born_surface(a, q=1.0, eps1=1.0, eps2=80.0, kappa=0.0):
    """(phi, dphi1/dnu) on the sphere for a central charge q."""
    phi = q / (FOURPI * eps2 * a * (1.0 + kappa * a))
    psi = -q / (FOURPI * eps1 * a * a)
    return phi, psi


def born_energy(a, q=1.0, eps1=1.0, eps2=80.0, kappa=0.0):
    """Solvation energy (kcal/mol) of a central charge q in a sphere."""
    phi_reac = q / (FOURPI * a) * (1.0 / (eps2 * (1.0 + kappa * a)) - 1.0 / eps1)
    return 0.5 * q * phi_reac * FOURPI * COULOMB


# -------------------------------------------------------------- Kirkwood
def kirkwood_g(nmax, z):
    """g_n = z k_n'(z)/k_n(z), n = 0..nmax, by the ratio recurrence."""
    n = np.arange(nmax + 1)
    if z == 0.0:
        return -(n + 1.0)
    g = np.empty(nmax + 1)
    g[0] = -(1.0 + z)
    t = 1.0 + 1.0 / z          # k_1 / k_0
    for k in range(1, nmax + 1):
        if k > 1:
            t = 1.0 / t + (2.0 * k - 1.0) / z   # k_k / k_{k-1}
        g[k] = -z / t - (k + 1.0)
    return g


def kirkwood_B(nmax, a, eps1, eps2, kappa):
    n = np.arange(nmax + 1, dtype=np.float64)
    g = kirkwood_g(nmax, kappa * a)
    return (eps1 * (n + 1.0) + eps2 * g) / (eps1 * n - eps2 * g)


def _legendre_sum(coef, x, w):
    """sum_n coef[n] * w^n * P_n(x), elementwise over arrays x, w."""
    p0 = np.ones_like(x)
    p1 = x.copy()
    wn = np.ones_like(x)
    s = coef[0] * p0
    if len(coef) > 1:
        wn = wn * w
        s = s + coef[1] * wn * p1
    for n in range(1, len(coef) - 1):
        p2 = ((2 * n + 1) * x * p1 - n * p0) / (n + 1)
        wn = wn * w
        s = s + coef[n + 1] * wn * p2
        p0, p1 = p1, p2
    return s


def _nterms(ratio, tol=1e-17):
    if ratio <= 0.0:
        return 1
    return int(min(4000, max(2, math.ceil(math.log(tol) / math.log(ratio)) + 2)))


def kirkwood_reaction_potential(pos, q, a, eps1=1.0, eps2=80.0, kappa=0.0):
    """phi_reac at each charge position (charges at pos, inside r < a)."""
    pos = np.atleast_2d(np.asarray(pos, float))
    q = np.asarray(q, float)
    r = np.linalg.norm(pos, axis=1)
    w = np.outer(r, r) / (a * a)                   # (j, k)
    with np.errstate(invalid="ignore", divide="ignore"):
        cosg = (pos @ pos.T) / np.outer(r, r)
    cosg = np.where(np.outer(r, r) > 0, np.clip(cosg, -1, 1), 1.0)
    nmax = _nterms(w.max())
    B = kirkwood_B(nmax, a, eps1, eps2, kappa)
    S = _legendre_sum(B, cosg, w) / a              # (j, k)
    return (S @ q) / (FOURPI * eps1)


def kirkwood_energy(pos, q, a, eps1=1.0, eps2=80.0, kappa=0.0):
    phi = kirkwood_reaction_potential(pos, q, a, eps1, eps2, kappa)
    return 0.5 * float(np.dot(q, phi)) * FOURPI * COULOMB


def kirkwood_surface(points, pos, q, a, eps1=1.0, eps2=80.0, kappa=0.0):
    """(phi, dphi1/dnu) at the directions of ``points`` on the sphere r = a."""
    pts = np.atleast_2d(np.asarray(points, float))
    u = pts / np.linalg.norm(pts, axis=1, keepdims=True)
    pos = np.atleast_2d(np.asarray(pos, float))
    q = np.asarray(q, float)
    rk = np.linalg.norm(pos, axis=1)
    with np.errstate(invalid="ignore", divide="ignore"):
        cosg = (u @ pos.T) / rk[None, :]
    cosg = np.where(rk[None, :] > 0, np.clip(cosg, -1, 1), 1.0)
    w = np.broadcast_to(rk[None, :] / a, cosg.shape)
    nmax = _nterms(float(w.max()))
    B = kirkwood_B(nmax, a, eps1, eps2, kappa)
    n = np.arange(nmax + 1, dtype=np.float64)
    phi = _legendre_sum(1.0 + B, cosg, w) / a
    psi = _legendre_sum(n * B - (n + 1.0), cosg, w) / (a * a)
    return (phi @ q) / (FOURPI * eps1), (psi @ q) / (FOURPI * eps1)


# ------------------------------------------------- sphere kernel integrals
def sphere_kernel_integrals(a, kappa, eps):
    """Integrals of K1..K4 over the sphere r = a for x on the sphere.

    K1 = G0 - Gk, K2 = eps dGk/dnu_y - dG0/dnu_y, K3 = dG0/dnu_x -
    (1/eps) dGk/dnu_x, K4 = d2Gk - d2G0 (Section 2.1 with eps = eps2/eps1),
    integrated in closed form where one exists and by adaptive quadrature
    over the chord for K4.
    """
    from scipy.integrate import quad
    iG0 = a
    iGk = (1.0 - math.exp(-2.0 * kappa * a)) / (2.0 * kappa) if kappa else a
    iG0n = -0.5                            # both d/dnu_y and d/dnu_x
    if kappa:
        iGkn = -(2.0 / kappa - math.exp(-2 * kappa * a) * (2.0 / kappa + 2 * a)) / (4 * a)
    else:
        iGkn = -0.5

    def k4(rho):
        e = math.exp(-kappa * rho)
        A = e * (1 + kappa * rho)
        Bc = e * (3 + 3 * kappa * rho + (kappa * rho) ** 2)
        nn = 1 - rho * rho / (2 * a * a)
        uxuy = -rho ** 4 / (4 * a * a)
        k = ((A - 1) * nn / rho ** 3 - (Bc - 3) * uxuy / rho ** 5) / FOURPI
        return 2 * math.pi * rho * k

    iK4 = quad(k4, 0.0, 2 * a, epsabs=1e-14, epsrel=1e-13, limit=200)[0]
    # dG/dnu_y = dGdnu_x on the sphere (u_y = -u_x), so
    iK1 = iG0 - iGk
    iK2 = eps * iGkn - iG0n
    iK3 = iG0n - iGkn / eps
    return iK1, iK2, iK3, iK4


def rotation(rng):
    """Random proper rotation matrix."""
    qm, r = np.linalg.qr(rng.normal(size=(3, 3)))
    qm = qm * np.sign(np.diag(r))
    if np.linalg.det(qm) < 0:
        qm[:, 0] = -qm[:, 0]
    return qm
