// Device arithmetic for one target/source pair of the boundary-integral
// operator (arXiv:1301.5885, Section 2.1 eq. (Eq_Ls), Section 2.2 eqs.
// (eqdbef1)/(eqdbef2)) on gfx950.
//
// Notation for a target x (unit normal nu_x) and a source y:
//   r = x - y, rho = |r|, tau = kappa rho, E = exp(-tau),
//   A = E (1 + tau), B = E (3 + 3 tau + tau^2), u_x = r . nu_x.
// With the 1/(4 pi) of G0/Gk moved into the source weights
//   s_j = W_j psi_j / (4 pi)          (psi = d phi_1 / d nu)
//   m_j = W_j phi_j nu_j / (4 pi)     (a vector: folds phi_j and nu_j)
// the two row sums of the product are
//   top_i = sum_j (1-E)/rho s_j + (eps A - 1)/rho^3 (r . m_j)
//         = sum_j W_j [K1 psi_j + K2 phi_j]
//   bot_i = sum_j -(1 - A/eps) u_x/rho^3 s_j + (A-1)/rho^3 (nu_x . m_j)
//                 - (B-3) u_x (r . m_j)/rho^5
//         = sum_j W_j [K3 psi_j + K4 phi_j]
// since 4 pi K1 = (1-E)/rho, 4 pi K2 = (eps A - 1) u_y/rho^3,
// 4 pi K3 = -(1 - A/eps) u_x/rho^3 and
// 4 pi K4 = (A-1) (nu_x . nu_y)/rho^3 - (B-3) u_x u_y/rho^5, u_y = r . nu_y.
#pragma once
#include <hip/hip_runtime.h>

namespace gabi {

// ---------------------------------------------------------------------------
// FP64 e^{-t} for t >= 0 (no FP64 exponential instruction exists on gfx950).
// Reduction e^{-t} = 2^k e^f with k = rint(-t / ln 2) and f = -t - k ln 2 in
// [-ln2/2, ln2/2], taken in two fused multiply-adds against ln 2 split into
// its double rounding and the rounding's remainder (Cody and Waite), so f
// carries an error of about one rounding for every k; then e^f by the
// degree-10 polynomial of least maximum relative error on that interval
// (coefficients from a Remez exchange computed for this code, relative error
// 2.1e-16 before rounding), then an exponent add.  Measured against a
// 64-bit-mantissa exponential over t in [0, 60]: at most 3 ulp, 1 ulp on
// average (the degree-12 Taylor form with a one-constant reduction it
// replaces: 18 ulp at most, one multiply-add more).  t is clamped to 746 so
// the exponent stays in range: e^{-t} < 2^-1075 for t > 745.14, which rounds
// to zero, and 2^k e^f at t = 746 (k = -1076) does.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double exp_neg_f64(double t) {
    t = fmin(t, 746.0);
    const double x = -t;
    const double kf = __builtin_rint(x * 1.4426950408889634074);  // x / ln2
    double f = __builtin_fma(-kf, 0x1.62e42fefa39efp-1, x);        // ln 2, rounded
    f = __builtin_fma(-kf, 0x1.abc9e3b39803fp-56, f);              // its remainder
    double p = 2.748844352290197084599319e-7;
    p = __builtin_fma(p, f, 2.763976825135432675936493e-6);
    p = __builtin_fma(p, f, 2.480191768787706887800884e-5);
    p = __builtin_fma(p, f, 1.984117138422559520510458e-4);
    p = __builtin_fma(p, f, 1.38888884991382898631281e-3);
    p = __builtin_fma(p, f, 8.333333384665794360899767e-3);
    p = __builtin_fma(p, f, 4.166666666842601715777246e-2);
    p = __builtin_fma(p, f, 1.666666666655774121978414e-1);
    p = __builtin_fma(p, f, 4.999999999999728701115992e-1);
    p = __builtin_fma(p, f, 1.000000000000006442614511);
    p = __builtin_fma(p, f, 1.000000000000000066064118);
    return __builtin_ldexp(p, (int)kf);
}

// FP64 1/sqrt(a) for a > 0: the hardware reciprocal square root estimate
// refined by one Newton-Raphson step y <- y + y (1 - a y^2) / 2, which
// squares the estimate's relative error.
__device__ __forceinline__ double rsqrt_f64(double a) {
    double y = __builtin_amdgcn_rsq(a);
    const double h = a * y;
    const double e = __builtin_fma(-h, y, 1.0);
    return __builtin_fma(0.5 * y, e, y);
}

// ---------------------------------------------------------------------------
// FP64 pair: accumulate the contributions of source j to target i.
//   (tx,ty,tz) target centroid, (tnx,tny,tnz) target normal,
//   (sx,sy,sz) source centroid, s = W psi/(4 pi), (mx,my,mz) = W phi nu/(4 pi)
// ---------------------------------------------------------------------------
struct PairConstF64 {
    double kappa, eps, inv_eps;
};

// Both precisions evaluate the row sums in the factored form
//   top += rinv [ (1-E) s + (eps A - 1) w rinv^2 ]
//   bot += rinv^3 [ u_x ((A/eps - 1) s - (B-3) w rinv^2) + (A-1) q_n ]
// with w = r . m_j and q_n = nu_x . m_j; (1-E) s, (A-1) q_n and B-3 are each
// formed by one fused multiply-add, so at kappa = 0 (E = A = 1, B = 3) the
// K1 and K4 contributions vanish exactly.
__device__ __forceinline__ void pair_f64(
    const PairConstF64 &c, double tx, double ty, double tz, double tnx,
    double tny, double tnz, double sx, double sy, double sz, double s,
    double mx, double my, double mz, double &top, double &bot) {
    const double dx = tx - sx, dy = ty - sy, dz = tz - sz;
    const double r2 = __builtin_fma(dx, dx, __builtin_fma(dy, dy, dz * dz));
    const double rinv = rsqrt_f64(r2);
    const double rinv2 = rinv * rinv;
    const double rinv3 = rinv2 * rinv;
    const double tau = c.kappa * (r2 * rinv);
    const double E = exp_neg_f64(tau);
    const double A = __builtin_fma(E, tau, E);                                  // E(1+tau)
    const double B3 = __builtin_fma(E, __builtin_fma(tau, tau + 3.0, 3.0), -3.0);  // B - 3
    const double ux = __builtin_fma(dx, tnx, __builtin_fma(dy, tny, dz * tnz));
    const double w = __builtin_fma(dx, mx, __builtin_fma(dy, my, dz * mz));
    const double qn = __builtin_fma(tnx, mx, __builtin_fma(tny, my, tnz * mz));
    const double k1 = __builtin_fma(-E, s, s);                                  // (1-E) s
    const double k2 = __builtin_fma(c.eps, A, -1.0) * w;                        // (eps A-1) w
    top = __builtin_fma(__builtin_fma(k2, rinv2, k1), rinv, top);
    const double k3 = __builtin_fma(__builtin_fma(A, c.inv_eps, -1.0), s, -(B3 * rinv2) * w);
    const double k4 = __builtin_fma(A, qn, -qn);                                // (A-1) q_n
    bot = __builtin_fma(__builtin_fma(ux, k3, k4), rinv3, bot);
}

// ---------------------------------------------------------------------------
// FP32 pair (the mixed product): coordinates relative to the molecule's
// bounding-box centre rounded once to FP32, the same factored form in FP32
// with the hardware exp2 and reciprocal-square-root instructions.
// ---------------------------------------------------------------------------
struct PairConstF32 {
    float kappa, neg_kappa_log2e, eps, inv_eps;
};

__device__ __forceinline__ void pair_f32(
    const PairConstF32 &c, float tx, float ty, float tz, float tnx,
    float tny, float tnz, float sx, float sy, float sz, float s, float mx,
    float my, float mz, float &top, float &bot) {
    const float dx = tx - sx, dy = ty - sy, dz = tz - sz;
    const float r2 = __builtin_fmaf(dx, dx, __builtin_fmaf(dy, dy, dz * dz));
    const float rinv = __builtin_amdgcn_rsqf(r2);
    const float rinv2 = rinv * rinv;
    const float rinv3 = rinv2 * rinv;
    const float rho = r2 * rinv;
    const float tau = c.kappa * rho;
    const float E = __builtin_amdgcn_exp2f(rho * c.neg_kappa_log2e);
    const float A = __builtin_fmaf(E, tau, E);
    const float B3 = __builtin_fmaf(E, __builtin_fmaf(tau, tau + 3.0f, 3.0f), -3.0f);
    const float ux = __builtin_fmaf(dx, tnx, __builtin_fmaf(dy, tny, dz * tnz));
    const float w = __builtin_fmaf(dx, mx, __builtin_fmaf(dy, my, dz * mz));
    const float qn = __builtin_fmaf(tnx, mx, __builtin_fmaf(tny, my, tnz * mz));
    const float k1 = __builtin_fmaf(-E, s, s);
    const float k2 = __builtin_fmaf(c.eps, A, -1.0f) * w;
    top = __builtin_fmaf(__builtin_fmaf(k2, rinv2, k1), rinv, top);
    const float k3 = __builtin_fmaf(__builtin_fmaf(A, c.inv_eps, -1.0f), s, -(B3 * rinv2) * w);
    const float k4 = __builtin_fmaf(A, qn, -qn);
    bot = __builtin_fmaf(__builtin_fmaf(ux, k3, k4), rinv3, bot);
}

// ---------------------------------------------------------------------------
// Symmetric evaluation: one unordered pair of elements a (target i) and b
// (target j) gives both the (target i, source j) and the (target j, source i)
// terms.  With m = t nu (t = W phi / (4 pi)) and d = x_i - x_j:
//   d . m_j = t_j u_j,  nu_i . m_j = t_j n,  d . m_i = t_i u_x,
//   nu_j . m_i = t_i n,  u_x = d . nu_i, u_j = d . nu_j, n = nu_i . nu_j,
// and the (j, i) term uses the separation -d.  Written with the factors
//   P = (1-E) rinv,  Q = (eps A - 1) rinv^3,  R = (A/eps - 1) rinv^3,
//   Y = rinv^3 [(A-1) n - (B-3) rinv^2 u_x u_j],
// which the two terms share, the four sums are
//   top_i += P s_j + (Q u_j) t_j,      bot_i += (R u_x) s_j + Y t_j,
//   top_j += P s_i - (Q u_x) t_i,      bot_j += -(R u_j) s_i + Y t_i,
// the same quantities as bot = rinv^3 [u_x ((A/eps-1) s - (B-3) w rinv^2)
// + (A-1) q_n] of the pair form with w = t u_j, q_n = t n.
// The (i, j) terms accumulate into top/bot, the (j, i) terms into ctop/cbot.
// ---------------------------------------------------------------------------
template <typename T>
struct SymElem {  // one element as a target and as a source
    T x, y, z, nx, ny, nz, s, t;
};

__device__ __forceinline__ void sym_f64(const PairConstF64 &c, const SymElem<double> &a,
                                        const SymElem<double> &b, double &top, double &bot,
                                        double &ctop, double &cbot) {
    const double dx = a.x - b.x, dy = a.y - b.y, dz = a.z - b.z;
    const double r2 = __builtin_fma(dx, dx, __builtin_fma(dy, dy, dz * dz));
    const double rinv = rsqrt_f64(r2);
    const double rinv2 = rinv * rinv;
    const double rinv3 = rinv2 * rinv;
    const double tau = c.kappa * (r2 * rinv);
    const double E = exp_neg_f64(tau);
    const double A = __builtin_fma(E, tau, E);
    const double B3 = __builtin_fma(E, __builtin_fma(tau, tau + 3.0, 3.0), -3.0);
    const double ux = __builtin_fma(dx, a.nx, __builtin_fma(dy, a.ny, dz * a.nz));
    const double uj = __builtin_fma(dx, b.nx, __builtin_fma(dy, b.ny, dz * b.nz));
    const double nn = __builtin_fma(a.nx, b.nx, __builtin_fma(a.ny, b.ny, a.nz * b.nz));
    const double P = __builtin_fma(-E, rinv, rinv);
    const double Q = __builtin_fma(c.eps, A, -1.0) * rinv3;
    const double R = __builtin_fma(A, c.inv_eps, -1.0) * rinv3;
    const double Bu = (B3 * rinv2) * ux;
    const double Y = __builtin_fma(-Bu, uj, __builtin_fma(A, nn, -nn)) * rinv3;
    top = __builtin_fma(P, b.s, __builtin_fma(Q * uj, b.t, top));
    bot = __builtin_fma(R * ux, b.s, __builtin_fma(Y, b.t, bot));
    ctop = __builtin_fma(P, a.s, __builtin_fma(-(Q * ux), a.t, ctop));
    cbot = __builtin_fma(-(R * uj), a.s, __builtin_fma(Y, a.t, cbot));
}

__device__ __forceinline__ void sym_f32(const PairConstF32 &c, const SymElem<float> &a,
                                        const SymElem<float> &b, float &top, float &bot,
                                        float &ctop, float &cbot) {
    const float dx = a.x - b.x, dy = a.y - b.y, dz = a.z - b.z;
    const float r2 = __builtin_fmaf(dx, dx, __builtin_fmaf(dy, dy, dz * dz));
    const float rinv = __builtin_amdgcn_rsqf(r2);
    const float rinv2 = rinv * rinv;
    const float rinv3 = rinv2 * rinv;
    const float rho = r2 * rinv;
    const float tau = c.kappa * rho;
    const float E = __builtin_amdgcn_exp2f(rho * c.neg_kappa_log2e);
    const float A = __builtin_fmaf(E, tau, E);
    const float B3 = __builtin_fmaf(E, __builtin_fmaf(tau, tau + 3.0f, 3.0f), -3.0f);
    const float ux = __builtin_fmaf(dx, a.nx, __builtin_fmaf(dy, a.ny, dz * a.nz));
    const float uj = __builtin_fmaf(dx, b.nx, __builtin_fmaf(dy, b.ny, dz * b.nz));
    const float nn = __builtin_fmaf(a.nx, b.nx, __builtin_fmaf(a.ny, b.ny, a.nz * b.nz));
    const float P = __builtin_fmaf(-E, rinv, rinv);
    const float Q = __builtin_fmaf(c.eps, A, -1.0f) * rinv3;
    const float R = __builtin_fmaf(A, c.inv_eps, -1.0f) * rinv3;
    const float Bu = (B3 * rinv2) * ux;
    const float Y = __builtin_fmaf(-Bu, uj, __builtin_fmaf(A, nn, -nn)) * rinv3;
    top = __builtin_fmaf(P, b.s, __builtin_fmaf(Q * uj, b.t, top));
    bot = __builtin_fmaf(R * ux, b.s, __builtin_fmaf(Y, b.t, bot));
    ctop = __builtin_fmaf(P, a.s, __builtin_fmaf(-(Q * ux), a.t, ctop));
    cbot = __builtin_fmaf(-(R * uj), a.s, __builtin_fmaf(Y, a.t, cbot));
}

}  // namespace gabi
