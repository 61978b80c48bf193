// Charge-dependent O(N Nc) terms of arXiv:1301.5885 on gfx950:
//   right-hand side (Section 2.1, eq. (Eq_Ss); Section 2.2)
//     b_i     =  sum_k q_k G0(x_i, y_k) / eps1 = sum_k q_k / (4 pi eps1 rho)
//     b_{N+i} =  sum_k q_k dG0(x_i, y_k)/dnu_x / eps1
//             = -sum_k q_k (x_i - y_k).nu_i / (4 pi eps1 rho^3)
//   reaction potential and solvation energy (Section 2.3,
//   eq. (solvation_energy))
//     phi_reac(y_k) = sum_j W_j [K1(y_k, x_j) psi_j + K2(y_k, x_j) phi_j]
//     E_sol = 1/2 sum_k q_k phi_reac(y_k)   (x 4 pi 332.0716 for kcal/mol)
// Charges are staged through LDS in tiles of 256 records (x, y, z, q).
#include "gabi_internal.h"
#include "pair_math.h"
#include "reduce.h"

namespace gabi {

__global__ __launch_bounds__(kBlock) void rhs_kernel(
    int n, int nc, const double4 *__restrict__ pos,
    const double4 *__restrict__ nrm, const double4 *__restrict__ chg,
    double scale, double *__restrict__ b) {
    __shared__ double4 s_c[kTile];
    const int tid = threadIdx.x;
    const int i = blockIdx.x * kBlock + tid;
    const int ic = min(i, n - 1);
    const double4 x = pos[ic];
    const double4 nu = nrm[ic];
    double s1 = 0.0, s2 = 0.0;
    for (int kt = 0; kt < nc; kt += kTile) {
        const int cnt = min(kTile, nc - kt);
        __syncthreads();
        if (tid < cnt) s_c[tid] = chg[kt + tid];
        __syncthreads();
        for (int kk = 0; kk < cnt; ++kk) {
            const double4 c = s_c[kk];
            const double dx = x.x - c.x, dy = x.y - c.y, dz = x.z - c.z;
            const double r2 = __builtin_fma(dx, dx, __builtin_fma(dy, dy, dz * dz));
            const double rinv = rsqrt_f64(r2);
            const double ux = __builtin_fma(dx, nu.x, __builtin_fma(dy, nu.y, dz * nu.z));
            s1 = __builtin_fma(c.w, rinv, s1);
            s2 = __builtin_fma(c.w * ux, rinv * rinv * rinv, s2);
        }
    }
    if (i < n) {
        b[i] = s1 * scale;
        b[n + i] = -s2 * scale;
    }
}

void launch_rhs(gabi_ctx *ctx, double *b) {
    const int n = (int)ctx->n;
    const int nc = (int)ctx->nc;
    const double scale = 1.0 / (4.0 * kPi * ctx->eps1);
    hipLaunchKernelGGL(rhs_kernel, dim3((n + kBlock - 1) / kBlock),
                       dim3(kBlock), 0, ctx->stream, n, nc, ctx->pos,
                       ctx->nrm, ctx->chg, scale, b);
}

// Reaction potential: thread = charge (target), workgroup column = one split
// of the surface elements (sources), partial sums [split][nc].
__global__ __launch_bounds__(kBlock) void reaction_kernel(
    int n, int nc, int tiles_per_split, const double4 *__restrict__ pos,
    const double4 *__restrict__ w64, const double4 *__restrict__ chg,
    PairConstF64 c, double *__restrict__ part) {
    __shared__ double4 s_pos[kTile];
    __shared__ double4 s_w[kTile];
    const int tid = threadIdx.x;
    const int k = blockIdx.x * kBlock + tid;
    const double4 y = chg[min(k, nc - 1)];
    double acc = 0.0;
    const int j_begin = blockIdx.y * tiles_per_split * kTile;
    for (int tile = 0; tile < tiles_per_split; ++tile) {
        const int jt = j_begin + tile * kTile;
        if (jt >= n) break;
        const int cnt = min(kTile, n - jt);
        __syncthreads();
        if (tid < cnt) {
            s_pos[tid] = pos[jt + tid];
            s_w[tid] = w64[jt + tid];
        }
        __syncthreads();
        for (int jj = 0; jj < cnt; ++jj) {
            const double4 p = s_pos[jj];
            const double4 w = s_w[jj];
            const double dx = y.x - p.x, dy = y.y - p.y, dz = y.z - p.z;
            const double r2 = __builtin_fma(dx, dx, __builtin_fma(dy, dy, dz * dz));
            const double rinv = rsqrt_f64(r2);
            const double rho = r2 * rinv;
            const double tau = c.kappa * rho;
            const double E = exp_neg_f64(tau);
            const double A = __builtin_fma(E, tau, E);
            const double wm = __builtin_fma(dx, w.y, __builtin_fma(dy, w.z, dz * w.w));
            const double k1s = __builtin_fma(-E, w.x, w.x) * rinv;
            acc += __builtin_fma(__builtin_fma(c.eps, A, -1.0) * rinv * rinv * rinv,
                                 wm, k1s);
        }
    }
    if (k < nc) part[(size_t)blockIdx.y * nc + k] = acc;
}

__global__ __launch_bounds__(kBlock) void reaction_finish_kernel(
    int nc, int splits, const double *__restrict__ part,
    const double4 *__restrict__ chg, double *__restrict__ phi,
    double *__restrict__ energy) {
    __shared__ double lds[kBlock / 64];
    double e = 0.0;
    for (int k = threadIdx.x; k < nc; k += kBlock) {
        double s = 0.0;
        for (int sp = 0; sp < splits; ++sp) s += part[(size_t)sp * nc + k];
        if (phi) phi[k] = s;
        e = __builtin_fma(chg[k].w, s, e);
    }
    const double tot = block_sum(e, lds);
    if (threadIdx.x == 0 && energy) energy[0] = 0.5 * tot * 4.0 * kPi * kCoulomb;
}

int launch_reaction(gabi_ctx *ctx, double *phi, double *energy_out) {
    const int n = (int)ctx->n;
    const int nc = (int)ctx->nc;
    if (nc == 0) {
        if (energy_out) GABI_HIP(ctx, hipMemsetAsync(energy_out, 0, sizeof(double), ctx->stream));
        return GABI_OK;
    }
    const int kblocks = (nc + kBlock - 1) / kBlock;
    const int tiles = (n + kTile - 1) / kTile;
    int want = (1024 + kblocks - 1) / kblocks;
    if (want < 1) want = 1;
    int tps = (tiles + want - 1) / want;
    if (tps < 1) tps = 1;
    const int splits = (tiles + tps - 1) / tps;
    const int64_t need = (int64_t)splits * nc;
    if (need > ctx->phi_part_len) {
        dev_free(ctx, (void **)&ctx->phi_part, ctx->phi_part_len * sizeof(double));
        ctx->phi_part_len = 0;
        int rc = dev_alloc(ctx, (void **)&ctx->phi_part, need * sizeof(double));
        if (rc) return rc;
        ctx->phi_part_len = need;
    }
    const double eps = ctx->eps2 / ctx->eps1;
    PairConstF64 c{ctx->kappa, eps, 1.0 / eps};
    hipLaunchKernelGGL(reaction_kernel, dim3(kblocks, splits), dim3(kBlock), 0,
                       ctx->stream, n, nc, tps, ctx->pos, ctx->wgt, ctx->chg,
                       c, ctx->phi_part);
    hipLaunchKernelGGL(reaction_finish_kernel, dim3(1), dim3(kBlock), 0,
                       ctx->stream, nc, splits, ctx->phi_part, ctx->chg, phi,
                       energy_out);
    GABI_HIP(ctx, hipGetLastError());
    return GABI_OK;
}

}  // namespace gabi
