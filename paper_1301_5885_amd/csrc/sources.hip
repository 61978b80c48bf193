// Charge-dependent O(N Nc) terms of arXiv:1301.5885 on gfx950, for a batch
// of molecules:
//   right-hand side (Section 2.1, eq. (Eq_Ss); Section 2.2)
//     b_i     =  sum_k q_k G0(x_i, y_k) / eps1 = sum_k q_k / (4 pi eps1 rho)
//     b_{N+i} =  sum_k q_k dG0(x_i, y_k)/dnu_x / eps1
//             = -sum_k q_k (x_i - y_k).nu_i / (4 pi eps1 rho^3)
//   reaction potential and solvation energy (Section 2.3,
//   eq. (solvation_energy))
//     phi_reac(y_k) = sum_j W_j [K1(y_k, x_j) psi_j + K2(y_k, x_j) phi_j]
//     E_sol = 1/2 sum_k q_k phi_reac(y_k)   (x 4 pi 332.0716 for kcal/mol)
// Charges (rhs) or surface elements (reaction) are staged through LDS in
// tiles of 256 records.
#include "gabi_internal.h"
#include "pair_math.h"
#include "reduce.h"

namespace gabi {

// Right-hand side: workgroup = 64 elements of a 256-element block (the block
// list entry blockIdx.x / 4, quarter blockIdx.x % 4); lane l of wave q takes
// element l and the charges q, q + 4, ... of every 256 staged; the four
// waves' sums of an element are added in wave order.
__global__ __launch_bounds__(kBlock) void rhs_kernel(const Mol *__restrict__ mols,
                                                     const int2 *__restrict__ list) {
    __shared__ double4 s_c[kTile];
    __shared__ double s_acc[2][kBlock];
    const int2 e = list[blockIdx.x / 4];
    const Mol &M = mols[e.x];
    const int n = M.n, nc = M.nc;
    const int tid = threadIdx.x, lane = tid & 63, q = tid >> 6;
    const int i = e.y * kBlock + (int)(blockIdx.x % 4) * 64 + lane;
    const int ic = min(i, n - 1);
    const double4 x = M.pos[ic];
    const double4 nu = M.nrm[ic];
    double s1 = 0.0, s2 = 0.0;
    for (int kt = 0; kt < nc; kt += kTile) {
        const int cnt = min(kTile, nc - kt);
        __syncthreads();
        if (tid < cnt) s_c[tid] = M.chg[kt + tid];
        __syncthreads();
        for (int kk = q; kk < cnt; kk += 4) {
            const double4 c = s_c[kk];
            const double dx = x.x - c.x, dy = x.y - c.y, dz = x.z - c.z;
            const double r2 = __builtin_fma(dx, dx, __builtin_fma(dy, dy, dz * dz));
            const double rinv = rsqrt_f64(r2);
            const double ux = __builtin_fma(dx, nu.x, __builtin_fma(dy, nu.y, dz * nu.z));
            s1 = __builtin_fma(c.w, rinv, s1);
            s2 = __builtin_fma(c.w * ux, rinv * rinv * rinv, s2);
        }
    }
    s_acc[0][tid] = s1;
    s_acc[1][tid] = s2;
    __syncthreads();
    if (q == 0 && i < n) {
        const double t1 = ((s_acc[0][lane] + s_acc[0][64 + lane]) + s_acc[0][128 + lane]) +
                          s_acc[0][192 + lane];
        const double t2 = ((s_acc[1][lane] + s_acc[1][64 + lane]) + s_acc[1][128 + lane]) +
                          s_acc[1][192 + lane];
        M.rhs_dst[i] = t1 * M.rhs_scale;
        M.rhs_dst[n + i] = -t2 * M.rhs_scale;
    }
}

void launch_rhs(const Batch &b, hipStream_t s) {
    hipLaunchKernelGGL(rhs_kernel, dim3(4 * b.n_elem), dim3(kBlock), 0, s, b.d_mols, b.d_elem);
}

// Reaction potential: tile = (molecule, block of 64 charges, split of the
// surface elements); partial sums [split][nc].  Lane l of wave q takes charge
// l of the block and, of every 256 staged elements, the 64 elements
// q*64 .. q*64+63; the four waves' sums of a charge are added in wave order.
// The source weights s_j = W_j psi_j/(4 pi), m_j = W_j phi_j nu_j/(4 pi) of the
// evaluated vector (the solution or the product input u) are formed while the
// sources are staged, independent of the layout the products use.
constexpr int kRxCharges = 64;  // charges per reaction tile
static_assert(kBlock == 4 * kRxCharges && kTile == kBlock, "four waves of 64 charges");

__global__ __launch_bounds__(kBlock) void reaction_kernel(const Mol *__restrict__ mols,
                                                          const int4 *__restrict__ list,
                                                          int from_sol) {
    __shared__ double4 s_pos[kTile];
    __shared__ double4 s_w[kTile];
    __shared__ double s_acc[kBlock];
    const int4 e = list[blockIdx.x];
    const Mol &M = mols[e.x];
    const int n = M.n, nc = M.nc;
    const int tid = threadIdx.x, lane = tid & 63, q = tid >> 6;
    const int k = e.y * kRxCharges + lane;
    const double4 y = M.chg[min(k, nc - 1)];
    const PairConstF64 c{M.kappa, M.eps, M.inv_eps};
    double acc = 0.0;
    const int j_begin = e.z * M.rx_tps * kTile;
    for (int tile = 0; tile < M.rx_tps; ++tile) {
        const int jt = j_begin + tile * kTile;
        if (jt >= n) break;
        const int cnt = min(kTile, n - jt);
        __syncthreads();
        if (tid < cnt) {
            const double *u = from_sol ? M.sol : M.u;
            const double4 p = M.pos[jt + tid];
            const double4 nu = M.nrm[jt + tid];
            const double c = p.w * (1.0 / (4.0 * kPi));
            const double t = c * u[jt + tid];
            s_pos[tid] = p;
            s_w[tid] = make_double4(c * u[n + jt + tid], t * nu.x, t * nu.y, t * nu.z);
        }
        __syncthreads();
        const int j1 = min(cnt, (q + 1) * 64);
        for (int jj = q * 64; jj < j1; ++jj) {
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
            acc += __builtin_fma(__builtin_fma(c.eps, A, -1.0) * rinv * rinv * rinv, wm, k1s);
        }
    }
    s_acc[tid] = acc;
    __syncthreads();
    if (q == 0 && k < nc)
        M.phi_part[(size_t)e.z * nc + k] =
            ((s_acc[lane] + s_acc[64 + lane]) + s_acc[128 + lane]) + s_acc[192 + lane];
}

// one workgroup per molecule: phi_reac = sum over splits, E = 1/2 sum q phi
__global__ __launch_bounds__(kBlock) void reaction_finish_kernel(const Mol *__restrict__ mols) {
    __shared__ double lds[kBlock / 64];
    const Mol &M = mols[blockIdx.x];
    const int nc = M.nc;
    double e = 0.0;
    for (int k = threadIdx.x; k < nc; k += kBlock) {
        // in split order; eight reads are issued ahead of their sums
        double s = 0.0;
        int sp = 0;
        for (; sp + 8 <= M.rx_splits; sp += 8) {
            double a[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) a[q] = M.phi_part[(size_t)(sp + q) * nc + k];
#pragma unroll
            for (int q = 0; q < 8; ++q) s += a[q];
        }
        for (; sp < M.rx_splits; ++sp) s += M.phi_part[(size_t)sp * nc + k];
        M.phi[k] = s;
        e = __builtin_fma(M.chg[k].w, s, e);
    }
    const double tot = block_sum(e, lds);
    if (threadIdx.x == 0) M.st->energy = 0.5 * tot * 4.0 * kPi * kCoulomb;
}

void launch_reaction(const Batch &b, hipStream_t s, bool from_sol) {
    if (b.n_rx > 0)
        hipLaunchKernelGGL(reaction_kernel, dim3(b.n_rx), dim3(kBlock), 0, s, b.d_mols, b.d_rx,
                           (int)from_sol);
    hipLaunchKernelGGL(reaction_finish_kernel, dim3((int)b.slots.size()), dim3(kBlock), 0, s,
                       b.d_mols);
}

}  // namespace gabi
