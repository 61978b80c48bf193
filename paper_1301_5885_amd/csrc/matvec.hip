// The discrete boundary-integral product y = A u of arXiv:1301.5885,
// Section 2.2, eqs. (eqdbef1)/(eqdbef2), on gfx950.
//
//   y_i     = (1+eps)/2 phi_i   - sum_{j != i} W_j [K1 psi_j + K2 phi_j]
//   y_{N+i} = (1+1/eps)/2 psi_i - sum_{j != i} W_j [K3 psi_j + K4 phi_j]
//
// Three launches per product:
//   prep    O(N): source weights s_j = W_j psi_j/(4 pi) and
//           m_j = W_j phi_j nu_j/(4 pi) (FP64, or FP32 for the mixed path);
//   pair    O(N^2): each thread holds R target rows in registers; a
//           workgroup streams one split of the sources through LDS in
//           tiles of 256 (coalesced 32-byte records, broadcast reads), and
//           writes its two row sums per target to a partial buffer;
//   finish  O(N S): adds the S split partials in split order and applies
//           the diagonal.
// The split count S depends only on N and the precision, so a product's
// summation order is fixed (bitwise reproducible).  The self term j = i is
// skipped exactly: only the tiles that overlap the workgroup's own rows run
// the masked loop.
#include "gabi_internal.h"
#include "pair_math.h"

namespace gabi {

// ------------------------------------------------------------------ config
PairLaunch pair_launch(int64_t n, int precision) {
    PairLaunch L;
    L.rows_per_thread = (n >= 8192) ? 2 : 1;
    const int64_t rows_per_block = (int64_t)kBlock * L.rows_per_thread;
    L.row_blocks = (int)((n + rows_per_block - 1) / rows_per_block);
    const int64_t tiles = (n + kTile - 1) / kTile;
    const int64_t target_blocks = 2048;  // about 8 workgroups per CU
    int64_t want_splits = (target_blocks + L.row_blocks - 1) / L.row_blocks;
    if (want_splits < 1) want_splits = 1;
    int64_t tps = (tiles + want_splits - 1) / want_splits;
    if (tps < 1) tps = 1;
    L.tiles_per_split = (int)tps;
    L.splits = (int)((tiles + tps - 1) / tps);
    (void)precision;
    return L;
}

// ------------------------------------------------------------------ prep
__global__ __launch_bounds__(kBlock) void prep_kernel(
    int n, const double4 *__restrict__ pos, const double4 *__restrict__ nrm,
    const double *__restrict__ u, const double *__restrict__ scale,
    double *__restrict__ store, double4 *__restrict__ w64,
    float4 *__restrict__ w32, const int32_t *__restrict__ skip) {
    if (skip && *skip) return;
    const int j = blockIdx.x * kBlock + threadIdx.x;
    if (j >= n) return;
    double phi = u[j], psi = u[n + j];
    if (scale) {
        const double h = *scale;
        phi = phi / h;
        psi = psi / h;
    }
    if (store) {
        store[j] = phi;
        store[n + j] = psi;
    }
    const double4 p = pos[j];
    const double4 nu = nrm[j];
    const double c = p.w * (1.0 / (4.0 * kPi));
    const double s = c * psi;
    const double t = c * phi;
    if (w64) w64[j] = make_double4(s, t * nu.x, t * nu.y, t * nu.z);
    if (w32)
        w32[j] = make_float4((float)s, (float)(t * nu.x), (float)(t * nu.y),
                             (float)(t * nu.z));
}

// ------------------------------------------------------------------ pair
template <int R, bool MIXED>
__global__ __launch_bounds__(kBlock) void pair_kernel(
    int n, int tiles_per_split, const double4 *__restrict__ pos,
    const double4 *__restrict__ nrm, const float4 *__restrict__ nrm32,
    const double4 *__restrict__ w64, const float4 *__restrict__ w32,
    PairConstF64 c64, PairConstF32 c32, double *__restrict__ part,
    const int32_t *__restrict__ skip) {
    if (skip && *skip) return;
    __shared__ double4 s_pos[kTile];
    __shared__ double4 s_w64[MIXED ? 1 : kTile];
    __shared__ float4 s_w32[MIXED ? kTile : 1];

    const int tid = threadIdx.x;
    const int row0 = blockIdx.x * kBlock * R;
    const int row_end = min(n, row0 + kBlock * R);

    double tx[R], ty[R], tz[R];
    double tnx[R], tny[R], tnz[R];
    float fnx[R], fny[R], fnz[R];
    double top[R], bot[R];
    int ti[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int i = row0 + r * kBlock + tid;
        ti[r] = i;
        const int ic = min(i, n - 1);
        const double4 p = pos[ic];
        tx[r] = p.x;
        ty[r] = p.y;
        tz[r] = p.z;
        if constexpr (MIXED) {
            const float4 q = nrm32[ic];
            fnx[r] = q.x;
            fny[r] = q.y;
            fnz[r] = q.z;
        } else {
            const double4 q = nrm[ic];
            tnx[r] = q.x;
            tny[r] = q.y;
            tnz[r] = q.z;
        }
        top[r] = 0.0;
        bot[r] = 0.0;
    }

    const int j_begin = blockIdx.y * tiles_per_split * kTile;
    for (int tile = 0; tile < tiles_per_split; ++tile) {
        const int jt = j_begin + tile * kTile;
        if (jt >= n) break;
        const int cnt = min(kTile, n - jt);
        __syncthreads();
        if (tid < cnt) {
            s_pos[tid] = pos[jt + tid];
            if constexpr (MIXED)
                s_w32[tid] = w32[jt + tid];
            else
                s_w64[tid] = w64[jt + tid];
        }
        __syncthreads();
        const bool diag = (jt < row_end) && (jt + cnt > row0);
        if constexpr (MIXED) {
            float t32[R], b32[R];
#pragma unroll
            for (int r = 0; r < R; ++r) t32[r] = b32[r] = 0.0f;
            if (!diag) {
#pragma unroll 2
                for (int jj = 0; jj < cnt; ++jj) {
                    const double4 p = s_pos[jj];
                    const float4 w = s_w32[jj];
#pragma unroll
                    for (int r = 0; r < R; ++r)
                        pair_f32(c32, tx[r], ty[r], tz[r], fnx[r], fny[r],
                                 fnz[r], p.x, p.y, p.z, w.x, w.y, w.z, w.w,
                                 t32[r], b32[r]);
                }
            } else {
                for (int jj = 0; jj < cnt; ++jj) {
                    const double4 p = s_pos[jj];
                    const float4 w = s_w32[jj];
#pragma unroll
                    for (int r = 0; r < R; ++r)
                        if (jt + jj != ti[r])
                            pair_f32(c32, tx[r], ty[r], tz[r], fnx[r], fny[r],
                                     fnz[r], p.x, p.y, p.z, w.x, w.y, w.z,
                                     w.w, t32[r], b32[r]);
                }
            }
#pragma unroll
            for (int r = 0; r < R; ++r) {
                top[r] += (double)t32[r];
                bot[r] += (double)b32[r];
            }
        } else {
            if (!diag) {
#pragma unroll 2
                for (int jj = 0; jj < cnt; ++jj) {
                    const double4 p = s_pos[jj];
                    const double4 w = s_w64[jj];
#pragma unroll
                    for (int r = 0; r < R; ++r)
                        pair_f64(c64, tx[r], ty[r], tz[r], tnx[r], tny[r],
                                 tnz[r], p.x, p.y, p.z, w.x, w.y, w.z, w.w,
                                 top[r], bot[r]);
                }
            } else {
                for (int jj = 0; jj < cnt; ++jj) {
                    const double4 p = s_pos[jj];
                    const double4 w = s_w64[jj];
#pragma unroll
                    for (int r = 0; r < R; ++r)
                        if (jt + jj != ti[r])
                            pair_f64(c64, tx[r], ty[r], tz[r], tnx[r], tny[r],
                                     tnz[r], p.x, p.y, p.z, w.x, w.y, w.z,
                                     w.w, top[r], bot[r]);
                }
            }
        }
    }
    double *pt = part + (size_t)(2 * blockIdx.y) * n;
    double *pb = pt + n;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        if (ti[r] < n) {
            pt[ti[r]] = top[r];
            pb[ti[r]] = bot[r];
        }
    }
}

// ------------------------------------------------------------------ finish
__global__ __launch_bounds__(kBlock) void finish_kernel(
    int n, int splits, const double *__restrict__ part,
    const double *__restrict__ u, double d_top, double d_bot,
    double *__restrict__ y) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    double st = 0.0, sb = 0.0;
    for (int s = 0; s < splits; ++s) {
        st += part[(size_t)(2 * s) * n + i];
        sb += part[(size_t)(2 * s + 1) * n + i];
    }
    y[i] = d_top * u[i] - st;
    y[n + i] = d_bot * u[n + i] - sb;
}

// ------------------------------------------------------------------ host
static inline int cdiv(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

void launch_prep(gabi_ctx *ctx, int precision, const double *u,
                 const double *scale, double *store, const int32_t *skip) {
    const int n = (int)ctx->n;
    hipLaunchKernelGGL(prep_kernel, dim3(cdiv(n, kBlock)), dim3(kBlock), 0,
                       ctx->stream, n, ctx->pos, ctx->nrm, u, scale, store,
                       precision == GABI_FP64 ? ctx->wgt : nullptr,
                       precision == GABI_FP64 ? nullptr : ctx->wgt32, skip);
}

void launch_pair(gabi_ctx *ctx, int precision, const int32_t *skip) {
    const int n = (int)ctx->n;
    const PairLaunch L = pair_launch(n, precision);
    const double eps = ctx->eps2 / ctx->eps1;
    PairConstF64 c64{ctx->kappa, eps, 1.0 / eps};
    PairConstF32 c32{(float)ctx->kappa,
                     (float)(-ctx->kappa * 1.4426950408889634074), (float)eps,
                     (float)(1.0 / eps)};
    dim3 grid(L.row_blocks, L.splits);
    const int pi = precision == GABI_FP64 ? 0 : 1;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (ctx->timing.enabled) {
        if (hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess)
            (void)hipEventRecord(e0, ctx->stream);
    }
#define GABI_PAIR(R, MX)                                                      \
    hipLaunchKernelGGL((pair_kernel<R, MX>), grid, dim3(kBlock), 0,           \
                       ctx->stream, n, L.tiles_per_split, ctx->pos, ctx->nrm, \
                       ctx->nrm32, ctx->wgt, ctx->wgt32, c64, c32, ctx->part, \
                       skip)
    if (precision == GABI_FP64) {
        if (L.rows_per_thread == 2) GABI_PAIR(2, false);
        else GABI_PAIR(1, false);
    } else {
        if (L.rows_per_thread == 2) GABI_PAIR(2, true);
        else GABI_PAIR(1, true);
    }
#undef GABI_PAIR
    if (e0 && e1) {
        (void)hipEventRecord(e1, ctx->stream);
        ctx->timing.pending[pi].push_back({e0, e1});
    }
}

void launch_finish(gabi_ctx *ctx, int precision, const double *u, double *y) {
    const int n = (int)ctx->n;
    const PairLaunch L = pair_launch(n, precision);
    const double eps = ctx->eps2 / ctx->eps1;
    hipLaunchKernelGGL(finish_kernel, dim3(cdiv(n, kBlock)), dim3(kBlock), 0,
                       ctx->stream, n, L.splits, ctx->part, u,
                       0.5 * (1.0 + eps), 0.5 * (1.0 + 1.0 / eps), y);
}

int matvec_device(gabi_ctx *ctx, int precision, const double *u, double *y) {
    launch_prep(ctx, precision, u, nullptr, nullptr, nullptr);
    launch_pair(ctx, precision, nullptr);
    launch_finish(ctx, precision, u, y);
    GABI_HIP(ctx, hipGetLastError());
    return GABI_OK;
}

}  // namespace gabi
