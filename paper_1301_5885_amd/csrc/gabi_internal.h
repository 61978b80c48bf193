// Internal declarations of libgabi: device buffers, launch configuration
// and kernel launchers shared by the C-ABI layer and the Krylov driver.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/gabi.h"

namespace gabi {

constexpr int kBlock = 256;          // threads per workgroup (4 wave64)
constexpr int kTile = 256;           // sources staged in LDS per tile
constexpr int kBlasBlocksMax = 256;  // blocks of the reduction kernels
constexpr double kPi = 3.14159265358979323846;
constexpr double kCoulomb = 332.0716;  // kcal A / (mol e^2)

// Decomposition of one product: row blocks x source splits.  A function of
// N and the precision only, so every product of the same size sums in the
// same order (bitwise reproducible, independent of other work).
struct PairLaunch {
    int rows_per_thread = 1;
    int row_blocks = 0;
    int tiles_per_split = 0;
    int splits = 0;
};

PairLaunch pair_launch(int64_t n, int precision);

// Device status of one GMRES run (see krylov.hip).
struct KrylovStatus {
    int32_t k;       // Arnoldi steps taken in the current cycle
    int32_t done;    // cycle ended (estimate below tol, breakdown, maxit)
    int32_t iters;   // Arnoldi steps of this run
    int32_t maxit;
    double beta;     // ||b||
    double tol;
    double rnorm;    // ||r|| of the last explicit residual
    double gabs;     // |g_k|, the Givens estimate of ||r||
};

struct Timing {
    bool enabled = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> pending[2];
    double total_ms[2] = {0, 0};
    int64_t count[2] = {0, 0};
};

}  // namespace gabi

struct gabi_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;

    // surface, N elements
    int64_t n = 0;
    double4 *pos = nullptr;   // (cx, cy, cz, area)
    double4 *nrm = nullptr;   // (nx, ny, nz, 0)
    float4 *nrm32 = nullptr;  // FP32 normals for the mixed product
    double4 *wgt = nullptr;   // per-product source weights (s, mx, my, mz)
    float4 *wgt32 = nullptr;
    double *part = nullptr;   // pair partial sums [splits][2][n]
    int64_t part_len = 0;
    std::vector<double> host_centroids;  // 3n, for validation

    // charges
    int64_t nc = 0;
    bool charges_set = false;
    double4 *chg = nullptr;   // (px, py, pz, q)
    double *phi_dev = nullptr;   // reaction potential at the charges
    double *phi_part = nullptr;  // reaction-potential partials
    int64_t phi_part_len = 0;
    std::vector<double> host_charges;  // 4nc

    // parameters
    bool params_set = false;
    double eps1 = 1.0, eps2 = 80.0, kappa = 0.0;

    // vectors of length 2n
    double *vec_u = nullptr;    // product input / last solution
    double *vec_y = nullptr;    // product output
    double *vec_b = nullptr;    // right-hand side
    double *vec_in = nullptr;   // staging for host-pointer entry points
    bool have_solution = false;

    // reductions and small device scalars
    double *red = nullptr;      // [2][kBlasBlocksMax] ping-pong partials
    double *scalars = nullptr;  // small device scalars (energy, ...)

    // Krylov workspace (allocated on first solve, sized for `kry_m`)
    int kry_m = 0;
    double *V = nullptr;        // (m+1) x 2n basis
    double *H = nullptr;        // (m+1) x m Hessenberg, row-major
    double *givens = nullptr;   // cs[m], sn[m], g[m+1], hn[m]
    double *gm_b = nullptr;     // right-hand side of the current GMRES run
    double *gm_x = nullptr;     // iterate
    double *gm_r = nullptr;     // residual
    double *gm_w = nullptr;     // Arnoldi work vector
    double *ir_x = nullptr;     // refinement iterate
    double *ir_r = nullptr;     // refinement residual
    gabi::KrylovStatus *status = nullptr;       // device
    gabi::KrylovStatus *status_host = nullptr;  // pinned host mirror

    gabi::Timing timing;
    int64_t bytes = 0;
};

namespace gabi {

// ---- errors ---------------------------------------------------------------
int fail(gabi_ctx *ctx, int code, const std::string &msg);
int hip_fail(gabi_ctx *ctx, hipError_t e, const char *what);
#define GABI_HIP(ctx, expr)                                        \
    do {                                                           \
        hipError_t e_ = (expr);                                    \
        if (e_ != hipSuccess) return ::gabi::hip_fail(ctx, e_, #expr); \
    } while (0)

int dev_alloc(gabi_ctx *ctx, void **p, size_t bytes);
void dev_free(gabi_ctx *ctx, void **p, size_t bytes);

// ---- launchers (matvec.hip) -----------------------------------------------
// Source weights from u (length 2n, device) scaled by 1/(*scale) when scale
// is non-null; if store is non-null the scaled vector is written there.
void launch_prep(gabi_ctx *ctx, int precision, const double *u,
                 const double *scale, double *store, const int32_t *skip);
// Pair sums into ctx->part.  skip: device flag, non-zero skips the work.
void launch_pair(gabi_ctx *ctx, int precision, const int32_t *skip);
// y = diag(u) - sum of partials.
void launch_finish(gabi_ctx *ctx, int precision, const double *u, double *y);
// Full product y = A u (u, y device, length 2n).
int matvec_device(gabi_ctx *ctx, int precision, const double *u, double *y);

// ---- source terms and energy (sources.hip) --------------------------------
void launch_rhs(gabi_ctx *ctx, double *b);
// Reaction potential at the charges from the weights in ctx->wgt; writes
// nc values to phi (device).  If energy_out is non-null, also writes
// E_sol in kcal/mol there (device scalar).
int launch_reaction(gabi_ctx *ctx, double *phi, double *energy_out);

// ---- Krylov (krylov.hip) --------------------------------------------------
int ensure_krylov(gabi_ctx *ctx, int m);
int solve_device(gabi_ctx *ctx, const gabi_solve_opts &opts,
                 const double *x0, double *u, gabi_solve_info *info);

// ---- reductions -----------------------------------------------------------
int blas_blocks(int64_t n);

}  // namespace gabi
