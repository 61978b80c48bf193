// Restarted GMRES(m) on the device (arXiv:1301.5885, Section 2.2 and
// Section 2.4: GMRES of Saad and Schultz, x0 = 0, restarted every m steps
// from the current iterate) and the mixed-precision iterative refinement
// around it, for a batch of molecules.
//
// Arnoldi with modified Gram-Schmidt: for step j, w = A v_j, then for
// i = 0..j in order h_ij = <w, v_i>, w <- w - h_ij v_i; h_{j+1,j} = ||w||;
// Givens rotations reduce H to triangular form and carry the residual
// estimate |g_{j+1}|.  The MGS coefficients are formed from one reduction
// per step (gram_kernel, project_kernel below): each workgroup adds its
// molecule's fixed-order dot partials (all workgroups of a molecule agree
// bitwise).  A per molecule device flag ends its cycle early (estimate below
// tol, breakdown, iteration cap); the remaining launches skip that molecule.
//
// A round is: one cycle of m Arnoldi steps, x += V y, the explicit FP64
// residual, and the start of the next cycle.  For the FP64 solver the cycle
// products are FP64 (restarted GMRES exactly as the paper runs it); for the
// mixed solver they are FP32-pair products while the residual that starts
// every cycle is FP64 (iterative refinement whose inner solve is one cycle);
// the treecode refinement of a single context takes the cycle products from
// the treecode instead.  The host reads one status record per molecule per
// round.
//
// All Krylov vectors, H, the rotations and every reduction are FP64.
#include <algorithm>
#include <cmath>

#include "arnoldi.h"
#include "gabi_internal.h"
#include "reduce.h"

namespace gabi {

enum CopyMode { kCopyRhsToResOut = 0, kZeroResX = 1, kCopyResXToSol = 2 };

// MODE (compile time): res_out = rhs_dst, res_x = 0, or sol = res_x.
template <int MODE>
__global__ __launch_bounds__(kBlock) void copy_kernel(const Mol *__restrict__ mols,
                                                      const int2 *__restrict__ list) {
    const int2 e = list[blockIdx.x];
    const Mol &M = mols[e.x];
    const int i = e.y * kBlock + threadIdx.x;
    const int n = M.n;
    if (i >= n) return;
    double *dst = MODE == kCopyRhsToResOut ? M.res_out : MODE == kZeroResX ? M.res_x : M.sol;
    if constexpr (MODE == kZeroResX) {
        dst[i] = 0.0;
        dst[n + i] = 0.0;
    } else {
        const double *src = MODE == kCopyRhsToResOut ? M.rhs_dst : M.res_x;
        dst[i] = src[i];
        dst[n + i] = src[n + i];
    }
}

// partials of ||rhs||^2
__global__ __launch_bounds__(kBlock) void dot_rhs_kernel(const Mol *__restrict__ mols,
                                                         const int2 *__restrict__ list) {
    __shared__ double lds[kBlock / 64];
    const int2 e = list[blockIdx.x];
    const Mol &M = mols[e.x];
    const int n = M.n;
    const double *a = M.rhs_dst;
    double s = 0.0;
    for (int i = e.y * kBlock + threadIdx.x; i < n; i += M.nb * kBlock)
        s = __builtin_fma(a[i], a[i], __builtin_fma(a[n + i], a[n + i], s));
    s = block_sum(s, lds);
    if (threadIdx.x == 0) M.red[e.y] = s;
}

// one workgroup per molecule: ||b||, targets, counters
__global__ __launch_bounds__(kBlock) void init_kernel(const Mol *__restrict__ mols) {
    __shared__ double lds[kBlock / 64];
    const Mol &M = mols[blockIdx.x];
    const double bb = sum_partials(M.red, M.nb, lds);
    if (threadIdx.x == 0) {
        KrylovStatus *st = M.st;
        st->beta0 = sqrt(bb);
        st->beta = st->beta0;
        st->tol0 = M.tol0;
        st->tol = M.tol0;
        st->inner_tol = M.inner_tol;
        st->maxit = M.maxit;
        st->iters = 0;
        st->k = 0;
        store_done(st, 0);
        st->converged = 0;
        st->rnorm = st->beta0;
        st->gabs = st->beta0;
        st->energy = 0.0;
    }
}

// one workgroup per molecule: ||res_out|| from the residual partials, the
// convergence test, and the start of the next cycle
__global__ __launch_bounds__(kBlock) void start_kernel(const Mol *__restrict__ mols) {
    __shared__ double lds[kBlock / 64];
    const Mol &M = mols[blockIdx.x];
    const double rr = sum_partials(M.red, M.nb, lds);
    if (threadIdx.x != 0) return;
    KrylovStatus *st = M.st;
    const double rn = sqrt(rr);
    st->rnorm = rn;
    st->gabs = rn;
    st->k = 0;
    const int conv = (st->beta0 == 0.0 || rn == 0.0 || rn / st->beta0 <= st->tol0) ? 1 : 0;
    st->converged = conv;
    if (M.mode == kModeMixed && rn > 0.0) {
        st->beta = rn;
        st->tol = fmax(st->inner_tol, 0.1 * st->tol0 * st->beta0 / rn);
    } else {
        st->beta = st->beta0;
        st->tol = st->tol0;
    }
    for (int i = 0; i <= M.m; ++i) M.g[i] = 0.0;
    M.g[0] = rn;
    store_done(st, (conv || st->iters >= st->maxit) ? 1 : 0);
}

// Modified Gram-Schmidt in one reduction per step.  MGS takes h_i as the dot
// of v_i with w after the first i subtractions, so h_i = c_i - sum_{k<i}
// L_ik h_k with c_i = <w, v_i> and the Gram entries L_ik = <v_k, v_i>: every
// coefficient follows from dot products of the unmodified vectors, which
// one launch computes, instead of j + 1 dependent launches.
//
// gram_kernel: partials of the dot products of step j beyond <w, v_0> (the
// product's finish emits that one into slot 0).  Grid (blas blocks, 2j):
// slot d = 1..j gets <w, v_d>, slot j + 1 + k (k < j) gets <v_k, v_j>.
__global__ __launch_bounds__(kBlock) void gram_kernel(const Mol *__restrict__ mols,
                                                      const int2 *__restrict__ list, int j) {
    __shared__ double lds[kBlock / 64];
    const int2 e = list[blockIdx.x];
    const Mol &M = mols[e.x];
    if (load_done(M.st)) return;
    const int n = M.n, nb = M.nb;
    const size_t len = 2 * (size_t)n;
    const int d = (int)blockIdx.y + 1;
    const double *a = d <= j ? M.w : M.V + (size_t)(d - j - 1) * len;
    const double *c = M.V + (size_t)(d <= j ? d : j) * len;
    double s = 0.0;
    for (int t = e.y * kBlock + threadIdx.x; t < n; t += nb * kBlock)
        s = __builtin_fma(a[t], c[t], __builtin_fma(a[n + t], c[n + t], s));
    s = block_sum(s, lds);
    if (threadIdx.x == 0) M.red[(size_t)d * kBlasBlocksMax + e.y] = s;
}

// project_kernel: every workgroup adds the 2j + 1 dot products (wave q takes
// slots q, q + 4, ... in lane order, so all workgroups agree bitwise), solves
// for h_0..h_j, sets w <- w - sum_i h_i v_i on its slice (i ascending, as MGS
// subtracts) and emits its partial of ||w||^2.  The molecule's first
// workgroup stores column j of H and Gram row j for the later steps.
__global__ __launch_bounds__(kBlock) void project_kernel(const Mol *__restrict__ mols,
                                                         const int2 *__restrict__ list, int j) {
    __shared__ double s_dot[2 * kMaxRestart];
    __shared__ double s_L[kMaxRestart * (kMaxRestart - 1) / 2];
    __shared__ double s_h[kMaxRestart];
    __shared__ double lds[kBlock / 64];
    const int2 e = list[blockIdx.x];
    const Mol &M = mols[e.x];
    if (load_done(M.st)) return;
    const int n = M.n, nb = M.nb, m = M.m;
    const size_t len = 2 * (size_t)n;
    const int nl = j * (j - 1) / 2;  // Gram rows 1..j-1
    for (int t = threadIdx.x; t < nl; t += kBlock) s_L[t] = M.G[t];
    const int lane = threadIdx.x & 63;
    for (int d0 = 0; d0 <= 2 * j; d0 += kBlock / 64) {  // same trip count in every wave
        const int d = d0 + (threadIdx.x >> 6);
        double v = 0.0;
        if (d <= 2 * j) {
            const double *p = M.red + (size_t)d * kBlasBlocksMax;
            for (int t = lane; t < nb; t += 64) v += p[t];
        }
        v = wave_total_lane63(v);
        if (lane == 63 && d <= 2 * j) s_dot[d] = v;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const bool first = e.y == 0;
        for (int i = 0; i <= j; ++i) {
            const double *Li = i < j ? s_L + i * (i - 1) / 2 : s_dot + j + 1;
            double c = s_dot[i];
            for (int k = 0; k < i; ++k) c = __builtin_fma(-Li[k], s_h[k], c);
            s_h[i] = c;
            if (first) M.H[i * m + j] = c;
        }
        if (first)
            for (int k = 0; k < j; ++k) M.G[nl + k] = s_dot[j + 1 + k];
    }
    __syncthreads();
    double *w = M.w;
    double s = 0.0;
    for (int t = e.y * kBlock + threadIdx.x; t < n; t += nb * kBlock) {
        double wt = w[t], wb = w[n + t];
        const double *v = M.V + t;
#pragma unroll 4
        for (int i = 0; i <= j; ++i) {
            wt = __builtin_fma(-s_h[i], v[(size_t)i * len], wt);
            wb = __builtin_fma(-s_h[i], v[(size_t)i * len + n], wb);
        }
        w[t] = wt;
        w[n + t] = wb;
        s = __builtin_fma(wt, wt, __builtin_fma(wb, wb, s));
    }
    s = block_sum(s, lds);
    if (threadIdx.x == 0) norm_slot(M)[e.y] = s;
}

// one workgroup per molecule: the Givens step that closes step j (the last
// step of a cycle; the earlier ones run inside the next step's prep)
__global__ __launch_bounds__(kBlock) void givens_kernel(const Mol *__restrict__ mols, int j) {
    __shared__ double lds[kBlock / 64];
    const Mol &M = mols[blockIdx.x];
    if (load_done(M.st)) return;
    const double hn = sqrt(sum_partials(norm_slot(M), M.nb, lds));
    if (threadIdx.x == 0) givens_step(M, j, hn);
}

// upd_dst += V y with H(0:k,0:k) y = g(0:k); every workgroup solves the small
// triangular system itself (identical arithmetic in all of them).
__global__ __launch_bounds__(kBlock) void update_kernel(const Mol *__restrict__ mols,
                                                        const int2 *__restrict__ list) {
    __shared__ double y[kMaxRestart];
    const int2 e = list[blockIdx.x];
    const Mol &M = mols[e.x];
    const int m = M.m, n = M.n;
    const int k = min(max(M.st->k, 0), m);
    if (k == 0) return;
    if (threadIdx.x == 0) {
        for (int i = k - 1; i >= 0; --i) {
            double s = M.g[i];
            for (int t = i + 1; t < k; ++t) s -= M.H[i * m + t] * y[t];
            y[i] = s / M.H[i * m + i];
        }
    }
    __syncthreads();
    const size_t len = 2 * (size_t)n;
    double *x = M.upd_dst;
    for (int i = e.y * kBlock + threadIdx.x; i < n; i += M.nb * kBlock) {
        double xt = x[i], xb = x[n + i];
        for (int c = 0; c < k; ++c) {
            xt = __builtin_fma(y[c], M.V[c * len + i], xt);
            xb = __builtin_fma(y[c], M.V[c * len + n + i], xb);
        }
        x[i] = xt;
        x[n + i] = xb;
    }
}

__global__ void gather_status_kernel(const Mol *__restrict__ mols, int nmol,
                                     KrylovStatus *__restrict__ out) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < nmol) out[k] = *mols[k].st;
}

// ---------------------------------------------------------------- host
static void launch_copy(const Batch &b, hipStream_t s, int mode) {
    const dim3 g(b.n_elem), blk(kBlock);
    if (mode == kCopyRhsToResOut)
        hipLaunchKernelGGL(copy_kernel<kCopyRhsToResOut>, g, blk, 0, s, b.d_mols, b.d_elem);
    else if (mode == kZeroResX)
        hipLaunchKernelGGL(copy_kernel<kZeroResX>, g, blk, 0, s, b.d_mols, b.d_elem);
    else
        hipLaunchKernelGGL(copy_kernel<kCopyResXToSol>, g, blk, 0, s, b.d_mols, b.d_elem);
}

static int nmol(const Batch &b) { return (int)b.slots.size(); }

void enqueue_init(Batch &b, hipStream_t s, bool x0_given, const Timer *t) {
    launch_rhs(b, s);
    hipLaunchKernelGGL(dot_rhs_kernel, dim3(b.n_blas), dim3(kBlock), 0, s, b.d_mols, b.d_blas);
    hipLaunchKernelGGL(init_kernel, dim3(nmol(b)), dim3(kBlock), 0, s, b.d_mols);
    if (x0_given) {
        launch_prep(b, s, GABI_FP64, kPrepResX, 0, false);
        launch_pair(b, s, GABI_FP64, false, t);
        launch_finish(b, s, GABI_FP64, kFinishRes, 0, false);
    } else {
        launch_copy(b, s, kZeroResX);
        launch_copy(b, s, kCopyRhsToResOut);
    }
    hipLaunchKernelGGL(start_kernel, dim3(nmol(b)), dim3(kBlock), 0, s, b.d_mols);
}

void enqueue_round(Batch &b, hipStream_t s, const Timer *t) {
    const int prec = b.mode == kModeMixed ? GABI_FP32_PAIR : GABI_FP64;
    const int m = b.slots.empty() ? 0 : b.slots[0]->mol.m;
    for (int j = 0; j < m; ++j) {
        // the prep of step j > 0 also runs the Givens step that closes j - 1
        if (b.tree) {
            // treecode refinement: V_j from the FP64 prep, its treecode sums
            // as the single partial slot of the Arnoldi finish
            const Mol &M = b.slots[0]->mol;
            launch_prep(b, s, GABI_FP64, j == 0 ? kPrepCycle0 : kPrepCycleJ, j, true);
            launch_tree_sums(*b.tree, s, M, M.V + (size_t)j * 2 * M.n, M.part, true, b.tree_f32);
            launch_finish(b, s, kPrecTree, kFinishDot, j, true);
        } else {
            launch_prep(b, s, prec, j == 0 ? kPrepCycle0 : kPrepCycleJ, j, true);
            launch_pair(b, s, prec, true, t);
            launch_finish(b, s, prec, kFinishDot, j, true);
        }
        if (j > 0)
            hipLaunchKernelGGL(gram_kernel, dim3(b.n_blas, 2 * j), dim3(kBlock), 0, s,
                               b.d_mols, b.d_blas, j);
        hipLaunchKernelGGL(project_kernel, dim3(b.n_blas), dim3(kBlock), 0, s, b.d_mols,
                           b.d_blas, j);
    }
    if (m > 0)
        hipLaunchKernelGGL(givens_kernel, dim3(nmol(b)), dim3(kBlock), 0, s, b.d_mols, m - 1);
    hipLaunchKernelGGL(update_kernel, dim3(b.n_blas), dim3(kBlock), 0, s, b.d_mols, b.d_blas);
    launch_prep(b, s, GABI_FP64, kPrepResX, 0, false);
    launch_pair(b, s, GABI_FP64, false, t);
    launch_finish(b, s, GABI_FP64, kFinishRes, 0, false);
    hipLaunchKernelGGL(start_kernel, dim3(nmol(b)), dim3(kBlock), 0, s, b.d_mols);
}

void enqueue_gather(Batch &b, hipStream_t s) {
    const int nm = nmol(b);
    hipLaunchKernelGGL(gather_status_kernel, dim3((nm + 63) / 64), dim3(64), 0, s,
                       b.d_mols, nm, b.d_status);
    (void)hipMemcpyAsync(b.h_status, b.d_status, sizeof(KrylovStatus) * nm,
                         hipMemcpyDeviceToHost, s);
}

void enqueue_finalize(Batch &b, hipStream_t s) {
    launch_copy(b, s, kCopyResXToSol);
    launch_reaction(b, s, true);
}

// One round, eager or as a replay of the captured graph of this batch.  A
// timed round is captured with event records around its product launches
// (Batch::graph_events; read them with graph_round_times once the replay has
// completed); a change of the timing choice captures the round again.
int run_round(Batch &b, hipStream_t s, hipStream_t capture, const Timer *t,
              bool use_graph, std::string &err) {
    const bool timed = t && (t->pending[0] || t->pending[1]);
    {
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) {
            err = std::string("an earlier device call failed: ") + hipGetErrorString(e);
            return GABI_EDEVICE;
        }
    }
    if (use_graph && capture) {
        if (!b.graph_valid || b.graph_timed != timed) {
            release_graph(b);
            Timer gt;
            if (timed) {
                gt.pending[0] = &b.graph_events[0];
                gt.pending[1] = &b.graph_events[1];
            }
            hipGraph_t g = nullptr;
            const char *step = "begin capture";
            hipError_t e = hipStreamBeginCapture(capture, hipStreamCaptureModeRelaxed);
            if (e == hipSuccess) {
                enqueue_round(b, capture, timed ? &gt : nullptr);
                const hipError_t ec = hipGetLastError();  // a launch or record in capture
                e = hipStreamEndCapture(capture, &g);
                step = "capture";
                if (e == hipSuccess) e = ec;
            }
            if (e == hipSuccess) {
                step = "instantiate";
                e = hipGraphInstantiate(&b.graph, g, nullptr, nullptr, 0);
            }
            if (g) (void)hipGraphDestroy(g);
            if (e != hipSuccess) {
                release_graph(b);
                err = std::string("graph ") + step + " of a round failed: " +
                      hipGetErrorString(e);
                return GABI_EDEVICE;
            }
            b.graph_valid = true;
            b.graph_timed = timed;
        }
        hipError_t e = hipGraphLaunch(b.graph, s);
        if (e != hipSuccess) {
            err = std::string("graph launch failed: ") + hipGetErrorString(e);
            return GABI_EDEVICE;
        }
    } else {
        enqueue_round(b, s, t);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        err = std::string("round launch failed: ") + hipGetErrorString(e);
        return GABI_EDEVICE;
    }
    return GABI_OK;
}

// Adds the product-launch times of the last replay of a timed captured round
// (index 0 FP64, 1 FP32-pair); the replay must have completed.
void graph_round_times(const Batch &b, double *ms, int64_t *count) {
    if (!b.graph_valid || !b.graph_timed) return;
    for (int p = 0; p < 2; ++p)
        for (const auto &ev : b.graph_events[p]) {
            float t = 0.0f;
            if (hipEventElapsedTime(&t, ev.first, ev.second) == hipSuccess) {
                ms[p] += t;
                count[p] += 1;
            } else {
                (void)hipGetLastError();
            }
        }
}

}  // namespace gabi
