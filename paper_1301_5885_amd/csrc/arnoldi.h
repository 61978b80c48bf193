// Device steps of the Arnoldi process (restarted GMRES of Saad and Schultz,
// arXiv:1301.5885 Section 2.4) used by more than one kernel.
#pragma once
#include <hip/hip_runtime.h>

#include "gabi_internal.h"
#include "reduce.h"

namespace gabi {

// The cycle-end flag of a molecule.  Within one launch of the prep kernel
// the molecule's first workgroup may set it (the Givens step) while the
// other workgroups read it, so every access is a relaxed atomic at agent
// scope; launches on one stream are ordered, so no stronger order is needed.
__device__ __forceinline__ int load_done(const KrylovStatus *st) {
    return __hip_atomic_load(&st->done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void store_done(KrylovStatus *st, int v) {
    __hip_atomic_store(&st->done, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Sum of a molecule's nb per-workgroup partials in block order (every
// workgroup that calls it gets the same bits).  Contains __syncthreads().
__device__ __forceinline__ double sum_partials(const double *red, int nb, double *lds) {
    double v = 0.0;
    for (int t = threadIdx.x; t < nb; t += kBlock) v += red[t];
    return block_sum(v, lds);
}

// The slot of M.red that holds the partials of the projected ||w||^2.
__device__ __forceinline__ double *norm_slot(const Mol &M) {
    return M.red + (size_t)2 * M.m * kBlasBlocksMax;
}

// Step j of the cycle closes with h_{j+1,j} = hn = ||w||: the earlier
// rotations are applied to column j of H, a new rotation zeroes h_{j+1,j},
// the residual estimate |g_{j+1}| is updated, and the cycle stops on the
// estimate, the iteration cap or a breakdown (hn = 0).  One thread.
__device__ inline void givens_step(const Mol &M, int j, double hn) {
    KrylovStatus *st = M.st;
    const int m = M.m;
    double *H = M.H, *cs = M.cs, *sn = M.sn, *g = M.g;
    M.hn[j] = hn;
    H[(j + 1) * m + j] = hn;
    for (int i = 0; i < j; ++i) {
        const double a = H[i * m + j], c = H[(i + 1) * m + j];
        H[i * m + j] = cs[i] * a + sn[i] * c;
        H[(i + 1) * m + j] = -sn[i] * a + cs[i] * c;
    }
    const double a = H[j * m + j], c = H[(j + 1) * m + j];
    const double den = hypot(a, c);
    cs[j] = a / den;
    sn[j] = c / den;
    H[j * m + j] = den;
    H[(j + 1) * m + j] = 0.0;
    g[j + 1] = -sn[j] * g[j];
    g[j] = cs[j] * g[j];
    st->iters += 1;
    st->k = j + 1;
    st->gabs = fabs(g[j + 1]);
    if (fabs(g[j + 1]) / st->beta <= st->tol || st->iters >= st->maxit || hn == 0.0)
        store_done(st, 1);
}

}  // namespace gabi
