// The discrete boundary-integral product y = A u of arXiv:1301.5885,
// Section 2.2, eqs. (eqdbef1)/(eqdbef2), on gfx950, for a batch of molecules.
//
//   y_i     = (1+eps)/2 phi_i   - sum_{j != i} W_j [K1 psi_j + K2 phi_j]
//   y_{N+i} = (1+1/eps)/2 psi_i - sum_{j != i} W_j [K3 psi_j + K4 phi_j]
//
// Three launches per product:
//   prep    O(N): source weights s_j = W_j psi_j/(4 pi), m_j = W_j phi_j
//           nu_j/(4 pi) (FP64, or FP32 for the mixed product);
//   pair    O(N^2): a tile = (molecule, row block, source split).  Each
//           thread holds R target rows in registers; the workgroup streams
//           the split's sources through LDS, 256 records per stage
//           (coalesced loads, broadcast reads), and writes its two row sums
//           per target to the molecule's partial buffer.  Tiles of every
//           molecule in the batch are listed longest first; the persistent
//           form runs a fixed grid that drains the list in the order of
//           next_tile (first round by workgroup id, then an atomic counter,
//           the last partial round by workgroup id again), the flat form
//           launches one workgroup per tile;
//   finish  O(N S): adds the split partials in split order, applies the
//           diagonal, and (inside GMRES) emits the first MGS dot partial.
// A symmetric product whose partial slots would exceed the partial-sum
// budget runs as several passes (pair launch, then a fold of the pass's
// slots into an FP64 accumulator; the finish adds the last pass).
// The decomposition depends only on N, the precision, the tuning table and
// the budget, so a molecule's summation order is the same alone or in any
// batch (bitwise reproducible).
// The self term j = i is skipped exactly: only the source stages that overlap
// the tile's own rows run the masked loop.
#include "arnoldi.h"
#include "gabi_internal.h"
#include "pair_math.h"
#include "reduce.h"

namespace gabi {

// ------------------------------------------------------------------ prep
// MODE (compile time) selects the input vector: the cycle start r/||r||
// (stored as V_0), the Arnoldi vector w/h_{j,j-1} (stored as V_j), the
// residual iterate, or the product input u.
//
// kPrepCycleJ also closes step j - 1: every workgroup reduces the partials
// of ||w||^2 to h_{j,j-1} itself (the same bits in all of them), and the
// molecule's first workgroup applies the Givens step, which may end the
// cycle; the other workgroups may then still write V_j and weights that no
// later step reads.
template <int MODE>
__global__ __launch_bounds__(kBlock) void prep_kernel(
    const Mol *__restrict__ mols, const int2 *__restrict__ list, int precision,
    int j, int skip) {
    const int2 e = list[blockIdx.x];
    const Mol &M = mols[e.x];
    double hj = 0.0;
    if constexpr (MODE == kPrepCycleJ) {
        // done can change during this launch (the Givens step below), so the
        // workgroup takes one reading of it
        __shared__ int s_done;
        __shared__ double lds[kBlock / 64];
        if (threadIdx.x == 0) s_done = skip && load_done(M.st);
        __syncthreads();
        if (s_done) return;
        hj = sqrt(sum_partials(norm_slot(M), M.nb, lds));
        if (e.y == 0 && threadIdx.x == 0) givens_step(M, j - 1, hj);
        if (hj == 0.0) return;  // breakdown: the cycle has ended
    } else {
        if (skip && load_done(M.st)) return;
    }
    const int i = e.y * kBlock + threadIdx.x;
    const int n = M.n;
    if (i >= n) return;
    const double *src = MODE == kPrepCycle0 ? M.cyc_src
                      : MODE == kPrepCycleJ ? M.w
                      : MODE == kPrepResX   ? M.res_x
                                            : M.u;
    double phi = src[i], psi = src[n + i];
    if constexpr (MODE == kPrepCycle0 || MODE == kPrepCycleJ) {
        const double h = MODE == kPrepCycle0 ? M.st->rnorm : hj;
        double *store = M.V + (size_t)(MODE == kPrepCycle0 ? 0 : j) * 2 * n;
        phi = phi / h;
        psi = psi / h;
        store[i] = phi;
        store[n + i] = psi;
    }
    const double4 p = M.pos[i];
    const double4 nu = M.nrm[i];
    const double c = p.w * (1.0 / (4.0 * kPi));
    const double s = c * psi;
    const double t = c * phi;
    // The symmetric product reads (s, t) and forms the m terms from the
    // normal; the split product reads (s, m).
    const bool sym = precision == GABI_FP64 ? M.sym64 : M.sym32;
    if (precision == GABI_FP64)
        M.wgt[i] = sym ? make_double4(s, t, 0.0, 0.0)
                       : make_double4(s, t * nu.x, t * nu.y, t * nu.z);
    else
        M.wgt32[i] = sym ? make_float4((float)s, (float)t, 0.0f, 0.0f)
                         : make_float4((float)s, (float)(t * nu.x), (float)(t * nu.y),
                                       (float)(t * nu.z));
}

// ------------------------------------------------------------ tile order
// A persistent grid of G workgroups drains T >= G tiles (sorted longest
// first) in three phases.  Workgroup w takes tile w first, with no atomic:
// G workgroups contending for one counter at the launch would start their
// first tiles staggered.  Tiles G .. G floor(T/G) - 1 come from an atomic
// counter, so faster workgroups take more of them.  The last partial round,
// the remaining T mod G tiles, goes one each to workgroups 0, 1, ...: ids
// are spread evenly over the CUs, whereas the workgroups that happen to be
// free first are not, and a partial round taken from the queue can leave
// some CUs with eight tiles and others with none.  A non-persistent launch
// has one workgroup per tile.  Every thread of a workgroup calls next_tile
// (it contains barriers, which also end the previous tile's use of LDS).
__device__ __forceinline__ int next_tile(int persistent, int t, int ntiles, int *counter,
                                         int *s_next) {
    if (!persistent) return ntiles;
    const int G = (int)gridDim.x;
    const int queued_end = ntiles - ntiles % G;
    if (t >= queued_end) return ntiles;  // its tile of the last partial round is done
    if (queued_end > G) {
        __syncthreads();
        if (threadIdx.x == 0) *s_next = G + atomicAdd(counter, 1);
        __syncthreads();
        const int u = *s_next;
        if (u < queued_end) return u;
    } else {
        __syncthreads();
    }
    return queued_end + (int)blockIdx.x;
}

// ------------------------------------------------------------------ pair
// Per-precision views of a molecule: the FP64 product reads FP64 centroids
// (cx, cy, cz, area) and weights (s, mx, my, mz); the FP32 one reads the
// centred FP32 coordinates and FP32 weights.
template <bool MIXED> struct PairView;
template <> struct PairView<false> {
    using T = double;
    using T4 = double4;
    static __device__ __forceinline__ const T4 *pos(const Mol &M) { return M.pos; }
    static __device__ __forceinline__ const T4 *nrm(const Mol &M) { return M.nrm; }
    static __device__ __forceinline__ const T4 *wgt(const Mol &M) { return M.wgt; }
    static __device__ __forceinline__ int tps(const Mol &M) { return M.tps64; }
    static __device__ __forceinline__ int head(const Mol &M) { return M.head64; }
    static __device__ __forceinline__ int tail(const Mol &M) { return M.tail64; }
};
template <> struct PairView<true> {
    using T = float;
    using T4 = float4;
    static __device__ __forceinline__ const T4 *pos(const Mol &M) { return M.pos32; }
    static __device__ __forceinline__ const T4 *nrm(const Mol &M) { return M.nrm32; }
    static __device__ __forceinline__ const T4 *wgt(const Mol &M) { return M.wgt32; }
    static __device__ __forceinline__ int tps(const Mol &M) { return M.tps32; }
    static __device__ __forceinline__ int head(const Mol &M) { return M.head32; }
    static __device__ __forceinline__ int tail(const Mol &M) { return M.tail32; }
};

template <bool MIXED>
__device__ __forceinline__ void pair_eval(const Mol &M, typename PairView<MIXED>::T tx,
                                          typename PairView<MIXED>::T ty,
                                          typename PairView<MIXED>::T tz,
                                          typename PairView<MIXED>::T tnx,
                                          typename PairView<MIXED>::T tny,
                                          typename PairView<MIXED>::T tnz,
                                          const typename PairView<MIXED>::T4 &p,
                                          const typename PairView<MIXED>::T4 &w,
                                          typename PairView<MIXED>::T &top,
                                          typename PairView<MIXED>::T &bot) {
    if constexpr (MIXED) {
        const PairConstF32 c{M.kappa_f, M.nkl2e_f, M.eps_f, M.inv_eps_f};
        pair_f32(c, tx, ty, tz, tnx, tny, tnz, p.x, p.y, p.z, w.x, w.y, w.z, w.w, top, bot);
    } else {
        const PairConstF64 c{M.kappa, M.eps, M.inv_eps};
        pair_f64(c, tx, ty, tz, tnx, tny, tnz, p.x, p.y, p.z, w.x, w.y, w.z, w.w, top, bot);
    }
}

// One tile: R target rows per thread against the split's sources.  The FP64
// product accumulates each row in FP64 directly; the FP32 product sums each
// 256-source stage in FP32 and adds the stage sum to an FP64 accumulator.
template <int R, bool MIXED>
__device__ __forceinline__ void pair_tile(const Mol &M, int rb, int sp,
                                          typename PairView<MIXED>::T4 *s_pos,
                                          typename PairView<MIXED>::T4 *s_w) {
    using V = PairView<MIXED>;
    using T = typename V::T;
    using T4 = typename V::T4;
    const int n = M.n;
    const int tid = threadIdx.x;
    const int row0 = rb * kBlock * R;
    const int row_end = min(n, row0 + kBlock * R);
    int j_begin, j_end;
    split_range(n, V::tps(M), V::head(M), V::tail(M), sp, j_begin, j_end);
    const T4 *pos = V::pos(M), *nrm = V::nrm(M), *wgt = V::wgt(M);

    T tx[R], ty[R], tz[R], tnx[R], tny[R], tnz[R];
    double top[R], bot[R];
    int ti[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int i = row0 + r * kBlock + tid;
        ti[r] = i;
        const int ic = min(i, n - 1);
        const T4 p = pos[ic], q = nrm[ic];
        tx[r] = p.x;
        ty[r] = p.y;
        tz[r] = p.z;
        tnx[r] = q.x;
        tny[r] = q.y;
        tnz[r] = q.z;
        top[r] = 0.0;
        bot[r] = 0.0;
    }

    for (int jt = j_begin; jt < j_end; jt += kTile) {
        const int cnt = min(kTile, j_end - jt);
        __syncthreads();
        if (tid < cnt) {
            s_pos[tid] = pos[jt + tid];
            s_w[tid] = wgt[jt + tid];
        }
        __syncthreads();
        const bool diag = (jt < row_end) && (jt + cnt > row0);
        T st[R], sb[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if constexpr (MIXED) {
                st[r] = sb[r] = T(0);
            } else {
                st[r] = top[r];
                sb[r] = bot[r];
            }
        }
        if (!diag) {
#pragma unroll 2
            for (int jj = 0; jj < cnt; ++jj) {
                const T4 p = s_pos[jj];
                const T4 w = s_w[jj];
#pragma unroll
                for (int r = 0; r < R; ++r)
                    pair_eval<MIXED>(M, tx[r], ty[r], tz[r], tnx[r], tny[r], tnz[r], p, w,
                                     st[r], sb[r]);
            }
        } else {
            for (int jj = 0; jj < cnt; ++jj) {
                const T4 p = s_pos[jj];
                const T4 w = s_w[jj];
#pragma unroll
                for (int r = 0; r < R; ++r)
                    if (jt + jj != ti[r])
                        pair_eval<MIXED>(M, tx[r], ty[r], tz[r], tnx[r], tny[r], tnz[r], p,
                                         w, st[r], sb[r]);
            }
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if constexpr (MIXED) {
                top[r] += (double)st[r];
                bot[r] += (double)sb[r];
            } else {
                top[r] = st[r];
                bot[r] = sb[r];
            }
        }
    }
    double *pt = M.part + (size_t)(2 * sp) * n;
    double *pb = pt + n;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        if (ti[r] < n) {
            pt[ti[r]] = top[r];
            pb[ti[r]] = bot[r];
        }
    }
}

// In a launch that may be skipped (a later step of a GMRES cycle that can
// have ended), a workgroup returns at once when every molecule's cycle has
// ended: handing out the tiles one by one only to skip each would cost the
// queue's atomics and barriers for every tile (about 0.7 ms per launch at
// N = 81,920).  The flags are set by earlier launches and do not change
// during this one, so every workgroup takes the same decision.
__device__ __forceinline__ bool all_done(const Mol *__restrict__ mols, int nmol) {
    for (int m = 0; m < nmol; ++m)
        if (!load_done(mols[m].st)) return false;
    return true;
}

// One workgroup per tile (flat) or a fixed grid draining the tile queue
// (persistent).  The loop exits for every workgroup once the counter passes
// the end of the list.  The FP32-pair variant is held to 7 waves per SIMD
// (at most 72 VGPRs, which it fits without spilling); the FP64 variant
// needs its registers and runs at 4.
template <bool MIXED, int R>
__global__ __launch_bounds__(kBlock, MIXED ? 7 : 1) void pair_kernel(
    const Mol *__restrict__ mols, int nmol, const int4 *__restrict__ tiles, int ntiles,
    int *__restrict__ counter, int persistent, int skip) {
    using T4 = typename PairView<MIXED>::T4;
    __shared__ T4 s_pos[kTile];
    __shared__ T4 s_w[kTile];
    __shared__ int s_next;
    if (skip && all_done(mols, nmol)) return;
    for (int t = (int)blockIdx.x; t < ntiles;
         t = next_tile(persistent, t, ntiles, counter, &s_next)) {
        const int4 tile = tiles[t];
        const Mol &M = mols[tile.x];
        if (!(skip && load_done(M.st))) pair_tile<R, MIXED>(M, tile.y, tile.z, s_pos, s_w);
    }
}

// ------------------------------------------------------------- symmetric
// Tile (I, J) of the symmetric scheme (I <= J), one element of block I per
// thread, writing partial-sum slot `slot` of its rows and columns.
// The workgroup stages block J in LDS (two 4-vectors per element:
// (x, y, z, s) and (nx, ny, nz, t), where m = t nu), taken in four chunks of
// 64 elements.  At step s of a chunk lane l reads element (l - s) mod 64, so the
// 64 lanes of a wave read 64 different elements (no bank conflicts) and meet
// every element of the chunk once in 64 steps:
//  * I < J: each unordered pair is evaluated once; the (i, j) terms add to the
//    lane's own row sums, the (j, i) terms to column sums that rotate through
//    the wave with the read pattern (wave_rotate) and are back in their
//    home lane after 64 steps.  The four waves' column sums of an element are
//    added in wave order through LDS.  Row sums go to the tile's slot of row
//    i, column sums to the same slot of row j.
//  * I = J: the ordered pairs (i, j), i != j, of the block (row sums only)
//    go to the tile's slot.
// The tiles come in rounds in which every block takes part once, and the
// tiles of round r write slot r mod (slots per pass): every slot of every row
// is written by exactly one tile of a pass, and the slots are added in round
// order.  Elements past N (the ragged last block) sit far
// away (rows and columns on opposite sides) with zero weights, so their terms
// are exactly zero and every lane takes part in the rotation; their own sums
// are not stored.
template <bool MIXED>
__device__ __forceinline__ SymElem<typename PairView<MIXED>::T> sym_load(const Mol &M, int e,
                                                                        bool active,
                                                                        float far) {
    using V = PairView<MIXED>;
    using T = typename V::T;
    const int ec = active ? e : M.n - 1;
    const typename V::T4 p = V::pos(M)[ec], q = V::nrm(M)[ec], w = V::wgt(M)[ec];
    SymElem<T> a;
    a.x = active ? p.x : T(far);
    a.y = active ? p.y : T(far);
    a.z = active ? p.z : T(far);
    a.nx = q.x;
    a.ny = q.y;
    a.nz = q.z;
    a.s = active ? w.x : T(0);  // weights (s, t) of the symmetric layout
    a.t = active ? w.y : T(0);
    return a;
}

template <bool MIXED>
__device__ __forceinline__ void sym_tile(const Mol &M, int I, int J, int slot,
                                         typename PairView<MIXED>::T4 *s_stage) {
    using T = typename PairView<MIXED>::T;
    using T4 = typename PairView<MIXED>::T4;
    const int n = M.n;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int i = I * kTile + tid;
    const bool act = i < n;
    const SymElem<T> a = sym_load<MIXED>(M, i, act, 1e17f);
    const int jt = J * kTile;
    const int cnt = min(kTile, n - jt);
    // (x, y, z, s) and (nx, ny, nz, t); each chunk of 64 is stored twice in a
    // row, so element (l - s) mod 64 is entry l + 64 - s of its chunk copy
    T4 *sa = s_stage, *sb = s_stage + 2 * kTile;
    {
        const SymElem<T> e = sym_load<MIXED>(M, jt + tid, tid < cnt, -1e17f);
        const int at = (tid >> 6) * 128 + (tid & 63);
        sa[at] = sa[at + 64] = T4{e.x, e.y, e.z, e.s};
        sb[at] = sb[at + 64] = T4{e.nx, e.ny, e.nz, e.t};
    }
    __syncthreads();
    T *part = reinterpret_cast<T *>(M.part);  // float for the FP32-pair product
    T top = T(0), bot = T(0);
#pragma unroll 1
    for (int c = 0; c < kTile / 64; ++c) {
        if (c * 64 >= cnt) break;
        const T4 *ca = sa + c * 128 + lane + 64, *cb = sb + c * 128 + lane + 64;
        if (I == J) {
            for (int s = 0; s < 64; ++s) {
                const int k = -s;
                if (c == wave && s == 0) continue;  // i paired with itself
                const T4 p = ca[k], q = cb[k];
                if constexpr (MIXED) {
                    const PairConstF32 kc{M.kappa_f, M.nkl2e_f, M.eps_f, M.inv_eps_f};
                    pair_f32(kc, a.x, a.y, a.z, a.nx, a.ny, a.nz, p.x, p.y, p.z, p.w, q.w * q.x,
                             q.w * q.y, q.w * q.z, top, bot);
                } else {
                    const PairConstF64 kc{M.kappa, M.eps, M.inv_eps};
                    pair_f64(kc, a.x, a.y, a.z, a.nx, a.ny, a.nz, p.x, p.y, p.z, p.w, q.w * q.x,
                             q.w * q.y, q.w * q.z, top, bot);
                }
            }
        } else {
            T ctop = T(0), cbot = T(0);
            const int from = rotate_from();
            // the next element is read one step ahead: step s reads element
            // s + 1, which for the last step is entry 0 of the chunk copy (in
            // bounds, unused).  Groups of 8 steps share one base address, so
            // the reads take immediate offsets.
            T4 p = ca[0], q = cb[0];
            const T4 *pa = ca, *pb = cb;
#pragma unroll 1
            for (int g = 0; g < 8; ++g) {
                pa -= 8;
                pb -= 8;
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const T4 pn = pa[7 - u], qn = pb[7 - u];
                    __builtin_amdgcn_sched_barrier(0);  // keep the reads ahead of the step
                    const SymElem<T> b{p.x, p.y, p.z, q.x, q.y, q.z, p.w, q.w};
                    if constexpr (MIXED) {
                        const PairConstF32 kc{M.kappa_f, M.nkl2e_f, M.eps_f, M.inv_eps_f};
                        sym_f32(kc, a, b, top, bot, ctop, cbot);
                    } else {
                        const PairConstF64 kc{M.kappa, M.eps, M.inv_eps};
                        sym_f64(kc, a, b, top, bot, ctop, cbot);
                    }
                    ctop = wave_rotate(ctop, from);
                    cbot = wave_rotate(cbot, from);
                    p = pn;
                    q = qn;
                }
            }
            // once every wave is past chunk c, its (x, y, z, s) entries (both
            // copies, 128 4-vectors) are free: they take each wave's 64 column
            // sums of top and bot, so no registers carry them across chunks
            static_assert(2 * kBlock <= 4 * 128, "column sums exceed a chunk's entries");
            __syncthreads();
            T *cs = reinterpret_cast<T *>(sa + c * 128);
            cs[wave * 64 + lane] = ctop;
            cs[kBlock + wave * 64 + lane] = cbot;
        }
    }
    if (I != J) {
        __syncthreads();
        if (tid < cnt) {
            const T *cs = reinterpret_cast<const T *>(sa + (tid >> 6) * 128);
            T ct = cs[lane], cbs = cs[kBlock + lane];
#pragma unroll
            for (int w = 1; w < kBlock / 64; ++w) {
                ct += cs[w * 64 + lane];
                cbs += cs[kBlock + w * 64 + lane];
            }
            part[(size_t)(2 * slot) * n + jt + tid] = ct;
            part[(size_t)(2 * slot + 1) * n + jt + tid] = cbs;
        }
    }
    if (act) {
        part[(size_t)(2 * slot) * n + i] = top;
        part[(size_t)(2 * slot + 1) * n + i] = bot;
    }
}

// The tiles of one pass come as kXcdLists lists, list x = tiles
// [xoff[x], xoff[x+1]), each a contiguous range of row blocks (the host
// sorts a pass by block I and cuts it into lists of equal cost), so that
// the tiles a list's workgroups run at the same time share their blocks in
// one L2.  Workgroups are placed on the XCDs in turn (id mod 8), and list x
// is drained by the C workgroups with id mod 8 = x (its home workgroups,
// local index k = id / 8) in the three phases of next_tile: entry k first
// (no atomic), then entries C .. Q - 1 from the list's counter, Q = the
// list's length less its length mod C, and the last partial round, entry
// Q + k, by local index, which spreads it over the XCD's CUs.  A workgroup
// whose home list is done helps the other lists, in turn, with their
// counter phases.  Every entry of every list is taken exactly once, and a
// tile's sums go to its own slot, so the order in which tiles run does not
// change any result.  A non-persistent launch has one workgroup per tile
// (xoff unused).
// A list no longer than kStaticRounds x C entries is taken by local index
// alone, entries k, k + C, ..., and gets no help: through the counter all
// home workgroups ask for their second tile at about the same moment and
// queue on one atomic (at N = 23,120, 4,186 tiles, that cost the FP32-pair
// product 10%).
// The FP32-pair variant is held to 8 waves per SIMD (at most 64 VGPRs).
constexpr int kStaticRounds = 4;
template <bool MIXED>
__global__ __launch_bounds__(kBlock, MIXED ? 8 : 1) void sym_pair_kernel(
    const Mol *__restrict__ mols, int nmol, const int4 *__restrict__ tiles, int ntiles,
    const int *__restrict__ xoff, int *__restrict__ xcnt, int persistent, int skip) {
    using T4 = typename PairView<MIXED>::T4;
    // two 4-vectors per element of block J, each chunk stored twice; the
    // first copies also take the column sums (2 x 4 waves x 64 per chunk)
    __shared__ T4 s_stage[4 * kTile];
    __shared__ int s_next;
    auto run = [&](int t) {
        const int4 tile = tiles[t];
        const Mol &M = mols[tile.x];
        if (!(skip && load_done(M.st))) sym_tile<MIXED>(M, tile.y, tile.z, tile.w & 0xffff, s_stage);
    };
    if (skip && all_done(mols, nmol)) return;
    if (!persistent) {
        if ((int)blockIdx.x < ntiles) run((int)blockIdx.x);
        return;
    }
    const int G = (int)gridDim.x;
    const int home = (int)blockIdx.x % kXcdLists, k = (int)blockIdx.x / kXcdLists;
#pragma unroll 1
    for (int l = 0; l < kXcdLists; ++l) {
        const int x = (home + l) % kXcdLists;
        const int a = xoff[x], len = xoff[x + 1] - a;
        const int C = (G - x + kXcdLists - 1) / kXcdLists;  // home workgroups of list x
        if (len <= kStaticRounds * C) {
            // a short list: its home workgroups take entries k, k + C, ...
            // (no counter, whose atomics all of them would reach at once)
            if (l == 0)
                for (int u = k; u < len; u += C) {
                    if (u != k) __syncthreads();  // the previous tile is done with LDS
                    run(a + u);
                }
            continue;
        }
        const int Q = C > 0 && len > C ? len - len % C : len;  // end of the counter phase
        if (l == 0 && k < len) run(a + k);
#pragma unroll 1
        for (;;) {
            if (Q <= C) break;  // no counter phase
            __syncthreads();    // the previous tile is done with LDS and s_next
            if (threadIdx.x == 0) s_next = C + atomicAdd(&xcnt[x], 1);
            __syncthreads();
            const int u = s_next;
            if (u >= Q) break;
            run(a + u);
        }
        if (l == 0 && Q + k < len && Q >= C) {
            __syncthreads();  // the previous tile is done with LDS
            run(a + Q + k);
        }
    }
}

// ------------------------------------------------------------------ finish
// MODE kFinishDot: w = D V_j - sum part, partials of <w, V_0>
//      kFinishRes: res_out = res_b - (D res_x - sum part), partials of ||.||^2
//      kFinishY:   y = D u - sum part
// where sum part = the slots of the product's last pass, preceded by the
// FP64 sums of its earlier passes when it has several.
// A workgroup of kFinishQ x 256 threads covers 256 elements per pass: thread
// group q adds the partial slots [q S / kFinishQ, (q+1) S / kFinishQ) of its
// element in slot order, and the groups' sums are added in group order, so
// the result does not depend on the launch (bitwise reproducible) while four
// times as many waves keep memory requests in flight.
constexpr int kFinishQ = 4;
constexpr int kPairVariants = 3;  // split R = 2, split R = 1, symmetric

// The finish also rearms the tile queues of the product it completes: the
// pair launches of this precision start from zero counters, and only the
// finish that follows them reads or writes those counters in between.
// st += slot 2p, sb += slot 2p + 1 of element i for p = p0 .. p1 - 1, added
// in slot order.  The reads of eight slots are issued before their sums, so
// a thread waits for memory once per eight slots rather than once per slot.
template <typename P>
__device__ __forceinline__ void sum_slots(const P *__restrict__ part, int n, int i, int p0,
                                          int p1, double &st, double &sb) {
    constexpr int kAhead = 8;
    int p = p0;
    for (; p + kAhead <= p1; p += kAhead) {
        P a[kAhead], b[kAhead];
#pragma unroll
        for (int k = 0; k < kAhead; ++k) {
            a[k] = part[(size_t)(2 * (p + k)) * n + i];
            b[k] = part[(size_t)(2 * (p + k) + 1) * n + i];
        }
#pragma unroll
        for (int k = 0; k < kAhead; ++k) {
            st += (double)a[k];
            sb += (double)b[k];
        }
    }
    for (; p < p1; ++p) {
        st += (double)part[(size_t)(2 * p) * n + i];
        sb += (double)part[(size_t)(2 * p + 1) * n + i];
    }
}

template <int MODE>
__global__ __launch_bounds__(kBlock * kFinishQ) void finish_kernel(
    const Mol *__restrict__ mols, const int2 *__restrict__ list, int precision,
    int j, int skip, int *__restrict__ counters) {
    __shared__ double acc[2][kFinishQ - 1][kBlock];
    __shared__ double lds[kBlock * kFinishQ / 64];
    if (blockIdx.x == 0 && threadIdx.x < kPairVariants) counters[threadIdx.x] = 0;
    if (blockIdx.x == 0 && threadIdx.x < kXcdLists) counters[kXcdCounters + threadIdx.x] = 0;
    const int2 e = list[blockIdx.x];
    const Mol &M = mols[e.x];
    if (skip && load_done(M.st)) return;
    const int n = M.n, nb = M.nb;
    const int q = threadIdx.x / kBlock, t = threadIdx.x % kBlock;
    // kPrecTree: the treecode sums, one FP64 slot
    const int splits = precision == kPrecTree ? 1 : precision == GABI_FP64 ? M.last64 : M.last32;
    const bool multi = precision != kPrecTree && (precision == GABI_FP64 ? M.np64 : M.np32) > 1;
    const int p0 = q * splits / kFinishQ, p1 = (q + 1) * splits / kFinishQ;
    const double *v = MODE == kFinishDot ? M.V + (size_t)j * 2 * n
                    : MODE == kFinishRes ? M.res_x
                                         : M.u;
    double *out = MODE == kFinishDot ? M.w : MODE == kFinishRes ? M.res_out : M.y;
    const double dt = M.d_top, db = M.d_bot;
    const bool f32 = precision == GABI_FP32_PAIR && M.sym32;  // float partial sums
    const float *pf = reinterpret_cast<const float *>(M.part);
    double s = 0.0;
    for (int base = e.y * kBlock; base < n; base += nb * kBlock) {
        const int i = base + t;
        double st = 0.0, sb = 0.0;
        if (i < n) {
            if (f32)
                sum_slots(pf, n, i, p0, p1, st, sb);
            else
                sum_slots(static_cast<const double *>(M.part), n, i, p0, p1, st, sb);
        }
        if (q > 0) {
            acc[0][q - 1][t] = st;
            acc[1][q - 1][t] = sb;
        }
        __syncthreads();
        if (q == 0 && i < n) {
#pragma unroll
            for (int r = 0; r < kFinishQ - 1; ++r) {
                st += acc[0][r][t];
                sb += acc[1][r][t];
            }
            if (multi) {
                st = M.acc[i] + st;
                sb = M.acc[n + i] + sb;
            }
            double yt = dt * v[i] - st;
            double yb = db * v[n + i] - sb;
            if constexpr (MODE == kFinishRes) {
                yt = M.res_b[i] - yt;
                yb = M.res_b[n + i] - yb;
            }
            out[i] = yt;
            out[n + i] = yb;
            if constexpr (MODE == kFinishDot)
                s = __builtin_fma(yt, M.V[i], __builtin_fma(yb, M.V[n + i], s));
            else if constexpr (MODE == kFinishRes)
                s = __builtin_fma(yt, yt, __builtin_fma(yb, yb, s));
        }
        __syncthreads();  // acc is reused by the next pass
    }
    if constexpr (MODE != kFinishY) {
        s = block_sum(s, lds);
        if (threadIdx.x == 0) M.red[e.y] = s;
    }
}

// ------------------------------------------------------------------ fold
// After pass `pass` of a symmetric product taken in several passes (not its
// last): acc = (acc of the earlier passes, if any) + the pass's slots, added
// as the finish adds them.  Also rearms the symmetric tile queues of this
// precision for the next pass's launch.
__global__ __launch_bounds__(kBlock * kFinishQ) void fold_kernel(
    const Mol *__restrict__ mols, const int2 *__restrict__ list, int precision, int pass,
    int skip, int *__restrict__ counters) {
    __shared__ double accs[2][kFinishQ - 1][kBlock];
    if (blockIdx.x == 0 && threadIdx.x < kXcdLists) counters[kXcdCounters + threadIdx.x] = 0;
    const int2 e = list[blockIdx.x];
    const Mol &M = mols[e.x];
    if (skip && load_done(M.st)) return;
    const int np = precision == GABI_FP64 ? M.np64 : M.np32;
    if (pass >= np - 1) return;
    const int n = M.n, nb = M.nb;
    const int q = threadIdx.x / kBlock, t = threadIdx.x % kBlock;
    const int splits = precision == GABI_FP64 ? M.sp64 : M.sp32;
    const int p0 = q * splits / kFinishQ, p1 = (q + 1) * splits / kFinishQ;
    const float *pf = reinterpret_cast<const float *>(M.part);
    for (int base = e.y * kBlock; base < n; base += nb * kBlock) {
        const int i = base + t;
        double st = 0.0, sb = 0.0;
        if (i < n) {
            if (precision != GABI_FP64)  // several passes: the symmetric scheme
                sum_slots(pf, n, i, p0, p1, st, sb);
            else
                sum_slots(static_cast<const double *>(M.part), n, i, p0, p1, st, sb);
        }
        if (q > 0) {
            accs[0][q - 1][t] = st;
            accs[1][q - 1][t] = sb;
        }
        __syncthreads();
        if (q == 0 && i < n) {
#pragma unroll
            for (int r = 0; r < kFinishQ - 1; ++r) {
                st += accs[0][r][t];
                sb += accs[1][r][t];
            }
            if (pass > 0) {
                st = M.acc[i] + st;
                sb = M.acc[n + i] + sb;
            }
            M.acc[i] = st;
            M.acc[n + i] = sb;
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------ host
void launch_prep(const Batch &b, hipStream_t s, int precision, int mode, int j, bool skip) {
    const dim3 g(b.n_elem), blk(kBlock);
    switch (mode) {
        case kPrepCycle0:
            hipLaunchKernelGGL(prep_kernel<kPrepCycle0>, g, blk, 0, s, b.d_mols, b.d_elem,
                               precision, j, (int)skip);
            break;
        case kPrepCycleJ:
            hipLaunchKernelGGL(prep_kernel<kPrepCycleJ>, g, blk, 0, s, b.d_mols, b.d_elem,
                               precision, j, (int)skip);
            break;
        case kPrepResX:
            hipLaunchKernelGGL(prep_kernel<kPrepResX>, g, blk, 0, s, b.d_mols, b.d_elem,
                               precision, j, (int)skip);
            break;
        default:
            hipLaunchKernelGGL(prep_kernel<kPrepU>, g, blk, 0, s, b.d_mols, b.d_elem,
                               precision, j, (int)skip);
            break;
    }
}

// R = 2 or 1: split scheme with R rows per thread, one queue (counter);
// R = 0: symmetric scheme, lists xoff[0..8] with queues counter[0..7]
template <bool MIXED, int R>
static void pair_group(Batch &b, hipStream_t s, const int4 *tiles, int ntiles, int *counter,
                       int grid_cap, bool skip, const int *xoff = nullptr) {
    if (ntiles == 0) return;
    // the counters are zero: set by the batch upload, rearmed by every finish
    // (and, for the symmetric queues, by the fold between passes)
    const int grid = b.persistent ? std::min(ntiles, grid_cap) : ntiles;
    const int nmol = (int)b.slots.size();
    if constexpr (R == 0)
        hipLaunchKernelGGL((sym_pair_kernel<MIXED>), dim3(grid), dim3(kBlock), 0, s, b.d_mols,
                           nmol, tiles, ntiles, xoff, counter, (int)b.persistent, (int)skip);
    else
        hipLaunchKernelGGL((pair_kernel<MIXED, R>), dim3(grid), dim3(kBlock), 0, s, b.d_mols,
                           nmol, tiles, ntiles, counter, (int)b.persistent, (int)skip);
}

// Records e on s; on a stream under capture the record becomes an
// event-record node of the graph (added by hand after the nodes captured so
// far), so that every replay timestamps it.
static void record_event(hipEvent_t e, hipStream_t s) {
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    unsigned long long id = 0;
    hipGraph_t g = nullptr;
    const hipGraphNode_t *deps = nullptr;
    size_t nd = 0;
    if (hipStreamGetCaptureInfo_v2(s, &st, &id, &g, &deps, &nd) != hipSuccess ||
        st != hipStreamCaptureStatusActive) {
        (void)hipEventRecord(e, s);
        return;
    }
    hipGraphNode_t node = nullptr;
    if (hipGraphAddEventRecordNode(&node, g, deps, nd, e) == hipSuccess)
        (void)hipStreamUpdateCaptureDependencies(s, &node, 1, hipStreamSetCaptureDependencies);
}

void launch_pair(Batch &b, hipStream_t s, int precision, bool skip, const Timer *t) {
    const bool mixed = precision != GABI_FP64;
    const int *cnt = mixed ? b.n_tiles32 : b.n_tiles64;
    const int4 *tiles = mixed ? b.d_tiles32 : b.d_tiles64;
    if (cnt[0] + cnt[1] + cnt[2] == 0) return;
    const int pi = mixed ? 1 : 0;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (t && t->pending[pi]) {
        if (hipEventCreate(&e0) != hipSuccess) {
            e0 = nullptr;
        } else if (hipEventCreate(&e1) != hipSuccess) {
            (void)hipEventDestroy(e0);
            e0 = e1 = nullptr;
        } else {
            record_event(e0, s);
        }
    }
    int *c = b.d_counter + (mixed ? kCountersPerPrecision : 0);
    const int4 *t1 = tiles + cnt[0], *t2 = t1 + cnt[1];
    if (mixed) {
        pair_group<true, 2>(b, s, tiles, cnt[0], c, b.grid32[0], skip);
        pair_group<true, 1>(b, s, t1, cnt[1], c + 1, b.grid32[1], skip);
    } else {
        pair_group<false, 2>(b, s, tiles, cnt[0], c, b.grid64[0], skip);
        pair_group<false, 1>(b, s, t1, cnt[1], c + 1, b.grid64[1], skip);
    }
    // symmetric tiles pass by pass, each pass but the last folded into the
    // accumulator before the next reuses the slots
    const int *off = mixed ? b.sym_off32 : b.sym_off64;
    const int *xoff = mixed ? b.d_xoff32 : b.d_xoff64;
    const int passes = mixed ? b.n_pass32 : b.n_pass64;
    for (int p = 0; p < passes; ++p) {
        const int a = off[p], z = off[p + 1];
        const int *xo = xoff + (size_t)p * (kXcdLists + 1);
        if (mixed)
            pair_group<true, 0>(b, s, t2 + a, z - a, c + kXcdCounters, b.grid32[2], skip, xo);
        else
            pair_group<false, 0>(b, s, t2 + a, z - a, c + kXcdCounters, b.grid64[2], skip, xo);
        if (p + 1 < passes) launch_fold(b, s, precision, p, skip);
    }
    if (e0 && e1) {
        record_event(e1, s);
        t->pending[pi]->push_back({e0, e1});
    }
}

void launch_finish(const Batch &b, hipStream_t s, int precision, int mode, int j, bool skip) {
    const dim3 g(b.n_blas), blk(kBlock * kFinishQ);
    int *c = b.d_counter + (precision == GABI_FP32_PAIR ? kCountersPerPrecision : 0);
    if (mode == kFinishDot)
        hipLaunchKernelGGL(finish_kernel<kFinishDot>, g, blk, 0, s, b.d_mols, b.d_blas,
                           precision, j, (int)skip, c);
    else if (mode == kFinishRes)
        hipLaunchKernelGGL(finish_kernel<kFinishRes>, g, blk, 0, s, b.d_mols, b.d_blas,
                           precision, j, (int)skip, c);
    else
        hipLaunchKernelGGL(finish_kernel<kFinishY>, g, blk, 0, s, b.d_mols, b.d_blas,
                           precision, j, (int)skip, c);
}

void launch_fold(const Batch &b, hipStream_t s, int precision, int pass, bool skip) {
    int *c = b.d_counter + (precision == GABI_FP64 ? 0 : kCountersPerPrecision);
    hipLaunchKernelGGL(fold_kernel, dim3(b.n_blas), dim3(kBlock * kFinishQ), 0, s, b.d_mols,
                       b.d_blas, precision, pass, (int)skip, c);
}

template <typename K>
static int resident_blocks(K kernel) {
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 1024;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 1024;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kBlock, 0) != hipSuccess ||
        per_cu < 1)
        per_cu = 1;
    return per_cu * cus;
}

// Workgroups of a pair-kernel variant resident on the whole device at once
// (the persistent grid size): variant 0 split with R = 2, 1 split with R = 1,
// 2 symmetric.
int pair_occupancy_grid(int precision, int variant) {
    if (precision == GABI_FP64)
        return variant == 0   ? resident_blocks(pair_kernel<false, 2>)
               : variant == 1 ? resident_blocks(pair_kernel<false, 1>)
                              : resident_blocks(sym_pair_kernel<false>);
    return variant == 0   ? resident_blocks(pair_kernel<true, 2>)
           : variant == 1 ? resident_blocks(pair_kernel<true, 1>)
                          : resident_blocks(sym_pair_kernel<true>);
}

}  // namespace gabi
