// Treecode approximation of the boundary-integral product y = A u of
// arXiv:1301.5885 (Section 2.2, eqs. (eqdbef1)/(eqdbef2)); the paper names
// tree codes, O(N log N), as the route past its O(N^2) direct sum
// (Section 1; Section 4).  The method is the barycentric Lagrange treecode
// (BLTC) of Wang, Krasny and Tlupova (Commun. Comput. Phys. 28, 2020) in
// its particle-cluster form with target batches:
//
//  * tree (host): the element centroids are split recursively; a node keeps
//    the minimal box of its points and, with more than `leaf` points, is cut
//    at the box midpoint in every dimension whose extent is at least 1/sqrt 2
//    of the largest (points with coordinate >= midpoint go up); children are
//    kept in the order of their bit codes, empty ones dropped.  Elements are
//    renumbered in depth-first leaf order (increasing index within a leaf),
//    so every node is a contiguous range.  Leaves are the target batches.
//  * proxies: a cluster with more than P = (n+1)^3 elements that acts on
//    some batch through interpolation carries the tensor Chebyshev points of
//    the second kind of its box and modified weights
//    W_k = sum_{j in C} L_k(y_j) w_j, L_k the product of barycentric Lagrange
//    bases, w_j = (s_j, m_j) the element's weights of the product.
//  * interactions (host): for batch B each cluster C is visited from the
//    root; (r_B + r_C)^2 < theta^2 R^2 makes C act through its proxies (or
//    directly when it has at most P elements), else a leaf acts directly and
//    an inner node hands over to its children.
//
// Per product five kernels run: weights in tree order (tree_prep), the
// modified weights of every proxy cluster in pieces of 256-2,048 elements
// (tree_weights, one workgroup per piece, so that the largest clusters do
// not serialise the launch and small trees still fill the device) and their sum in piece order
// (tree_wsum), the sums (tree_eval) and their reduction (tree_finish).  A batch's interaction
// list is cut into work items of a bounded number of sources, one workgroup
// each: the item's sources are staged through LDS up to 256 records at a
// time, consecutive list entries packed into one stage (the entry holding
// the batch's own elements is staged alone), and every target of the batch
// is served by 256/H threads (H half the batch size, rounded up; integer
// division), each thread serving two targets, that take interleaved
// sources, their sums added in thread order; the item writes one partial per target, and
// tree_finish adds a batch's items in list order.  In the treecode
// refinement (GABI_SOLVE_TREE_IR) the same kernels form the inner products of
// a GMRES cycle: the finish then stores the sums in element order as the
// molecule's single partial-sum slot, the Arnoldi finish applies the diagonal
// and the dot products, and every kernel returns at once once the cycle has
// ended (the round's later steps).  The pair arithmetic is
// the direct product's, FP64 (or, on request, FP32 as in the FP32-pair
// product).  Every sum is taken in a fixed order, so results are
// reproducible bit for bit.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <functional>
#include <type_traits>
#include <vector>

#include "arnoldi.h"
#include "gabi_internal.h"
#include "pair_math.h"

namespace gabi {

constexpr int kTreeMaxDeg = 8;        // P <= 729 proxies per cluster
constexpr int kTreeMaxLeaf = kBlock;  // a batch fits one workgroup

struct TreeNode {
    double lo[3], hi[3];
    int begin = 0, end = 0;  // range in tree order
    std::vector<int> children;
    int proxy = -1;          // index of its proxy cluster, if it has one
};

struct TreeState {
    // what the tree was built for
    int64_t version = -1;
    double theta = -1.0;
    int degree = -1, leaf = -1;
    // host
    std::vector<TreeNode> nodes;
    std::vector<int> perm;  // tree position -> element index
    gabi_tree_info info{};
    int n = 0, P = 0, n_clusters = 0, n_batches = 0;
    double bary[kTreeMaxDeg + 1] = {0};
    // device block
    void *mem = nullptr;
    int64_t bytes = 0;
    double4 *spos = nullptr, *snrm = nullptr, *sw = nullptr, *ppos = nullptr, *pw = nullptr;
    // FP32 copies for the FP32 evaluation: positions relative to the centre
    // of the surface's bounding box (rounded once), normals, weights
    float4 *spos32 = nullptr, *snrm32 = nullptr, *sw32 = nullptr, *ppos32 = nullptr,
           *pw32 = nullptr;
    int *perm_d = nullptr;
    double *cheb = nullptr;   // 3 (n+1) nodes per cluster
    int4 *clusters = nullptr;  // (begin, end, proxy offset, first piece)
    int4 *batches = nullptr;   // (begin, end, first item, item count)
    int4 *list = nullptr;      // (0 near | 1 far, begin, end, 0)
    int4 *items = nullptr;     // (batch, list begin, list end, 0)
    double2 *ipart = nullptr;  // [item][kBlock] partial (top, bot) per target
    int n_items = 0;
    int4 *pieces = nullptr;    // (cluster, element begin, element end, 0)
    double4 *wpart = nullptr;  // [piece][P] partial modified weights
    int n_pieces = 0;
    int piece = 0;             // elements per piece (the last of a cluster: fewer)
    int64_t generation = 0;  // counts rebuilds (captured rounds compare it)
};

namespace {

int build_node(TreeState &T, const double4 *pos, std::vector<int> idx, int leaf) {
    const int id = (int)T.nodes.size();
    T.nodes.emplace_back();
    {
        TreeNode &nd = T.nodes[id];
        for (int d = 0; d < 3; ++d) {
            nd.lo[d] = INFINITY;
            nd.hi[d] = -INFINITY;
        }
        for (int j : idx) {
            const double c[3] = {pos[j].x, pos[j].y, pos[j].z};
            for (int d = 0; d < 3; ++d) {
                nd.lo[d] = std::min(nd.lo[d], c[d]);
                nd.hi[d] = std::max(nd.hi[d], c[d]);
            }
        }
        nd.begin = (int)T.perm.size();
    }
    double ext[3], mid[3], L = 0.0;
    for (int d = 0; d < 3; ++d) {
        ext[d] = T.nodes[id].hi[d] - T.nodes[id].lo[d];
        mid[d] = (T.nodes[id].lo[d] + T.nodes[id].hi[d]) / 2.0;
        L = std::max(L, ext[d]);
    }
    if ((int)idx.size() <= leaf || L == 0.0) {
        T.perm.insert(T.perm.end(), idx.begin(), idx.end());
        T.nodes[id].end = (int)T.perm.size();
        return id;
    }
    int dims[3], nd = 0;
    for (int d = 0; d < 3; ++d)
        if (ext[d] >= L / std::sqrt(2.0)) dims[nd++] = d;
    std::vector<std::vector<int>> parts((size_t)1 << nd);
    for (int j : idx) {
        const double c[3] = {pos[j].x, pos[j].y, pos[j].z};
        int code = 0;
        for (int t = 0; t < nd; ++t)
            if (c[dims[t]] >= mid[dims[t]]) code |= 1 << t;
        parts[(size_t)code].push_back(j);
    }
    for (auto &p : parts) {
        if (p.empty()) continue;
        const int child = build_node(T, pos, std::move(p), leaf);
        T.nodes[id].children.push_back(child);
    }
    T.nodes[id].end = (int)T.perm.size();
    return id;
}

void centre_radius(const TreeNode &nd, double c[3], double &r) {
    double h[3];
    for (int d = 0; d < 3; ++d) {
        c[d] = (nd.lo[d] + nd.hi[d]) / 2.0;
        h[d] = (nd.hi[d] - nd.lo[d]) / 2.0;
    }
    r = std::sqrt(h[0] * h[0] + h[1] * h[1] + h[2] * h[2]);
}

// Builds the tree, the interaction lists and the statistics on the host.
// Outputs the lists as (kind, node) pairs per batch.
void plan(TreeState &T, const double4 *pos, int64_t n, double theta, int degree, int leaf,
          std::vector<int> &batch_nodes, std::vector<std::vector<std::pair<int, int>>> &lists) {
    T.nodes.clear();
    T.perm.clear();
    T.nodes.reserve((size_t)(4 * n / std::max(1, leaf) + 16));
    std::vector<int> all((size_t)n);
    for (int64_t j = 0; j < n; ++j) all[(size_t)j] = (int)j;
    build_node(T, pos, std::move(all), leaf);
    T.n = (int)n;
    T.P = (degree + 1) * (degree + 1) * (degree + 1);
    batch_nodes.clear();
    for (int i = 0; i < (int)T.nodes.size(); ++i)
        if (T.nodes[(size_t)i].children.empty()) batch_nodes.push_back(i);
    // leaves in tree order (their ranges increase)
    std::sort(batch_nodes.begin(), batch_nodes.end(),
              [&](int a, int b) { return T.nodes[(size_t)a].begin < T.nodes[(size_t)b].begin; });
    lists.assign(batch_nodes.size(), {});
    gabi_tree_info info{};
    info.leaves = (int64_t)batch_nodes.size();
    const double th2 = theta * theta;
    int n_clusters = 0;
    for (size_t b = 0; b < batch_nodes.size(); ++b) {
        const TreeNode &B = T.nodes[(size_t)batch_nodes[b]];
        double cb[3], rb;
        centre_radius(B, cb, rb);
        const int64_t nb = B.end - B.begin;
        auto &lst = lists[b];
        std::function<void(int)> visit = [&](int ci) {
            TreeNode &C = T.nodes[(size_t)ci];
            double cc[3], rc;
            centre_radius(C, cc, rc);
            const double d0 = cb[0] - cc[0], d1 = cb[1] - cc[1], d2 = cb[2] - cc[2];
            const double R2 = d0 * d0 + d1 * d1 + d2 * d2;
            const double rr = rb + rc;
            const int64_t cnt = C.end - C.begin;
            if (rr * rr < th2 * R2) {
                if (cnt > T.P) {
                    if (C.proxy < 0) C.proxy = n_clusters++;
                    lst.emplace_back(1, ci);
                    info.far_entries++;
                    info.far_pairs += (int64_t)T.P * nb;
                } else {
                    lst.emplace_back(0, ci);
                    info.near_entries++;
                    info.near_pairs += cnt * nb;
                }
            } else if (C.children.empty()) {
                lst.emplace_back(0, ci);
                info.near_entries++;
                info.near_pairs += cnt * nb;
            } else {
                for (int ch : C.children) visit(ch);
            }
        };
        visit(0);
    }
    info.clusters_with_proxies = n_clusters;
    T.n_clusters = n_clusters;
    T.n_batches = (int)batch_nodes.size();
    T.info = info;
}

int validate_tree_opts(const gabi_tree_opts *o, std::string &msg) {
    if (!o) {
        msg = "null treecode options";
        return GABI_EINVAL;
    }
    if (!(o->theta >= 0.0 && o->theta < 1.0)) {
        msg = "theta must be in [0, 1)";
        return GABI_EINVAL;
    }
    if (o->degree < 1 || o->degree > kTreeMaxDeg) {
        msg = "degree must be in [1, " + std::to_string(kTreeMaxDeg) + "]";
        return GABI_EINVAL;
    }
    if (o->leaf_size < 1 || o->leaf_size > kTreeMaxLeaf) {
        msg = "leaf_size must be in [1, " + std::to_string(kTreeMaxLeaf) + "]";
        return GABI_EINVAL;
    }
    if (o->precision != GABI_FP64 && o->precision != GABI_FP32_PAIR) {
        msg = "precision must be GABI_FP64 or GABI_FP32_PAIR";
        return GABI_EINVAL;
    }
    return GABI_OK;
}

// Chebyshev points of the second kind of a cluster's box, per dimension
// (flat dimensions widened to 1e-6 of the largest half-width).
void cheb_nodes(const TreeNode &C, int degree, double *out) {
    double hw[3], mid[3], big = 0.0;
    for (int d = 0; d < 3; ++d) {
        hw[d] = (C.hi[d] - C.lo[d]) / 2.0;
        mid[d] = (C.lo[d] + C.hi[d]) / 2.0;
        big = std::max(big, hw[d]);
    }
    for (int d = 0; d < 3; ++d) {
        const double h = std::max(hw[d], 1e-6 * big);
        for (int k = 0; k <= degree; ++k)
            out[d * (degree + 1) + k] = mid[d] + h * std::cos(k * kPi / degree);
    }
}

}  // namespace

// ------------------------------------------------------------------ kernels
struct TreeDev {
    const double4 *spos, *snrm;
    double4 *sw;
    const double4 *ppos;
    double4 *pw;
    const float4 *spos32, *snrm32, *ppos32;
    float4 *sw32, *pw32;
    const int *perm;
    const double *cheb;
    const int4 *clusters, *batches, *list, *items, *pieces;
    double2 *ipart;
    double4 *wpart;
    int n, degree, P, piece;
    double bary[kTreeMaxDeg + 1];
};

// Weights of the product in tree order: s = W psi/(4 pi), m = W phi nu/(4 pi)
// (F32: also rounded to FP32 for the FP32 evaluation).
template <bool F32>
__global__ __launch_bounds__(kBlock) void tree_prep_kernel(TreeDev T, const double *__restrict__ u,
                                                          const KrylovStatus *st, int skip) {
    if (skip && load_done(st)) return;
    const int p = blockIdx.x * kBlock + threadIdx.x;
    if (p >= T.n) return;
    const int j = T.perm[p];
    const double4 q = T.spos[p], nu = T.snrm[p];
    const double c = q.w * (1.0 / (4.0 * kPi));
    const double s = c * u[T.n + j], t = c * u[j];
    const double4 w = make_double4(s, t * nu.x, t * nu.y, t * nu.z);
    T.sw[p] = w;
    if constexpr (F32) T.sw32[p] = make_float4((float)w.x, (float)w.y, (float)w.z, (float)w.w);
}

// Partial modified weights of one piece (at most T.piece elements) of a
// proxy cluster: W_k = sum_j L_k(y_j) w_j over the piece's elements in tree
// order.  The 1-D bases of 64 elements are formed at a time (one (element,
// dimension) per thread), then each thread adds the chunk's terms to its
// proxies k = tid, tid + 256, ...
constexpr int kTreeChunk = 64;
constexpr int kTreeProxPerThread = (729 + kBlock - 1) / kBlock;
// elements per workgroup of the modified weights: the largest power of two
// in [kTreePieceMin, kTreePieceMax] that still gives kTreePieceGroups pieces
constexpr int kTreePieceMax = 2048, kTreePieceMin = 256, kTreePieceGroups = 1024;

__global__ __launch_bounds__(kBlock) void tree_weights_kernel(TreeDev T, const KrylovStatus *st,
                                                             int skip) {
    __shared__ double s_l[3][kTreeChunk][kTreeMaxDeg + 1];
    __shared__ double4 s_w[kTreeChunk];
    if (skip && load_done(st)) return;
    const int4 pc = T.pieces[blockIdx.x];
    const int deg = T.degree, np1 = deg + 1;
    const double *nodes = T.cheb + (size_t)pc.x * 3 * np1;
    double4 acc[kTreeProxPerThread];
#pragma unroll
    for (int r = 0; r < kTreeProxPerThread; ++r) acc[r] = make_double4(0.0, 0.0, 0.0, 0.0);
    for (int c0 = pc.y; c0 < pc.z; c0 += kTreeChunk) {
        const int cnt = min(kTreeChunk, pc.z - c0);
        __syncthreads();
        if (threadIdx.x < 3 * kTreeChunk) {
            const int e = threadIdx.x / 3, d = threadIdx.x % 3;
            if (e < cnt) {
                const double4 q = T.spos[c0 + e];
                const double y = d == 0 ? q.x : d == 1 ? q.y : q.z;
                const double *s = nodes + d * np1;
                int hit = -1;
                double sum = 0.0;
                for (int k = 0; k < np1; ++k) {
                    const double diff = y - s[k];
                    if (diff == 0.0 && hit < 0) hit = k;
                    const double qk = T.bary[k] / diff;
                    s_l[d][e][k] = qk;
                    sum += qk;
                }
                for (int k = 0; k < np1; ++k)
                    s_l[d][e][k] = hit >= 0 ? (k == hit ? 1.0 : 0.0) : s_l[d][e][k] / sum;
            }
        } else if (threadIdx.x - 3 * kTreeChunk < cnt) {
            const int e = threadIdx.x - 3 * kTreeChunk;
            s_w[e] = T.sw[c0 + e];
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < kTreeProxPerThread; ++r) {
            const int k = threadIdx.x + r * kBlock;
            if (k >= T.P) break;
            const int k1 = k / (np1 * np1), k2 = (k / np1) % np1, k3 = k % np1;
            double4 a = acc[r];
            for (int e = 0; e < cnt; ++e) {
                const double L = s_l[0][e][k1] * s_l[1][e][k2] * s_l[2][e][k3];
                const double4 w = s_w[e];
                a.x = __builtin_fma(L, w.x, a.x);
                a.y = __builtin_fma(L, w.y, a.y);
                a.z = __builtin_fma(L, w.z, a.z);
                a.w = __builtin_fma(L, w.w, a.w);
            }
            acc[r] = a;
        }
    }
#pragma unroll
    for (int r = 0; r < kTreeProxPerThread; ++r) {
        const int k = threadIdx.x + r * kBlock;
        if (k < T.P) T.wpart[(size_t)blockIdx.x * T.P + k] = acc[r];
    }
}

// Modified weights of one proxy cluster: its pieces' partials added in piece
// order (F32: also rounded to FP32).
template <bool F32>
__global__ __launch_bounds__(kBlock) void tree_wsum_kernel(TreeDev T, const KrylovStatus *st,
                                                          int skip) {
    if (skip && load_done(st)) return;
    const int4 cl = T.clusters[blockIdx.x];
    const int k = (int)(blockIdx.y * kBlock + threadIdx.x);
    if (k >= T.P) return;
    const int count = (cl.y - cl.x + T.piece - 1) / T.piece;
    double4 a = T.wpart[(size_t)cl.w * T.P + k];
    for (int q = 1; q < count; ++q) {
        const double4 v = T.wpart[(size_t)(cl.w + q) * T.P + k];
        a.x += v.x;
        a.y += v.y;
        a.z += v.z;
        a.w += v.w;
    }
    T.pw[(size_t)cl.z + k] = a;
    if constexpr (F32) T.pw32[(size_t)cl.z + k] = make_float4((float)a.x, (float)a.y, (float)a.z, (float)a.w);
}

// The sums of one work item: the batch's targets against the sources of its
// list entries [l0, l1) in list order (near: elements, the target itself
// skipped; far: proxies), staged in list order up to kBlock at a time.
// Each thread serves two targets, t and t + H of the batch's P (H = the
// half of P rounded up; the second is absent when t + H = P), so that a
// staged source is read once for two pair terms.  With G = 256 / H
// (integer division), thread t < G H serves targets t mod H and
// t mod H + H with the staged sources j = t / H (mod G) of every stage; a
// target's G sums are added in thread order through LDS and stored as the
// item's partial.  F32: the pair terms in FP32 (the direct product's
// pair_f32, on coordinates relative to the centre of the surface's bounding
// box), each stage summed in FP32 and added to FP64 sums.
template <bool F32>
__global__ __launch_bounds__(kBlock) void tree_eval_kernel(TreeDev T, PairConstF64 pc,
                                                          PairConstF32 pc32,
                                                          const KrylovStatus *st, int skip) {
    using V4 = typename std::conditional<F32, float4, double4>::type;
    __shared__ V4 s_pos[kBlock];
    __shared__ V4 s_w[kBlock];
    __shared__ double2 s_sum[2][kBlock];
    if (skip && load_done(st)) return;
    const int4 item = T.items[blockIdx.x];
    const int4 bt = T.batches[item.x];
    const int P = bt.y - bt.x;  // 1 <= P <= kBlock targets
    const int H = (P + 1) / 2;
    const int G = kBlock / H;
    const int tid = (int)threadIdx.x, tg = tid % H, grp = tid / H;
    const bool act = grp < G;           // the last kBlock mod H threads idle
    const bool two = tg + H < P;        // the thread's second target exists
    const int pa = bt.x + tg;
    const int pb = two ? pa + H : pa;   // (absent: a copy of the first, discarded)
    V4 xa, na, xb, nb;
    if constexpr (F32) {
        xa = T.spos32[pa];
        na = T.snrm32[pa];
        xb = T.spos32[pb];
        nb = T.snrm32[pb];
    } else {
        xa = T.spos[pa];
        na = T.snrm[pa];
        xb = T.spos[pb];
        nb = T.snrm[pb];
    }
    double topa = 0.0, bota = 0.0, topb = 0.0, botb = 0.0;
    int e = item.y, off = 0;  // the next source: offset off into entry e
    while (e < item.z) {
        // One stage: either the rest (up to kBlock elements) of the entry
        // that holds the batch's own elements, staged alone so that each
        // target can skip itself, or up to kBlock sources taken from
        // consecutive other entries, near and far alike.
        int fill = 0, self0 = -1;  // self0 >= 0: the own entry's first staged element
        __syncthreads();
        for (;;) {
            const int4 it = T.list[e];
            const bool far = it.x == 1;
            const bool own = !far && it.y < bt.y && it.z > bt.x;
            if (own && fill > 0) break;
            const V4 *src_p, *src_w;
            if constexpr (F32) {
                src_p = far ? T.ppos32 : T.spos32;
                src_w = far ? T.pw32 : T.sw32;
            } else {
                src_p = far ? T.ppos : T.spos;
                src_w = far ? T.pw : T.sw;
            }
            const int j0 = it.y + off;
            const int take = min(kBlock - fill, it.z - j0);
            if (tid < take) {
                s_pos[fill + tid] = src_p[j0 + tid];
                s_w[fill + tid] = src_w[j0 + tid];
            }
            if (own) self0 = j0;
            fill += take;
            off += take;
            if (j0 + take == it.z) {
                ++e;
                off = 0;
            }
            if (own || fill == kBlock || e == item.z) break;
        }
        __syncthreads();
        if (!act) continue;
        // the staged elements that are the thread's own targets (none
        // outside the own entry's stage, whose loop alone carries the test)
        const int skip_a = self0 >= 0 ? pa - self0 : -1;
        const int skip_b = self0 >= 0 ? pb - self0 : -1;
        if constexpr (F32) {
            float ta = 0.0f, ba = 0.0f, tb = 0.0f, bb = 0.0f;
            auto run = [&](auto test) {
                for (int jj = grp; jj < fill; jj += G) {
                    const float4 q = s_pos[jj], w = s_w[jj];
                    if (!(test && jj == skip_a))
                        pair_f32(pc32, xa.x, xa.y, xa.z, na.x, na.y, na.z, q.x, q.y, q.z, w.x,
                                 w.y, w.z, w.w, ta, ba);
                    if (!(test && jj == skip_b))
                        pair_f32(pc32, xb.x, xb.y, xb.z, nb.x, nb.y, nb.z, q.x, q.y, q.z, w.x,
                                 w.y, w.z, w.w, tb, bb);
                }
            };
            if (self0 >= 0) run(std::true_type{});
            else run(std::false_type{});
            topa += (double)ta;
            bota += (double)ba;
            topb += (double)tb;
            botb += (double)bb;
        } else {
            auto run = [&](auto test) {
                for (int jj = grp; jj < fill; jj += G) {
                    const double4 q = s_pos[jj], w = s_w[jj];
                    if (!(test && jj == skip_a))
                        pair_f64(pc, xa.x, xa.y, xa.z, na.x, na.y, na.z, q.x, q.y, q.z, w.x, w.y,
                                 w.z, w.w, topa, bota);
                    if (!(test && jj == skip_b))
                        pair_f64(pc, xb.x, xb.y, xb.z, nb.x, nb.y, nb.z, q.x, q.y, q.z, w.x, w.y,
                                 w.z, w.w, topb, botb);
                }
            };
            if (self0 >= 0) run(std::true_type{});
            else run(std::false_type{});
        }
    }
    __syncthreads();
    s_sum[0][tid] = make_double2(topa, bota);
    s_sum[1][tid] = make_double2(topb, botb);
    __syncthreads();
    if (grp == 0) {
        for (int h = 0; h < (two ? 2 : 1); ++h) {
            double2 acc = s_sum[h][tg];
            for (int g = 1; g < G; ++g) {
                const double2 v = s_sum[h][g * H + tg];
                acc.x += v.x;
                acc.y += v.y;
            }
            T.ipart[(size_t)blockIdx.x * kBlock + tg + h * H] = acc;
        }
    }
}

// MODE kTreeY:    y = D u - sums at the elements' own indices;
//      kTreeSlot: the sums themselves, top at out[j], bot at out[n + j] (a
//                 partial-sum slot of the Arnoldi finish).
// A batch's item partials are added in list order.
enum TreeFinish { kTreeY = 0, kTreeSlot = 1 };

template <int MODE>
__global__ __launch_bounds__(kBlock) void tree_finish_kernel(TreeDev T, double d_top,
                                                            double d_bot,
                                                            const double *__restrict__ u,
                                                            double *__restrict__ y,
                                                            const KrylovStatus *st, int skip) {
    if (skip && load_done(st)) return;
    const int4 bt = T.batches[blockIdx.x];
    const int tg = (int)threadIdx.x;
    if (tg >= bt.y - bt.x) return;
    double top = 0.0, bot = 0.0;
    for (int k = bt.z; k < bt.z + bt.w; ++k) {
        const double2 v = T.ipart[(size_t)k * kBlock + tg];
        top += v.x;
        bot += v.y;
    }
    const int j = T.perm[bt.x + tg];
    if constexpr (MODE == kTreeY) {
        y[j] = d_top * u[j] - top;
        y[T.n + j] = d_bot * u[T.n + j] - bot;
    } else {
        y[j] = top;
        y[T.n + j] = bot;
    }
}

// ------------------------------------------------------------------ host
void tree_free(TreeState *T) {
    if (!T) return;
    if (T->mem) (void)hipFree(T->mem);
    delete T;
}

namespace {

// Device vectors u, y of 2N doubles for the host entry point (one block).
int tree_io_buffers(gabi_ctx *ctx) {
    if (ctx->tree_u && ctx->tree_io_n == ctx->n) return GABI_OK;
    if (ctx->stream) GABI_HIP(ctx, hipStreamSynchronize(ctx->stream));
    if (ctx->tree_u) (void)hipFree(ctx->tree_u);
    ctx->tree_u = ctx->tree_y = nullptr;
    ctx->tree_io_n = 0;
    hipError_t e = hipMalloc(&ctx->tree_u, sizeof(double) * 4 * (size_t)ctx->n);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        ctx->tree_u = nullptr;
        return fail(ctx, GABI_ENOMEM, "treecode vector allocation failed");
    }
    ctx->tree_y = ctx->tree_u + 2 * ctx->n;
    ctx->tree_io_n = ctx->n;
    return GABI_OK;
}

// (Re)builds the tree, its lists and device data when the surface or the
// options changed.
int tree_ensure(gabi_ctx *ctx, const gabi_tree_opts *o) {
    std::string msg;
    int rc = validate_tree_opts(o, msg);
    if (rc) return fail(ctx, rc, msg);
    if (!ctx->tree) ctx->tree = new (std::nothrow) TreeState();
    if (!ctx->tree) return fail(ctx, GABI_ENOMEM, "treecode state allocation failed");
    TreeState &T = *ctx->tree;
    if (T.version == ctx->geom_version && T.theta == o->theta && T.degree == o->degree &&
        T.leaf == o->leaf_size && T.mem)
        return GABI_OK;
    const int64_t n = ctx->n;
    const double4 *pos = ctx->host_pos.data();
    const double4 *nrm = ctx->host_nrm.data();
    std::vector<int> batch_nodes;
    std::vector<std::vector<std::pair<int, int>>> lists;
    plan(T, pos, n, o->theta, o->degree, o->leaf_size, batch_nodes, lists);
    const int deg = o->degree, np1 = deg + 1;
    for (int k = 0; k <= deg; ++k)
        T.bary[k] = (k % 2 ? -1.0 : 1.0) * ((k == 0 || k == deg) ? 0.5 : 1.0);
    // host images of the device arrays
    std::vector<double4> spos((size_t)n), snrm((size_t)n);
    for (int64_t p = 0; p < n; ++p) {
        spos[(size_t)p] = pos[T.perm[(size_t)p]];
        snrm[(size_t)p] = nrm[T.perm[(size_t)p]];
    }
    // centre of the bounding box (the FP32 copies are relative to it)
    double cen[3];
    {
        const TreeNode &R = T.nodes[0];
        for (int d = 0; d < 3; ++d) cen[d] = (R.lo[d] + R.hi[d]) / 2.0;
    }
    std::vector<float4> spos32((size_t)n), snrm32((size_t)n);
    for (int64_t p = 0; p < n; ++p) {
        const double4 a = spos[(size_t)p], b = snrm[(size_t)p];
        spos32[(size_t)p] = make_float4((float)(a.x - cen[0]), (float)(a.y - cen[1]),
                                        (float)(a.z - cen[2]), 0.0f);
        snrm32[(size_t)p] = make_float4((float)b.x, (float)b.y, (float)b.z, 0.0f);
    }
    const int nc = T.n_clusters;
    std::vector<double> cheb((size_t)nc * 3 * np1);
    std::vector<int4> clusters((size_t)nc);
    std::vector<double4> ppos((size_t)nc * T.P);
    for (const TreeNode &C : T.nodes) {
        if (C.proxy < 0) continue;
        double *cn = cheb.data() + (size_t)C.proxy * 3 * np1;
        cheb_nodes(C, deg, cn);
        clusters[(size_t)C.proxy] = make_int4(C.begin, C.end, C.proxy * T.P, 0);
        for (int k = 0; k < T.P; ++k) {
            const int k1 = k / (np1 * np1), k2 = (k / np1) % np1, k3 = k % np1;
            ppos[(size_t)C.proxy * T.P + k] =
                make_double4(cn[k1], cn[np1 + k2], cn[2 * np1 + k3], 0.0);
        }
    }
    // pieces of at most T.piece elements per proxy cluster, in cluster
    // order, so that large clusters spread over many workgroups; smaller
    // pieces where the clusters hold few elements in all, so that the launch
    // still has about kTreePieceGroups workgroups
    int64_t members = 0;
    for (int c = 0; c < nc; ++c) members += clusters[(size_t)c].y - clusters[(size_t)c].x;
    T.piece = kTreePieceMax;
    while (T.piece > kTreePieceMin && members / T.piece < kTreePieceGroups) T.piece /= 2;
    std::vector<int4> pieces;
    for (int c = 0; c < nc; ++c) {
        clusters[(size_t)c].w = (int)pieces.size();
        for (int b0 = clusters[(size_t)c].x; b0 < clusters[(size_t)c].y; b0 += T.piece)
            pieces.push_back(make_int4(c, b0, std::min(b0 + T.piece, clusters[(size_t)c].y), 0));
    }
    T.n_pieces = (int)pieces.size();
    std::vector<float4> ppos32(ppos.size());
    for (size_t k = 0; k < ppos.size(); ++k)
        ppos32[k] = make_float4((float)(ppos[k].x - cen[0]), (float)(ppos[k].y - cen[1]),
                                (float)(ppos[k].z - cen[2]), 0.0f);
    std::vector<int4> batches(batch_nodes.size()), list, items;
    int64_t total_src = 0;
    for (size_t b = 0; b < batch_nodes.size(); ++b)
        for (auto &kn : lists[b]) {
            const TreeNode &C = T.nodes[(size_t)kn.second];
            total_src += kn.first == 1 ? T.P : (C.end - C.begin);
        }
    // sources per work item: enough items to fill the device several times
    // over, each item at least a few LDS stages
    const int64_t item_src = std::min<int64_t>(
        32768, std::max<int64_t>(1024, total_src / 8192 / 256 * 256));
    for (size_t b = 0; b < batch_nodes.size(); ++b) {
        const TreeNode &B = T.nodes[(size_t)batch_nodes[b]];
        const int first_item = (int)items.size();
        int l0 = (int)list.size();
        int64_t acc = 0;
        for (auto &kn : lists[b]) {
            const TreeNode &C = T.nodes[(size_t)kn.second];
            const int64_t cnt = kn.first == 1 ? T.P : (C.end - C.begin);
            if (acc > 0 && acc + cnt > item_src) {  // close the item before this entry
                items.push_back(make_int4((int)b, l0, (int)list.size(), 0));
                l0 = (int)list.size();
                acc = 0;
            }
            if (kn.first == 1)
                list.push_back(make_int4(1, C.proxy * T.P, C.proxy * T.P + T.P, 0));
            else
                list.push_back(make_int4(0, C.begin, C.end, 0));
            acc += cnt;
        }
        items.push_back(make_int4((int)b, l0, (int)list.size(), 0));
        batches[b] = make_int4(B.begin, B.end, first_item, (int)items.size() - first_item);
    }
    T.n_items = (int)items.size();
    // one device block
    auto al = [](int64_t v) { return (v + 255) & ~int64_t(255); };
    const int64_t o_spos = 0;
    const int64_t o_snrm = al(o_spos + 32 * n);
    const int64_t o_sw = al(o_snrm + 32 * n);
    const int64_t o_ppos = al(o_sw + 32 * n);
    const int64_t o_pw = al(o_ppos + 32 * std::max<int64_t>(1, (int64_t)ppos.size()));
    const int64_t o_perm = al(o_pw + 32 * std::max<int64_t>(1, (int64_t)ppos.size()));
    const int64_t o_cheb = al(o_perm + 4 * n);
    const int64_t o_cl = al(o_cheb + 8 * std::max<int64_t>(1, (int64_t)cheb.size()));
    const int64_t o_bt = al(o_cl + 16 * std::max<int64_t>(1, (int64_t)nc));
    const int64_t o_li = al(o_bt + 16 * (int64_t)batches.size());
    const int64_t o_it = al(o_li + 16 * std::max<int64_t>(1, (int64_t)list.size()));
    const int64_t o_ip = al(o_it + 16 * (int64_t)items.size());
    const int64_t np_ = std::max<int64_t>(1, (int64_t)ppos.size());
    const int64_t o_sp32 = al(o_ip + 16 * (int64_t)kBlock * (int64_t)items.size());
    const int64_t o_sn32 = al(o_sp32 + 16 * n);
    const int64_t o_sw32 = al(o_sn32 + 16 * n);
    const int64_t o_pp32 = al(o_sw32 + 16 * n);
    const int64_t o_pw32 = al(o_pp32 + 16 * np_);
    const int64_t o_pc = al(o_pw32 + 16 * np_);
    const int64_t o_wp = al(o_pc + 16 * std::max<int64_t>(1, (int64_t)pieces.size()));
    const int64_t total = al(o_wp + 32 * (int64_t)T.P * std::max<int64_t>(1, (int64_t)pieces.size()));
    if (ctx->stream) GABI_HIP(ctx, hipStreamSynchronize(ctx->stream));
    if (T.mem) (void)hipFree(T.mem);
    T.mem = nullptr;
    T.version = -1;
    hipError_t e = hipMalloc(&T.mem, total);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        T.mem = nullptr;
        return fail(ctx, GABI_ENOMEM, "treecode device allocation failed");
    }
    T.bytes = total;
    char *base = static_cast<char *>(T.mem);
    T.spos = reinterpret_cast<double4 *>(base + o_spos);
    T.snrm = reinterpret_cast<double4 *>(base + o_snrm);
    T.sw = reinterpret_cast<double4 *>(base + o_sw);
    T.ppos = reinterpret_cast<double4 *>(base + o_ppos);
    T.pw = reinterpret_cast<double4 *>(base + o_pw);
    T.perm_d = reinterpret_cast<int *>(base + o_perm);
    T.cheb = reinterpret_cast<double *>(base + o_cheb);
    T.clusters = reinterpret_cast<int4 *>(base + o_cl);
    T.batches = reinterpret_cast<int4 *>(base + o_bt);
    T.list = reinterpret_cast<int4 *>(base + o_li);
    T.items = reinterpret_cast<int4 *>(base + o_it);
    T.ipart = reinterpret_cast<double2 *>(base + o_ip);
    T.spos32 = reinterpret_cast<float4 *>(base + o_sp32);
    T.snrm32 = reinterpret_cast<float4 *>(base + o_sn32);
    T.sw32 = reinterpret_cast<float4 *>(base + o_sw32);
    T.ppos32 = reinterpret_cast<float4 *>(base + o_pp32);
    T.pw32 = reinterpret_cast<float4 *>(base + o_pw32);
    T.pieces = reinterpret_cast<int4 *>(base + o_pc);
    T.wpart = reinterpret_cast<double4 *>(base + o_wp);
    auto up = [&](void *dst, const void *src, size_t bytes) -> hipError_t {
        return bytes ? hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, ctx->stream)
                     : hipSuccess;
    };
    GABI_HIP(ctx, up(T.spos, spos.data(), 32 * (size_t)n));
    GABI_HIP(ctx, up(T.snrm, snrm.data(), 32 * (size_t)n));
    GABI_HIP(ctx, up(T.ppos, ppos.data(), 32 * ppos.size()));
    GABI_HIP(ctx, up(T.perm_d, T.perm.data(), 4 * (size_t)n));
    GABI_HIP(ctx, up(T.cheb, cheb.data(), 8 * cheb.size()));
    GABI_HIP(ctx, up(T.clusters, clusters.data(), 16 * clusters.size()));
    GABI_HIP(ctx, up(T.batches, batches.data(), 16 * batches.size()));
    GABI_HIP(ctx, up(T.list, list.data(), 16 * list.size()));
    GABI_HIP(ctx, up(T.items, items.data(), 16 * items.size()));
    GABI_HIP(ctx, up(T.spos32, spos32.data(), 16 * (size_t)n));
    GABI_HIP(ctx, up(T.snrm32, snrm32.data(), 16 * (size_t)n));
    GABI_HIP(ctx, up(T.ppos32, ppos32.data(), 16 * ppos32.size()));
    GABI_HIP(ctx, up(T.pieces, pieces.data(), 16 * pieces.size()));
    GABI_HIP(ctx, hipStreamSynchronize(ctx->stream));
    T.version = ctx->geom_version;
    ++T.generation;
    T.theta = o->theta;
    T.degree = o->degree;
    T.leaf = o->leaf_size;
    return GABI_OK;
}

TreeDev tree_dev(const TreeState &T) {
    TreeDev d{};
    d.spos = T.spos;
    d.snrm = T.snrm;
    d.sw = T.sw;
    d.ppos = T.ppos;
    d.pw = T.pw;
    d.perm = T.perm_d;
    d.cheb = T.cheb;
    d.clusters = T.clusters;
    d.batches = T.batches;
    d.list = T.list;
    d.items = T.items;
    d.ipart = T.ipart;
    d.pieces = T.pieces;
    d.wpart = T.wpart;
    d.spos32 = T.spos32;
    d.snrm32 = T.snrm32;
    d.ppos32 = T.ppos32;
    d.sw32 = T.sw32;
    d.pw32 = T.pw32;
    d.n = T.n;
    d.piece = T.piece;
    d.degree = T.degree;
    d.P = T.P;
    for (int k = 0; k <= kTreeMaxDeg; ++k) d.bary[k] = T.bary[k];
    return d;
}

// prep, modified weights and sums of one product in the given precision
void launch_tree_sums3(const TreeState &T, const TreeDev &d, hipStream_t s, bool f32,
                       const PairConstF64 &pc, const PairConstF32 &pc32, const double *u,
                       const KrylovStatus *st, int skip) {
    const dim3 gp((T.n + kBlock - 1) / kBlock), blk(kBlock);
    const dim3 gs(T.n_clusters, (T.P + kBlock - 1) / kBlock);
    if (f32) {
        hipLaunchKernelGGL(tree_prep_kernel<true>, gp, blk, 0, s, d, u, st, skip);
        if (T.n_clusters > 0) {
            hipLaunchKernelGGL(tree_weights_kernel, dim3(T.n_pieces), blk, 0, s, d, st, skip);
            hipLaunchKernelGGL(tree_wsum_kernel<true>, gs, blk, 0, s, d, st, skip);
        }
        hipLaunchKernelGGL(tree_eval_kernel<true>, dim3(T.n_items), blk, 0, s, d, pc, pc32, st,
                           skip);
    } else {
        hipLaunchKernelGGL(tree_prep_kernel<false>, gp, blk, 0, s, d, u, st, skip);
        if (T.n_clusters > 0) {
            hipLaunchKernelGGL(tree_weights_kernel, dim3(T.n_pieces), blk, 0, s, d, st, skip);
            hipLaunchKernelGGL(tree_wsum_kernel<false>, gs, blk, 0, s, d, st, skip);
        }
        hipLaunchKernelGGL(tree_eval_kernel<false>, dim3(T.n_items), blk, 0, s, d, pc, pc32, st,
                           skip);
    }
}

PairConstF32 pair_const_f32(double kappa, double eps) {
    return PairConstF32{(float)kappa, (float)(-kappa * 1.4426950408889634074), (float)eps,
                        (float)(1.0 / eps)};
}

int tree_product(gabi_ctx *ctx, const gabi_tree_opts *o, const double *u_dev, double *y_dev) {
    int rc = tree_ensure(ctx, o);
    if (rc) return rc;
    const TreeState &T = *ctx->tree;
    const TreeDev d = tree_dev(T);
    const double eps = ctx->eps2 / ctx->eps1;
    const PairConstF64 pc{ctx->kappa, eps, 1.0 / eps};
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (ctx->timing) {
        if (hipEventCreate(&e0) != hipSuccess) e0 = nullptr;
        else if (hipEventCreate(&e1) != hipSuccess) {
            (void)hipEventDestroy(e0);
            e0 = e1 = nullptr;
        }
        if (e0) (void)hipEventRecord(e0, ctx->stream);
    }
    launch_tree_sums3(T, d, ctx->stream, o->precision == GABI_FP32_PAIR, pc,
                      pair_const_f32(ctx->kappa, eps), u_dev, nullptr, 0);
    hipLaunchKernelGGL(tree_finish_kernel<kTreeY>, dim3(T.n_batches), dim3(kBlock), 0,
                       ctx->stream, d, 0.5 * (1.0 + eps), 0.5 * (1.0 + 1.0 / eps), u_dev, y_dev,
                       nullptr, 0);
    if (e0 && e1) {
        (void)hipEventRecord(e1, ctx->stream);
        ctx->pending[2].push_back({e0, e1});
    }
    GABI_HIP(ctx, hipGetLastError());
    return GABI_OK;
}

}  // namespace

int tree_for_solve(gabi_ctx *ctx, const gabi_tree_opts *o) { return tree_ensure(ctx, o); }

void launch_tree_sums(const TreeState &T, hipStream_t s, const Mol &M, const double *u,
                      double *slot, bool skip, bool f32) {
    const TreeDev d = tree_dev(T);
    const PairConstF64 pc{M.kappa, M.eps, M.inv_eps};
    const PairConstF32 pc32{M.kappa_f, M.nkl2e_f, M.eps_f, M.inv_eps_f};
    const int sk = skip ? 1 : 0;
    launch_tree_sums3(T, d, s, f32, pc, pc32, u, M.st, sk);
    hipLaunchKernelGGL(tree_finish_kernel<kTreeSlot>, dim3(T.n_batches), dim3(kBlock), 0, s, d,
                       0.0, 0.0, u, slot, M.st, sk);
}

int64_t tree_generation(const TreeState &T) { return T.generation; }

}  // namespace gabi

using namespace gabi;

extern "C" {

int gabi_tree_matvec_dev(gabi_ctx *ctx, const gabi_tree_opts *opts, const double *u_dev,
                         double *y_dev) {
    if (!ctx) return GABI_EINVAL;
    if (ctx->n == 0) return fail(ctx, GABI_ESTATE, "surface not set");
    if (!ctx->params_set) return fail(ctx, GABI_ESTATE, "parameters not set");
    if (!u_dev || !y_dev) return fail(ctx, GABI_EINVAL, "null vector");
    GABI_HIP(ctx, hipSetDevice(ctx->device));
    return tree_product(ctx, opts, u_dev, y_dev);
}

int gabi_tree_matvec(gabi_ctx *ctx, const gabi_tree_opts *opts, const double *u, double *y) {
    if (!ctx) return GABI_EINVAL;
    if (ctx->n == 0) return fail(ctx, GABI_ESTATE, "surface not set");
    if (!ctx->params_set) return fail(ctx, GABI_ESTATE, "parameters not set");
    if (!u || !y) return fail(ctx, GABI_EINVAL, "null vector");
    GABI_HIP(ctx, hipSetDevice(ctx->device));
    // the product's device vectors: the context's staging pair, allocated
    // with the slot on first use
    int rc = tree_io_buffers(ctx);
    if (rc) return rc;
    const size_t bytes = sizeof(double) * 2 * (size_t)ctx->n;
    GABI_HIP(ctx, hipMemcpyAsync(ctx->tree_u, u, bytes, hipMemcpyHostToDevice, ctx->stream));
    if ((rc = tree_product(ctx, opts, ctx->tree_u, ctx->tree_y))) return rc;
    GABI_HIP(ctx, hipMemcpyAsync(y, ctx->tree_y, bytes, hipMemcpyDeviceToHost, ctx->stream));
    GABI_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return GABI_OK;
}

int gabi_tree_info_get(gabi_ctx *ctx, const gabi_tree_opts *opts, gabi_tree_info *out) {
    if (!ctx || !out) return GABI_EINVAL;
    if (ctx->n == 0) return fail(ctx, GABI_ESTATE, "surface not set");
    GABI_HIP(ctx, hipSetDevice(ctx->device));
    int rc = tree_ensure(ctx, opts);
    if (rc) return rc;
    *out = ctx->tree->info;
    out->device_bytes = ctx->tree->bytes;
    return GABI_OK;
}

int gabi_tree_plan(int64_t n, const double *cx, const double *cy, const double *cz,
                   const gabi_tree_opts *opts, gabi_tree_info *out) {
    if (n < 1 || !cx || !cy || !cz || !out) return GABI_EINVAL;
    std::string msg;
    if (validate_tree_opts(opts, msg)) return GABI_EINVAL;
    std::vector<double4> pos((size_t)n);
    for (int64_t i = 0; i < n; ++i) pos[(size_t)i] = make_double4(cx[i], cy[i], cz[i], 0.0);
    TreeState T;
    std::vector<int> batch_nodes;
    std::vector<std::vector<std::pair<int, int>>> lists;
    plan(T, pos.data(), n, opts->theta, opts->degree, opts->leaf_size, batch_nodes, lists);
    *out = T.info;
    out->device_bytes = 0;
    return GABI_OK;
}

}  // extern "C"
