// Per-molecule device memory (slots), product decomposition and the tuning
// table it is read from, and batches (block lists over many molecules).
#include <algorithm>
#include <map>
#include <atomic>
#include <cmath>
#include <cstring>
#include <mutex>

#include "gabi_internal.h"

namespace gabi {

// ------------------------------------------------------- partial-sum budget
namespace {
std::atomic<int64_t> g_part_budget{int64_t(512) << 20};
}

int64_t part_budget() { return g_part_budget.load(); }
void set_part_budget(int64_t bytes) { g_part_budget.store(bytes); }

// ---------------------------------------------------------------- tuning
namespace {
constexpr int kBuckets = 40;
TuneEntry g_table[2][kBuckets];
bool g_table_init = false;
std::mutex g_table_mu;

int bucket_of(int64_t n) {
    int b = 0;
    while (b + 1 < kBuckets && (int64_t(1) << (b + 1)) <= n) ++b;
    return b;
}

void init_table_locked() {
    if (g_table_init) return;
    for (int p = 0; p < 2; ++p)
        for (int b = 0; b < kBuckets; ++b) {
            TuneEntry e;
            e.scheme = GABI_SCHEME_SPLIT;
            e.rows_per_thread = b >= 13 ? 2 : 1;  // N >= 8192: two rows per thread
            e.target_blocks = 2048;
            g_table[p][b] = e;
        }
    g_table_init = true;
}
}  // namespace

TuneEntry tune_entry(int precision, int64_t n) {
    std::lock_guard<std::mutex> lk(g_table_mu);
    init_table_locked();
    return g_table[precision == GABI_FP64 ? 0 : 1][bucket_of(n)];
}

int set_tune_entry(int precision, int bucket, TuneEntry e) {
    if (bucket < 0 || bucket >= kBuckets) return GABI_EINVAL;
    if (e.scheme != GABI_SCHEME_SPLIT && e.scheme != GABI_SCHEME_SYMMETRIC) return GABI_EINVAL;
    if (e.rows_per_thread != 1 && e.rows_per_thread != 2) return GABI_EINVAL;
    if (e.scheme == GABI_SCHEME_SYMMETRIC && e.rows_per_thread != 1) return GABI_EINVAL;
    if (e.target_blocks < 1 || e.target_blocks > (1 << 20)) return GABI_EINVAL;
    if (e.tail_pieces < 0 || e.tail_pieces > 4096) return GABI_EINVAL;
    std::lock_guard<std::mutex> lk(g_table_mu);
    init_table_locked();
    g_table[precision == GABI_FP64 ? 0 : 1][bucket] = e;
    return GABI_OK;
}

void reset_tuning() {
    std::lock_guard<std::mutex> lk(g_table_mu);
    g_table_init = false;
    init_table_locked();
}

PairLaunch pair_launch(int64_t n, int precision) {
    return pair_launch_budget(n, precision, part_budget());
}

PairLaunch pair_launch_budget(int64_t n, int precision, int64_t budget) {
    const TuneEntry e = tune_entry(precision, n);
    PairLaunch L;
    L.scheme = e.scheme;
    if (e.scheme == GABI_SCHEME_SYMMETRIC) {
        L.rows_per_thread = 1;
        L.row_blocks = (int)((n + kTile - 1) / kTile);
        L.tiles_per_split = 1;
        L.head = 0;
        const int64_t slot_bytes = 2 * n * (precision == GABI_FP64 ? 8 : 4);
        sym_passes(L.row_blocks, budget / std::max<int64_t>(1, slot_bytes), L.passes, L.splits);
        L.last = L.row_blocks - (L.passes - 1) * L.splits;
        L.tail_start = (int)n;
        return L;
    }
    L.rows_per_thread = e.rows_per_thread;
    const int64_t rows_per_block = (int64_t)kBlock * L.rows_per_thread;
    L.row_blocks = (int)((n + rows_per_block - 1) / rows_per_block);
    // the tail: the last tail_pieces pieces of kPiece sources (aligned to kPiece)
    const int64_t pieces = (n + kPiece - 1) / kPiece;
    const int64_t tail_start =
        std::min<int64_t>(n, std::max<int64_t>(0, pieces - e.tail_pieces) * kPiece);
    L.tail_start = (int)tail_start;
    const int64_t tiles = (tail_start + kTile - 1) / kTile;
    int64_t want = (e.target_blocks + L.row_blocks - 1) / L.row_blocks;
    if (want < 1) want = 1;
    int64_t tps = (tiles + want - 1) / want;
    if (tps < 1) tps = 1;
    L.tiles_per_split = (int)tps;
    L.head = (int)((tiles + tps - 1) / tps);
    L.splits = L.head + (int)((n - tail_start + kPiece - 1) / kPiece);
    L.passes = 1;
    L.last = L.splits;
    return L;
}

}  // namespace gabi

extern "C" int gabi_tune_set(int precision, int bucket, int scheme, int rows_per_thread,
                             int target_blocks, int tail_pieces) {
    if (precision != GABI_FP64 && precision != GABI_FP32_PAIR) return GABI_EINVAL;
    gabi::TuneEntry e;
    e.scheme = scheme;
    e.rows_per_thread = rows_per_thread;
    e.target_blocks = target_blocks;
    e.tail_pieces = tail_pieces;
    return gabi::set_tune_entry(precision, bucket, e);
}

extern "C" int gabi_set_part_budget(int64_t bytes) {
    if (bytes < 1) return GABI_EINVAL;
    gabi::set_part_budget(bytes);
    return GABI_OK;
}

extern "C" int64_t gabi_get_part_budget(void) { return gabi::part_budget(); }

extern "C" int gabi_tune_get(int precision, int bucket, int *scheme, int *rows_per_thread,
                             int *target_blocks, int *tail_pieces) {
    if ((precision != GABI_FP64 && precision != GABI_FP32_PAIR) || bucket < 0 || bucket >= 40)
        return GABI_EINVAL;
    const gabi::TuneEntry e = gabi::tune_entry(precision, int64_t(1) << bucket);
    if (scheme) *scheme = e.scheme;
    if (rows_per_thread) *rows_per_thread = e.rows_per_thread;
    if (target_blocks) *target_blocks = e.target_blocks;
    if (tail_pieces) *tail_pieces = e.tail_pieces;
    return GABI_OK;
}

namespace gabi {

int blas_blocks(int64_t n) {
    int64_t b = (n + kBlock - 1) / kBlock;
    return (int)std::max<int64_t>(1, std::min<int64_t>(b, kBlasBlocksMax));
}

// ---------------------------------------------------------------- slots
namespace {
struct Carver {
    char *base;
    int64_t off = 0;
    template <typename T>
    T *take(int64_t count) {
        off = (off + 255) & ~int64_t(255);
        T *p = base ? reinterpret_cast<T *>(base + off) : nullptr;
        off += std::max<int64_t>(1, count) * (int64_t)sizeof(T);
        return p;
    }
};

void reaction_split(int64_t n, int64_t nc, int &kblocks, int &tps, int &splits) {
    kblocks = (int)std::max<int64_t>(1, (nc + 63) / 64);  // 64 charges per reaction tile
    const int64_t tiles = (n + kTile - 1) / kTile;
    int64_t want = (1024 + kblocks - 1) / kblocks;
    if (want < 1) want = 1;
    int64_t t = (tiles + want - 1) / want;
    if (t < 1) t = 1;
    tps = (int)t;
    splits = (int)((tiles + t - 1) / t);
}

}  // namespace

void mol_decomposition(Mol &t, int64_t n, const PairLaunch &L64, const PairLaunch &L32) {
    t.R64 = L64.rows_per_thread;
    t.rb64 = L64.row_blocks;
    t.tps64 = L64.tiles_per_split;
    t.sp64 = L64.splits;
    t.R32 = L32.rows_per_thread;
    t.rb32 = L32.row_blocks;
    t.tps32 = L32.tiles_per_split;
    t.sp32 = L32.splits;
    t.head64 = L64.head;
    t.tail64 = L64.tail_start;
    t.head32 = L32.head;
    t.tail32 = L32.tail_start;
    t.sym64 = L64.scheme == GABI_SCHEME_SYMMETRIC;
    t.sym32 = L32.scheme == GABI_SCHEME_SYMMETRIC;
    t.np64 = L64.passes;
    t.np32 = L32.passes;
    t.last64 = L64.last;
    t.last32 = L32.last;
    t.nbk = (int32_t)((n + kTile - 1) / kTile);
}

namespace {

// Lays the buffers of one molecule out in one block starting at base (null:
// sizing only); returns the size in bytes.
int64_t layout(int64_t n, int64_t nc, int m, char *base, Mol *M) {
    const PairLaunch L64 = pair_launch(n, GABI_FP64), L32 = pair_launch(n, GABI_FP32_PAIR);
    int kb, tps, sp;
    reaction_split(n, nc, kb, tps, sp);
    Carver c{base};
    const int64_t len = 2 * n;
    Mol t{};
    t.pos = c.take<double4>(n);
    t.nrm = c.take<double4>(n);
    t.pos32 = c.take<float4>(2 * n);
    t.nrm32 = t.pos32 ? t.pos32 + n : nullptr;
    t.chg = c.take<double4>(nc);
    t.wgt = c.take<double4>(n);
    t.wgt32 = c.take<float4>(n);
    // partial sums: FP64 per (row, split); the symmetric FP32-pair product keeps
    // its per-block sums as float
    const int64_t part64 = len * L64.splits * 8;
    const int64_t part32 = len * L32.splits * (L32.scheme == GABI_SCHEME_SYMMETRIC ? 4 : 8);
    t.part = c.take<double>((std::max(part64, part32) + 7) / 8);
    // sums of the earlier passes of a product taken in several passes
    t.acc = (L64.passes > 1 || L32.passes > 1) ? c.take<double>(len) : nullptr;
    t.u = c.take<double>(len);
    t.y = c.take<double>(len);
    t.b = c.take<double>(len);
    t.x = c.take<double>(len);
    t.r = c.take<double>(len);
    t.w = c.take<double>(len);
    t.bo = c.take<double>(len);
    t.xo = c.take<double>(len);
    t.sol = c.take<double>(len);
    t.V = c.take<double>(len * (m + 1));
    t.H = c.take<double>((int64_t)(m + 1) * m);
    t.cs = c.take<double>(m);
    t.sn = c.take<double>(m);
    t.g = c.take<double>(m + 1);
    t.hn = c.take<double>(m);
    t.red = c.take<double>((int64_t)(2 * m + 1) * kBlasBlocksMax);
    t.G = c.take<double>(std::max<int64_t>(1, (int64_t)m * (m - 1) / 2));
    t.st = c.take<KrylovStatus>(1);
    t.phi = c.take<double>(nc);
    t.phi_part = c.take<double>(nc * sp);
    if (M) {
        t.n = (int32_t)n;
        t.nc = (int32_t)nc;
        t.nb = blas_blocks(n);
        t.m = m;
        mol_decomposition(t, n, L64, L32);
        t.rx_kblocks = kb;
        t.rx_tps = tps;
        t.rx_splits = sp;
        t.maxit = 100;
        t.tol0 = 1e-6;
        t.inner_tol = 1e-5;
        t.mode = M->mode;
        // keep parameters already set
        t.kappa = M->kappa; t.eps = M->eps; t.inv_eps = M->inv_eps;
        t.d_top = M->d_top; t.d_bot = M->d_bot; t.rhs_scale = M->rhs_scale;
        t.kappa_f = M->kappa_f; t.nkl2e_f = M->nkl2e_f; t.eps_f = M->eps_f;
        t.inv_eps_f = M->inv_eps_f;
        *M = t;
    }
    return c.off;
}
}  // namespace

int64_t slot_bytes(int64_t n, int64_t nc, int m) { return layout(n, nc, m, nullptr, nullptr); }

void slot_carve(Slot &s, int64_t n, int64_t nc, int m) {
    layout(n, nc, m, static_cast<char *>(s.mem), &s.mol);
    slot_set_mode(s, s.mol.mode);
}

void slot_set_params(Slot &s, double eps1, double eps2, double kappa) {
    mol_set_params(s.mol, eps1, eps2, kappa);
}

void mol_set_params(Mol &M, double eps1, double eps2, double kappa) {
    const double eps = eps2 / eps1;
    M.kappa = kappa;
    M.eps = eps;
    M.inv_eps = 1.0 / eps;
    M.d_top = 0.5 * (1.0 + eps);
    M.d_bot = 0.5 * (1.0 + 1.0 / eps);
    M.rhs_scale = 1.0 / (4.0 * kPi * eps1);
    M.kappa_f = (float)kappa;
    M.nkl2e_f = (float)(-kappa * 1.4426950408889634074);
    M.eps_f = (float)eps;
    M.inv_eps_f = (float)(1.0 / eps);
}

// Role of each vector in the two solvers:
//   FP64 GMRES:  b = rhs, x = iterate, r = residual (cycle start)
//   mixed IR:    bo = rhs, xo = iterate, b = FP64 residual bo - A xo, which
//                is also the right-hand side of the FP32-pair cycle whose
//                correction V y is added to xo directly.
void slot_set_mode(Slot &s, int mode) {
    Mol &M = s.mol;
    M.mode = mode;
    if (mode == kModeMixed) {
        M.rhs_dst = M.bo;
        M.cyc_src = M.b;
        M.upd_dst = M.xo;
        M.res_x = M.xo;
        M.res_b = M.bo;
        M.res_out = M.b;
    } else {
        M.rhs_dst = M.b;
        M.cyc_src = M.r;
        M.upd_dst = M.x;
        M.res_x = M.x;
        M.res_b = M.b;
        M.res_out = M.r;
    }
}

void set_solve_targets(Slot &slot, double tol, double inner_tol, int maxit) {
    slot.mol.tol0 = tol;
    slot.mol.inner_tol = inner_tol;
    slot.mol.maxit = maxit;
}

int64_t next_slot_uid() {
    static std::atomic<int64_t> uid{0};
    return ++uid;
}

// ---------------------------------------------------------------- batches
void release_graph(Batch &b) {
    if (b.graph) (void)hipGraphExecDestroy(b.graph);
    b.graph = nullptr;
    b.graph_valid = false;
    b.graph_timed = false;
    for (auto &v : b.graph_events) {
        for (auto &ev : v) {
            (void)hipEventDestroy(ev.first);
            (void)hipEventDestroy(ev.second);
        }
        v.clear();
    }
}

void batch_free(Batch &b) {
    release_graph(b);
    if (b.d_mem) (void)hipFree(b.d_mem);
    if (b.h_pinned) (void)hipHostFree(b.h_pinned);
    b.d_mem = nullptr;
    b.h_pinned = nullptr;
    b.h_status = nullptr;
    b.cap_bytes = 0;
    b.d_mols = nullptr;
    b.n_elem = b.n_blas = b.n_rx = 0;
    for (int g = 0; g < 3; ++g) b.n_tiles64[g] = b.n_tiles32[g] = 0;
    b.n_pass64 = b.n_pass32 = 1;
    std::memset(b.sym_off64, 0, sizeof(b.sym_off64));
    std::memset(b.sym_off32, 0, sizeof(b.sym_off32));
}

void pair_grids(int g64[3], int g32[3]) {
    static int grid[2][3] = {{0, 0, 0}, {0, 0, 0}};
    static std::once_flag once;
    std::call_once(once, [] {
        for (int v = 0; v < 3; ++v) {
            grid[0][v] = pair_occupancy_grid(GABI_FP64, v);
            grid[1][v] = pair_occupancy_grid(GABI_FP32_PAIR, v);
        }
    });
    for (int v = 0; v < 3; ++v) {
        g64[v] = grid[0][v];
        g32[v] = grid[1][v];
    }
}

namespace {

// The symmetric kernel's lists (see sym_pair_kernel): the tiles of each pass
// (entries [pass_off[p], pass_off[p+1]) of `sym`) are ordered by molecule,
// then by squares of kSquare x kSquare block pairs (I / kSquare, J / kSquare),
// then (I, J), and cut into kXcdLists lists of about equal cost (an
// off-diagonal tile costs two diagonal ones), each list's diagonal tiles
// moved to its end so that its last tiles are short ones.  The tiles an
// XCD runs at one time then come from a few squares, which touch few blocks
// (2 kSquare per square), so their element records stay in that XCD's L2.
// xoff receives kXcdLists + 1 offsets per pass, relative to the pass's
// first tile.
constexpr int kSquare = 16;

void xcd_lists(int4 *sym, const std::vector<int> &pass_off, std::vector<int> &xoff) {
    const int np = std::max<int>(1, (int)pass_off.size() - 1);
    xoff.assign((size_t)np * (kXcdLists + 1), 0);
    for (int p = 0; p + 1 < (int)pass_off.size(); ++p) {
        int4 *a = sym + pass_off[p];
        const int n = pass_off[p + 1] - pass_off[p];
        std::stable_sort(a, a + n, [](const int4 &u, const int4 &v) {
            if (u.x != v.x) return u.x < v.x;
            if (u.y / kSquare != v.y / kSquare) return u.y / kSquare < v.y / kSquare;
            if (u.z / kSquare != v.z / kSquare) return u.z / kSquare < v.z / kSquare;
            if (u.y != v.y) return u.y < v.y;
            return u.z < v.z;
        });
        int64_t total = 0;
        for (int t = 0; t < n; ++t) total += a[t].y == a[t].z ? 1 : 2;
        int *xo = xoff.data() + (size_t)p * (kXcdLists + 1);
        int64_t acc = 0;
        int x = 1;
        for (int t = 0; t < n && x < kXcdLists; ++t) {
            acc += a[t].y == a[t].z ? 1 : 2;
            while (x < kXcdLists && acc * kXcdLists >= total * x) xo[x++] = t + 1;
        }
        for (; x <= kXcdLists; ++x) xo[x] = n;
        for (int l = 0; l < kXcdLists; ++l)
            std::stable_partition(a + xo[l], a + xo[l + 1],
                                  [](const int4 &u) { return u.y != u.z; });
    }
}

}  // namespace

int batch_build(Batch &b, hipStream_t stream, std::string &err) {
    const int nm = (int)b.slots.size();
    std::vector<Mol> mols((size_t)nm);
    std::vector<int2> elem, blas;
    std::vector<int4> t64, t32, rx;
    for (int k = 0; k < nm; ++k) {
        const Mol &M = b.slots[k]->mol;
        mols[k] = M;
        const int eb = (M.n + kBlock - 1) / kBlock;
        for (int i = 0; i < eb; ++i) elem.push_back(make_int2(k, i));
        for (int i = 0; i < M.nb; ++i) blas.push_back(make_int2(k, i));
        // split scheme: (mol, row block, split, cost = rows per thread x
        // sources); symmetric scheme: (mol, block I, block J, slot | pass << 16)
        // for the tiles of every round in round order (sym_schedule.h), round
        // r in pass r / sp writing slot r mod sp
        auto tiles = [&](std::vector<int4> &t, int sym, int R, int rb, int sp, int tps, int head,
                         int tail) {
            if (sym) {
                std::vector<std::pair<int, int>> rt;
                for (int r = 0; r < M.nbk; ++r) {
                    sym_round(M.nbk, r, rt);
                    const int w = (r % sp) | ((r / sp) << 16);
                    for (const auto &pr : rt) t.push_back(make_int4(k, pr.first, pr.second, w));
                }
                return;
            }
            for (int s = 0; s < sp; ++s) {
                int j0, j1;
                split_range(M.n, tps, head, tail, s, j0, j1);
                for (int r = 0; r < rb; ++r) t.push_back(make_int4(k, r, s, R * (j1 - j0)));
            }
        };
        tiles(t64, M.sym64, M.R64, M.rb64, M.sp64, M.tps64, M.head64, M.tail64);
        tiles(t32, M.sym32, M.R32, M.rb32, M.sp32, M.tps32, M.head32, M.tail32);
        if (M.nc > 0)
            for (int sp = 0; sp < M.rx_splits; ++sp)
                for (int kb = 0; kb < M.rx_kblocks; ++kb) rx.push_back(make_int4(k, kb, sp, 0));
    }
    // group by kernel variant (split with two rows per thread, split with one,
    // symmetric), the symmetric tiles by pass, longest tiles first within a
    // group or pass; ties keep molecule and tile order
    // (a stable counting sort over the few distinct (group, pass, cost) keys:
    // a comparison sort of a large batch's tiles took milliseconds per rebuild)
    auto group = [&](std::vector<int4> &t, bool mixed, int *counts, std::vector<int> &sym_off) {
        std::vector<int> gm((size_t)nm);
        for (int k = 0; k < nm; ++k) {
            const Mol &M = b.slots[k]->mol;
            gm[k] = (mixed ? M.sym32 : M.sym64) ? 2 : (mixed ? M.R32 : M.R64) == 2 ? 0 : 1;
        }
        // ascending key = group ascending, then pass ascending, then cost
        // descending (a symmetric tile costs two diagonal ones)
        auto key = [&](const int4 &a) {
            const int g = gm[a.x];
            const int64_t pass = g == 2 ? (a.w >> 16) : 0;
            const int64_t cost = g == 2 ? (a.y == a.z ? kTile : 2 * kTile) : a.w;
            return ((int64_t)g << 56) | (pass << 32) | (int64_t)(0x7fffffff - cost);
        };
        // consecutive tiles mostly share a key, so the map is consulted only
        // when the key changes
        std::map<int64_t, size_t> start;
        {
            int64_t last = -1;
            size_t *cnt = nullptr;
            for (const int4 &a : t) {
                const int64_t kk = key(a);
                if (kk != last) {
                    cnt = &start[kk];
                    last = kk;
                }
                ++*cnt;
            }
        }
        size_t off = 0;
        for (auto &kv : start) {
            const size_t c = kv.second;
            kv.second = off;
            off += c;
        }
        std::vector<int4> out(t.size());
        {
            int64_t last = -1;
            size_t *pos = nullptr;
            for (const int4 &a : t) {
                const int64_t kk = key(a);
                if (kk != last) {
                    pos = &start[kk];
                    last = kk;
                }
                out[(*pos)++] = a;
            }
        }
        t.swap(out);
        counts[0] = counts[1] = counts[2] = 0;
        std::vector<int> per_pass;  // symmetric tiles of each pass
        for (const int4 &a : t) {
            const int g = gm[a.x];
            counts[g]++;
            if (g == 2) {
                const size_t pass = (size_t)(a.w >> 16);
                if (per_pass.size() <= pass) per_pass.resize(pass + 1, 0);
                per_pass[pass]++;
            }
        }
        sym_off.assign(1, 0);
        for (int c : per_pass) sym_off.push_back(sym_off.back() + c);
    };
    int c64[3], c32[3];
    std::vector<int> off64, off32;
    group(t64, false, c64, off64);
    group(t32, true, c32, off32);
    std::vector<int> xoff64, xoff32;
    xcd_lists(t64.data() + c64[0] + c64[1], off64, xoff64);
    xcd_lists(t32.data() + c32[0] + c32[1], off32, xoff32);

    auto al = [](int64_t v) { return (v + 255) & ~int64_t(255); };
    const int64_t o_mols = 0;
    const int64_t o_elem = al(o_mols + (int64_t)sizeof(Mol) * std::max(1, nm));
    const int64_t o_blas = al(o_elem + (int64_t)sizeof(int2) * std::max<size_t>(1, elem.size()));
    const int64_t o_t64 = al(o_blas + (int64_t)sizeof(int2) * std::max<size_t>(1, blas.size()));
    const int64_t o_t32 = al(o_t64 + (int64_t)sizeof(int4) * std::max<size_t>(1, t64.size()));
    const int64_t o_x64 = al(o_t32 + (int64_t)sizeof(int4) * std::max<size_t>(1, t32.size()));
    const int64_t o_x32 = al(o_x64 + (int64_t)sizeof(int) * xoff64.size());
    const int64_t o_rx = al(o_x32 + (int64_t)sizeof(int) * xoff32.size());
    const int64_t o_cnt = al(o_rx + (int64_t)sizeof(int4) * std::max<size_t>(1, rx.size()));
    const int64_t o_st = al(o_cnt + 256);
    const int64_t total = al(o_st + (int64_t)sizeof(KrylovStatus) * std::max(1, nm));

    release_graph(b);
    if (total > b.cap_bytes || !b.d_mem) {
        if (b.d_mem) (void)hipFree(b.d_mem);
        if (b.h_pinned) (void)hipHostFree(b.h_pinned);
        b.d_mem = nullptr;
        b.h_pinned = nullptr;
        b.h_status = nullptr;
        const int64_t cap = std::max<int64_t>(total * 2, 1 << 16);
        hipError_t e = hipMalloc(&b.d_mem, cap);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            b.d_mem = nullptr;
            err = std::string("batch allocation failed: ") + hipGetErrorString(e);
            return GABI_ENOMEM;
        }
        e = hipHostMalloc(&b.h_pinned, cap, hipHostMallocDefault);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            (void)hipFree(b.d_mem);
            b.d_mem = nullptr;
            b.h_pinned = nullptr;
            err = std::string("pinned status allocation failed: ") + hipGetErrorString(e);
            return GABI_ENOMEM;
        }
        b.cap_bytes = cap;
    }
    char *base = static_cast<char *>(b.d_mem);
    b.d_mols = reinterpret_cast<Mol *>(base + o_mols);
    b.d_elem = reinterpret_cast<int2 *>(base + o_elem);
    b.d_blas = reinterpret_cast<int2 *>(base + o_blas);
    b.d_tiles64 = reinterpret_cast<int4 *>(base + o_t64);
    b.d_tiles32 = reinterpret_cast<int4 *>(base + o_t32);
    b.d_xoff64 = reinterpret_cast<int *>(base + o_x64);
    b.d_xoff32 = reinterpret_cast<int *>(base + o_x32);
    b.d_rx = reinterpret_cast<int4 *>(base + o_rx);
    b.d_counter = reinterpret_cast<int *>(base + o_cnt);
    b.d_status = reinterpret_cast<KrylovStatus *>(base + o_st);
    b.n_elem = (int)elem.size();
    b.n_blas = (int)blas.size();
    for (int g = 0; g < 3; ++g) {
        b.n_tiles64[g] = c64[g];
        b.n_tiles32[g] = c32[g];
    }
    auto set_off = [](const std::vector<int> &off, int *dst, int &np) {
        np = std::max<int>(1, (int)off.size() - 1);
        for (int p = 0; p <= kMaxPasses; ++p)
            dst[p] = p < (int)off.size() ? off[p] : (off.empty() ? 0 : off.back());
    };
    set_off(off64, b.sym_off64, b.n_pass64);
    set_off(off32, b.sym_off32, b.n_pass32);
    b.n_rx = (int)rx.size();
    // stage everything in the pinned buffer, one upload
    char *h = reinterpret_cast<char *>(b.h_pinned);
    std::memset(h, 0, (size_t)total);
    if (nm) std::memcpy(h + o_mols, mols.data(), sizeof(Mol) * nm);
    if (!elem.empty()) std::memcpy(h + o_elem, elem.data(), sizeof(int2) * elem.size());
    if (!blas.empty()) std::memcpy(h + o_blas, blas.data(), sizeof(int2) * blas.size());
    if (!t64.empty()) std::memcpy(h + o_t64, t64.data(), sizeof(int4) * t64.size());
    if (!t32.empty()) std::memcpy(h + o_t32, t32.data(), sizeof(int4) * t32.size());
    std::memcpy(h + o_x64, xoff64.data(), sizeof(int) * xoff64.size());
    std::memcpy(h + o_x32, xoff32.data(), sizeof(int) * xoff32.size());
    if (!rx.empty()) std::memcpy(h + o_rx, rx.data(), sizeof(int4) * rx.size());
    hipError_t e = hipMemcpyAsync(b.d_mem, h, (size_t)total, hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) {
        err = std::string("batch upload failed: ") + hipGetErrorString(e);
        return GABI_EDEVICE;
    }
    b.h_status = reinterpret_cast<KrylovStatus *>(h + o_st);
    pair_grids(b.grid64, b.grid32);
    return GABI_OK;
}

}  // namespace gabi
