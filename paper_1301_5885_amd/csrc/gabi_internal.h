// Internal declarations of libgabi.
//
// Every kernel works on a *batch* of molecules described by an array of
// `Mol` records in device memory; a workgroup finds its molecule (and its
// block within that molecule) in a per-launch block list built on the host.
// A single solve is a batch of one, so a molecule is decomposed, reduced and
// iterated identically whether it runs alone or among others.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/gabi.h"
#include "sym_schedule.h"

namespace gabi {

constexpr int kBlock = 256;          // threads per workgroup (4 wave64)
constexpr int kTile = 256;           // sources staged in LDS per tile
constexpr int kPiece = 64;           // sources of one tail split
constexpr int kBlasBlocksMax = 256;  // workgroups per molecule in reductions
constexpr int kMaxRestart = 64;
// Tile queues of the product: per precision a block of kCountersPerPrecision
// ints, [0, 3) one per pair-kernel variant, [kXcdCounters, +kXcdLists) the
// symmetric kernel's per-list queues (one list per XCD).
constexpr int kXcdLists = 8;
constexpr int kXcdCounters = 8;
constexpr int kCountersPerPrecision = 16;
constexpr double kPi = 3.14159265358979323846;
constexpr double kCoulomb = 332.0716;  // kcal A / (mol e^2)

// ---------------------------------------------------------------------------
// Decomposition of one product: row blocks x source splits.  A function of
// N and the precision (and the loaded tuning table) only.
// Split scheme: sources [0, tail_start) form `head` splits of tiles_per_split
// tiles of 256; [tail_start, N) forms splits of kPiece sources; one pass.
// Symmetric scheme: row_blocks = nbk blocks of 256, whose block pairs are
// taken in nbk rounds (sym_schedule.h) grouped into `passes` passes of
// `splits` rounds; a round writes one partial-sum slot per row, so a pass
// needs `splits` slots (the last pass `last`), and passes after the first
// fold their slots into an FP64 accumulator.  splits is bounded by the
// partial-sum budget, so the buffer is O(N) for a given budget.
struct PairLaunch {
    int scheme = GABI_SCHEME_SPLIT;
    int rows_per_thread = 1;
    int row_blocks = 0;
    int tiles_per_split = 0;
    int splits = 0;      // partial-sum slots per row (per pass)
    int head = 0;
    int tail_start = 0;
    int passes = 1;
    int last = 0;        // slots of the last pass
};

// Bytes one precision's partial sums of one molecule may take (the
// symmetric scheme's slots per pass follow from it); library-wide.
int64_t part_budget();
void set_part_budget(int64_t bytes);

struct TuneEntry {  // one row of the tuning table
    int scheme = GABI_SCHEME_SPLIT;
    int rows_per_thread = 2;
    int target_blocks = 2048;
    int tail_pieces = 0;
};

// Source range [begin, end) of split sp.
__host__ __device__ inline void split_range(int n, int tps, int head, int tail_start, int sp,
                                            int &begin, int &end) {
    if (sp < head) {
        begin = sp * tps * kTile;
        end = begin + tps * kTile < tail_start ? begin + tps * kTile : tail_start;
    } else {
        begin = tail_start + (sp - head) * kPiece;
        end = begin + kPiece < n ? begin + kPiece : n;
    }
}

PairLaunch pair_launch(int64_t n, int precision);
PairLaunch pair_launch_budget(int64_t n, int precision, int64_t budget);
int blas_blocks(int64_t n);
// Tuning table (tune.hip): per precision and N bucket (bucket = floor(log2 N)).
TuneEntry tune_entry(int precision, int64_t n);
int set_tune_entry(int precision, int bucket, TuneEntry e);
void reset_tuning();

// ---------------------------------------------------------------------------
// Device status of one molecule's solve.
struct KrylovStatus {
    int32_t k;          // Arnoldi steps taken in the current cycle
    int32_t done;       // current cycle ended (estimate, breakdown, cap)
    int32_t iters;      // Arnoldi steps of the whole solve
    int32_t maxit;
    int32_t converged;  // explicit residual <= tol0 * beta0
    int32_t pad[3];
    double beta0;       // ||b|| of the Poisson-Boltzmann right-hand side
    double beta;        // norm the current cycle's estimate is relative to
    double tol;         // estimate threshold (relative to beta)
    double tol0;        // final tolerance (relative to beta0)
    double inner_tol;   // mixed refinement: relative target of one cycle
    double rnorm;       // last explicit residual norm
    double gabs;        // |g_k|, the Givens estimate
    double energy;      // solvation energy (kcal/mol) after launch_reaction
};

enum SolveMode { kModeFP64 = 0, kModeMixed = 1 };

// Device-visible description of one molecule (plain data).
struct Mol {
    int32_t n, nc, nb, m;
    int32_t mode;
    int32_t R64, rb64, tps64, sp64;   // FP64 product decomposition
    int32_t R32, rb32, tps32, sp32;   // FP32-pair product decomposition
    int32_t head64, tail64, head32, tail32;  // split source ranges (split_range)
    // symmetric scheme per precision (then R = 1, rb = nbk blocks of 256,
    // spXX = partial slots per pass, npXX passes, lastXX slots of the last
    // pass, and the FP32-pair partial sums are stored as float)
    int32_t sym64, sym32, nbk, pad_sym;
    int32_t np64, np32, last64, last32;
    int32_t rx_kblocks, rx_tps, rx_splits, maxit;
    double kappa, eps, inv_eps, d_top, d_bot, rhs_scale;
    double tol0, inner_tol;             // solve targets (copied into st)
    float kappa_f, nkl2e_f, eps_f, inv_eps_f;
    const double4 *pos;   // (cx, cy, cz, area)
    const double4 *nrm;   // (nx, ny, nz, 0)
    const float4 *pos32;  // FP32 (x, y, z, 0) relative to the bounding-box centre
    const float4 *nrm32;  // FP32 (nx, ny, nz, 0); follows pos32 in memory
    const double4 *chg;   // (x, y, z, q)
    double4 *wgt;         // (s, mx, my, mz)
    float4 *wgt32;
    double *part;         // partial sums [slots][2][n] (float: symmetric FP32 pair)
    double *acc;          // 2n FP64 sums of the passes before the last (or null)
    // vectors of length 2n
    double *u, *y;        // product input / output (matvec entry points)
    double *b, *x, *r, *w, *bo, *xo, *sol;
    // role pointers set by the solve mode (see krylov.hip)
    double *rhs_dst, *cyc_src, *upd_dst, *res_x, *res_b, *res_out;
    // Krylov.  red: partial-sum slots of kBlasBlocksMax doubles (slot 0
    // <w, v_0> or a residual norm, slots 1..2j a step's dot products, slot 2m
    // the projected ||w||^2); G: the cycle's Gram entries <v_k, v_i>, k < i,
    // packed by rows (row i at i(i-1)/2)
    double *V, *H, *cs, *sn, *g, *hn, *red, *G;
    KrylovStatus *st;
    // reaction potential at the charges
    double *phi, *phi_part;
};

// Host-side record of one molecule: its descriptor plus bookkeeping.
struct Slot {
    Mol mol{};
    // Unique per admission (never reused, unlike the Slot's address, which
    // the allocator hands out again once a finished slot is freed): batches
    // are compared by these ids to decide whether they must be rebuilt.
    int64_t uid = 0;
    void *mem = nullptr;      // one device block holding every buffer
    int64_t bytes = 0;
    bool from_arena = false;
    int64_t arena_off = 0;
    // solve bookkeeping
    int64_t tag = 0;
    int64_t ticket = 0;       // request sequence number (server) or index (batch)
    int32_t rounds = 0;
    int64_t products64 = 0, products32 = 0;
    int32_t last_iters = 0;
    double t_submit = 0, t_admit = 0, t_done = 0;
    double *u_out = nullptr;  // caller's host buffer for the solution
    int status = 0;
    KrylovStatus host_st{};   // last status read back
};

int64_t next_slot_uid();

// Size of the device block of a slot and the carving of its buffers.
int64_t slot_bytes(int64_t n, int64_t nc, int m);
void slot_carve(Slot &s, int64_t n, int64_t nc, int m);
void slot_set_params(Slot &s, double eps1, double eps2, double kappa);
void mol_set_params(Mol &M, double eps1, double eps2, double kappa);
// the product-decomposition fields of a descriptor
void mol_decomposition(Mol &t, int64_t n, const PairLaunch &L64, const PairLaunch &L32);
void slot_set_mode(Slot &s, int mode);

// ---------------------------------------------------------------------------
// A batch: the device array of Mol records and the per-launch block lists.
struct Batch {
    std::vector<Slot *> slots;
    Mol *d_mols = nullptr;
    int2 *d_elem = nullptr;   int n_elem = 0;   // (mol, block) over ceil(n/256)
    int2 *d_blas = nullptr;   int n_blas = 0;   // (mol, block) over nb
    // product tiles grouped by kernel variant: split scheme with two rows per
    // thread (mol, row block, split, cost), then one row per thread, then the
    // symmetric scheme (mol, block I, block J, cost): n_tilesXX[0..2] entries
    int4 *d_tiles64 = nullptr; int n_tiles64[3] = {0, 0, 0};
    int4 *d_tiles32 = nullptr; int n_tiles32[3] = {0, 0, 0};
    // symmetric tiles by pass: pass p is entries [sym_offXX[p], sym_offXX[p+1])
    // of the symmetric group (the molecules' passes p run in one launch)
    int n_pass64 = 1, n_pass32 = 1;
    int sym_off64[kMaxPasses + 1] = {0}, sym_off32[kMaxPasses + 1] = {0};
    // per pass, kXcdLists + 1 offsets (relative to the pass's first tile)
    // cutting its tiles into the symmetric kernel's lists
    int *d_xoff64 = nullptr, *d_xoff32 = nullptr;
    int4 *d_rx = nullptr;     int n_rx = 0;     // (mol, charge block, split, 0)
    int *d_counter = nullptr;  // tile queues (2 x kCountersPerPrecision)
    KrylovStatus *d_status = nullptr;  // gathered statuses, one per molecule
    KrylovStatus *h_status = nullptr;  // their pinned host mirror (in h_pinned)
    void *h_pinned = nullptr;          // staging for uploads, same layout as d_mem
    int mode = 0;                      // solve mode shared by the batch
    void *d_mem = nullptr;
    int64_t cap_bytes = 0;
    bool persistent = true;
    int grid64[3] = {0, 0, 0}, grid32[3] = {0, 0, 0};  // persistent grids per variant
    // captured round (hipGraph), valid while the batch is unchanged
    hipGraphExec_t graph = nullptr;
    bool graph_valid = false;
    // a round captured with timing holds event-record nodes around every
    // product launch; these are their events, whose timestamps each replay
    // overwrites
    std::vector<std::pair<hipEvent_t, hipEvent_t>> graph_events[2];
    bool graph_timed = false;
    // treecode refinement (a single context's batch): the inner products of
    // a cycle are the context's treecode products; tree_gen identifies the
    // tree the captured round was recorded with
    const struct TreeState *tree = nullptr;
    int64_t tree_gen = -1;
    bool tree_f32 = false;  // FP32 evaluation of the treecode sums
};

int batch_build(Batch &b, hipStream_t stream, std::string &err);
void pair_grids(int g64[3], int g32[3]);  // persistent grids of the pair kernels
void batch_free(Batch &b);
void release_graph(Batch &b);  // the captured round and its events

struct TreeState;                // treecode product (tree.hip)
void tree_free(TreeState *t);
// the context's tree for these options, built or rebuilt as needed
int tree_for_solve(gabi_ctx *ctx, const gabi_tree_opts *o);
// treecode sums of u (2n, element order) into slot (top at [j], bot at
// [n + j]); with skip, nothing once M's cycle has ended
void launch_tree_sums(const TreeState &T, hipStream_t s, const Mol &M, const double *u,
                      double *slot, bool skip, bool f32);
int64_t tree_generation(const TreeState &T);  // changes with every rebuild
// pseudo-precision of the Arnoldi finish for a product held as one FP64
// partial-sum slot (the treecode refinement's inner products)
constexpr int kPrecTree = 2;

}  // namespace gabi

// ---------------------------------------------------------------------------
struct gabi_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    hipStream_t capture = nullptr;  // records graphs only, never executes
    std::string err;

    gabi::Slot slot;
    gabi::Batch batch;
    bool batch_dirty = true;
    gabi::Mol uploaded{};  // descriptor the batch was last built from
    bool geom_dirty = true, chg_dirty = true;
    int64_t n = 0, nc = 0;
    int64_t slot_n = -1, slot_nc = -1;
    int m_alloc = 0;
    bool charges_set = false, params_set = false, have_solution = false;
    bool prev_solution = false;  // the slot's solution buffer holds a solve's result
    // energy and reaction potential (in the slot) of the last solution, as the
    // solve's final step computed them; valid while have_solution holds and
    // no energy of another u has been evaluated since
    bool solution_energy_valid = false;
    double solution_energy = 0.0;
    double eps1 = 1.0, eps2 = 80.0, kappa = 0.0;
    std::vector<double> host_centroids;  // 3n, for validation
    std::vector<double> host_charges;    // 4nc
    std::vector<double4> host_pos, host_nrm;
    std::vector<float4> host_geo32;  // pos32 then nrm32 (2n)

    bool timing = false;
    // event pairs per timed kind: FP64 products, FP32-pair products,
    // treecode products
    std::vector<std::pair<hipEvent_t, hipEvent_t>> pending[3];
    double total_ms[3] = {0, 0, 0};
    int64_t count[3] = {0, 0, 0};

    // treecode product: its tree and device data (rebuilt when the surface,
    // counted by geom_version, or the options change) and the device vectors
    // of the host entry point
    gabi::TreeState *tree = nullptr;
    int64_t geom_version = 0;
    double *tree_u = nullptr, *tree_y = nullptr;
    int64_t tree_io_n = 0;
};

namespace gabi {

// ---- errors ---------------------------------------------------------------
int fail(gabi_ctx *ctx, int code, const std::string &msg);
int hip_fail(gabi_ctx *ctx, hipError_t e, const char *what);
#define GABI_HIP(ctx, expr)                                            \
    do {                                                               \
        hipError_t e_ = (expr);                                        \
        if (e_ != hipSuccess) return ::gabi::hip_fail(ctx, e_, #expr); \
    } while (0)

// ---- launchers ---------------------------------------------------------------
enum PrepMode { kPrepCycle0 = 0, kPrepCycleJ = 1, kPrepResX = 2, kPrepU = 3 };
enum FinishMode { kFinishDot = 0, kFinishRes = 1, kFinishY = 2 };

struct Timer {  // optional event pairs around product launches
    std::vector<std::pair<hipEvent_t, hipEvent_t>> *pending[2] = {nullptr, nullptr};
};

// abi.hip: validation and staging shared with the batched paths
int validate_surface(int64_t n, const double *cx, const double *cy, const double *cz,
                     const double *nx, const double *ny, const double *nz,
                     const double *area, std::string &msg);
int validate_charges(int64_t nc, const double *px, const double *py, const double *pz,
                     const double *q, std::string &msg);
int check_charges_vs_centroids(int64_t n, const double *cx, const double *cy,
                               const double *cz, int64_t nc, const double *px,
                               const double *py, const double *pz, std::string &msg);
int params_valid(double eps1, double eps2, double kappa);
int opts_check(const gabi_solve_opts *in, gabi_solve_opts *o, std::string &msg);
int upload_geometry(Slot &sl, const double4 *pos, const double4 *nrm, const float4 *geo32,
                    hipStream_t s);
int upload_charges(Slot &sl, const double *chg4, hipStream_t s);
void stage_surface(int64_t n, const double *cx, const double *cy, const double *cz,
                   const double *nx, const double *ny, const double *nz, const double *area,
                   std::vector<double4> &pos, std::vector<double4> &nrm,
                   std::vector<float4> &geo32);

// matvec.hip
void launch_prep(const Batch &b, hipStream_t s, int precision, int mode, int j, bool skip);
void launch_pair(Batch &b, hipStream_t s, int precision, bool skip, const Timer *t);
void launch_finish(const Batch &b, hipStream_t s, int precision, int mode, int j, bool skip);
void launch_fold(const Batch &b, hipStream_t s, int precision, int pass, bool skip);
int pair_occupancy_grid(int precision, int variant);
// sources.hip
void launch_rhs(const Batch &b, hipStream_t s);
// phi_reac at the charges and the energy of u (from_sol: of the solution)
void launch_reaction(const Batch &b, hipStream_t s, bool from_sol);
// krylov.hip
void enqueue_init(Batch &b, hipStream_t s, bool x0_given, const Timer *t);
void enqueue_round(Batch &b, hipStream_t s, const Timer *t);
void enqueue_gather(Batch &b, hipStream_t s);
void enqueue_finalize(Batch &b, hipStream_t s);
int run_round(Batch &b, hipStream_t s, hipStream_t capture, const Timer *t,
              bool use_graph, std::string &err);
void graph_round_times(const Batch &b, double *ms, int64_t *count);
void set_solve_targets(Slot &slot, double tol, double inner_tol, int maxit);

}  // namespace gabi
