/*
 * gabi.h -- C ABI of libgabi, a direct-sum boundary-integral solver for the
 * linearized Poisson-Boltzmann equation on MI355X (gfx950).
 *
 * Method: W. Geng and F. Jacob, "A GPU-accelerated Direct-sum Boundary
 * Integral Poisson-Boltzmann Solver", arXiv:1301.5885.
 *   Problem (Section 1, eqs. (eq1)-(radiation)): a molecule (dielectric eps1,
 *   point charges q_k at y_k) bounded by a closed surface Gamma, immersed in
 *   solvent (dielectric eps2, inverse Debye length kappa).
 *   Unknowns (Section 2.2): u = [phi_1(x_i); d phi_1/d nu(x_i)], i = 0..N-1,
 *   at the centroids x_i of N flat triangles (centroid collocation).
 *   Operator (Section 2.2, eqs. (eqdbef1)/(eqdbef2)) with the kernels
 *   K1..K4 of (Eq_Ls); right-hand side S1, S2 of (Eq_Ss); energy
 *   (Section 2.3, eq. (solvation_energy)).
 *
 * Conventions fixed by this library where the paper is silent or
 * inconsistent:
 *   - eps = eps2/eps1 in the kernels and in the diagonal terms (1+eps)/2 and
 *     (1+1/eps)/2.
 *   - S1, S2 carry 1/eps1.
 *   - Charges in units of e, lengths in Angstrom, potentials include the
 *     1/(4 pi) of G0, energies in kcal/mol (4 pi * 332.0716 kcal A/(mol e^2)).
 *   - Vectors of length 2N are laid out [phi_0..phi_{N-1}, psi_0..psi_{N-1}].
 *
 * Ownership: every input array is copied (or read) during the call; the
 * caller keeps ownership of all its buffers.  "_dev" entry points take
 * device pointers (for example from torch tensors) and work on the stream
 * set with gabi_set_stream; the others take host pointers and synchronize.
 * A context is not thread-safe: use one context per host thread.
 *
 * Errors: every int-returning call returns a gabi_status.  On a negative
 * status the context is unchanged unless stated otherwise, and
 * gabi_last_error() describes the failure.
 */
#ifndef GABI_H
#define GABI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gabi_ctx gabi_ctx;

typedef enum {
    GABI_OK = 0,
    GABI_NOT_CONVERGED = 1, /* warning: the solution and info are valid      */
    GABI_EINVAL = -1,       /* bad argument (null pointer, non-finite value) */
    GABI_ESTATE = -2,       /* surface, charges or parameters not set        */
    GABI_EMESH = -3,        /* degenerate element data                       */
    GABI_ENOMEM = -4,       /* device allocation failed                      */
    GABI_EDEVICE = -5,      /* HIP runtime error                             */
    GABI_EBUSY = -6         /* resource limit reached (serving)              */
} gabi_status;

/* Precision of the pair kernels in a product.                              */
typedef enum {
    GABI_FP64 = 0,      /* every pair term in FP64                          */
    GABI_FP32_PAIR = 1  /* pair terms in FP32, row sums accumulated in FP64 */
} gabi_precision;
/* The FP32-pair product rounds the centroids, taken relative to the centre
 * of their bounding box, to FP32 once.  Its relative error therefore grows
 * with the ratio of the surface's extent L to the element size h: about
 * 2^-24 L/h normwise (6e-7 for a 20 A sphere of 20,480 elements, 2e-6 for a
 * 40 A sphere of 327,680).  Solves in GABI_SOLVE_MIXED_IR mode are not
 * limited by it: their residuals are formed with the FP64 product.          */

/* Solver modes.                                                           */
typedef enum {
    GABI_SOLVE_FP64 = 0,     /* restarted GMRES(m) on the FP64 product       */
    GABI_SOLVE_MIXED_IR = 1, /* FP64 iterative refinement around GMRES(m) on
                                the FP32-pair product                        */
    GABI_SOLVE_TREE_IR = 2   /* FP64 iterative refinement around GMRES(m) on
                                the treecode product (gabi_tree_matvec), for
                                large surfaces (Section 1 and Section 4 name
                                tree codes as the route past the direct
                                sum): the residuals are the FP64 direct
                                product's, so the solve meets the same
                                stopping rule.  Single contexts only
                                (gabi_batch_solve and servers: GABI_EINVAL)  */
} gabi_solve_mode;

typedef struct {
    int32_t restart;   /* m, Krylov steps per cycle, 1..64 (default 20, the
                          top of the 10-20 of Section 2.4)                   */
    int32_t maxit;     /* cap on Arnoldi steps over the whole solve (100)     */
    double tol;        /* stop when ||b - A u|| / ||b|| <= tol (1e-6), with
                          the residual always formed with the FP64 product    */
    int32_t mode;      /* gabi_solve_mode (GABI_SOLVE_FP64)                   */
    double inner_tol;  /* MIXED_IR, TREE_IR: each refinement step is one
                          GMRES(m) cycle on the FP32-pair (treecode) product;
                          it stops early once its estimate falls below
                          max(inner_tol, 0.1 tol ||b|| / ||r||) times the
                          current residual r (inner_tol 3e-6)                 */
    int32_t max_outer; /* MIXED_IR, TREE_IR: cap on refinement steps (20)     */
    int32_t use_graph; /* replay each round (cycle, update, residual) as a
                          captured HIP graph (1); with kernel timing on, the
                          captured round records events around its products */
    int32_t x0_previous; /* gabi_solve/gabi_solve_dev with a null x0: 1 starts
                          from the solution this context's last solve
                          returned, which stays on the device while the
                          surface keeps its number of elements (charges,
                          parameters and element data may have changed since:
                          the warm start of a sequence of nearby problems,
                          Section 4); 0, or no such solution, starts from
                          zero.  Batch and server calls ignore it (0)         */
    double tree_theta;   /* TREE_IR: treecode options of the inner products  */
    int32_t tree_degree; /* (gabi_tree_opts; defaults 0.6, 4, 128 and         */
    int32_t tree_leaf;   /* GABI_FP32_PAIR: the residuals are FP64 direct      */
    int32_t tree_precision; /* products whatever the inner precision)        */
} gabi_solve_opts;

typedef struct {
    int64_t iterations;   /* Arnoldi steps, inner steps included             */
    int64_t matvecs_fp64; /* FP64 products (explicit residuals included)     */
    int64_t matvecs_fp32; /* FP32-pair products                               */
    int64_t restarts;     /* completed GMRES cycles                           */
    int64_t outer;        /* refinement steps (MIXED_IR), else 0              */
    double rel_residual;  /* explicit FP64 ||b - A u|| / ||b|| at exit        */
    int32_t converged;    /* 1 if rel_residual <= tol                         */
    double seconds;       /* wall time of the call                            */
    int32_t warm_start;   /* 1 if the initial guess was not zero (x0 given or
                             the previous solution, see x0_previous)          */
    int64_t matvecs_tree; /* treecode products (TREE_IR)                      */
} gabi_solve_info;

/* Fill opts with the defaults listed above.                                */
void gabi_default_opts(gabi_solve_opts *opts);

/* Create a context on HIP device `device` (its null stream until
 * gabi_set_stream).  *out receives the handle.  GABI_EDEVICE if the device
 * cannot be used.                                                           */
int gabi_create(gabi_ctx **out, int device);

/* Free every device buffer of the context.  Null is accepted.              */
void gabi_destroy(gabi_ctx *ctx);

/* Text of the last error on this context (empty string if none).  The
 * pointer stays valid until the next call on the context.                  */
const char *gabi_last_error(const gabi_ctx *ctx);

/* Stream used by all later calls; `stream` is a hipStream_t (0 = null
 * stream).  The caller keeps ownership of the stream.                       */
int gabi_set_stream(gabi_ctx *ctx, void *stream);

/* Element data of a triangle mesh (Section 2.2; host utility, no device
 * work).  xyz: nv x 3 vertex coordinates, row-major.  tri: nf x 3 vertex
 * indices, counter-clockwise seen from outside.  Outputs (nf each):
 * centroid = mean of the vertices, unit normal = normalised
 * (v1-v0)x(v2-v0), area = half its length.  GABI_EMESH for an index out of
 * range or a zero-area triangle.                                            */
int gabi_mesh_elements(int64_t nv, const double *xyz, int64_t nf,
                       const int32_t *tri, double *cx, double *cy, double *cz,
                       double *nx, double *ny, double *nz, double *area);

/* Set the surface: N elements with centroid (cx,cy,cz), outward unit normal
 * (nx,ny,nz) and area, host arrays of length n (Section 2.4: the 7N element
 * arrays).  Rejects n < 4, non-finite values, area <= 0, |normal| off 1 by
 * more than 1e-6, and two elements with the same centroid (GABI_EMESH).
 * Discards any previous solution.                                           */
int gabi_set_surface(gabi_ctx *ctx, int64_t n, const double *cx,
                     const double *cy, const double *cz, const double *nx,
                     const double *ny, const double *nz, const double *area);

/* Same, from a triangle mesh (see gabi_mesh_elements).                      */
int gabi_set_surface_mesh(gabi_ctx *ctx, int64_t nv, const double *xyz,
                          int64_t nf, const int32_t *tri);

/* Set the point charges of the solute, the sources of the interior
 * equation (Section 1, eq. (eq1): the sum of point charges q_k at y_k on the
 * right-hand side; they enter the source terms S1, S2 of eq. (Eq_Ss) and the
 * energy sum of eq. (solvation_energy)): positions (px,py,pz) in Angstrom
 * and charges q in units of e, host arrays of length nc >= 0 (nc = 0 gives b = 0, u = 0 and
 * E = 0).  Non-finite values: GABI_EINVAL.  A charge exactly on an element
 * centroid is rejected with GABI_EINVAL when both surface and charges are
 * set.                                                                      */
int gabi_set_charges(gabi_ctx *ctx, int64_t nc, const double *px,
                     const double *py, const double *pz, const double *q);

/* Dielectric constants eps1 (inside), eps2 (outside) > 0 and inverse Debye
 * length kappa >= 0 in 1/Angstrom (Section 1, eqs. (eq1)-(eq2)).            */
int gabi_set_params(gabi_ctx *ctx, double eps1, double eps2, double kappa);

/* Right-hand side b = [S1(x_i); S2(x_i)] / eps1 of (Eq_Ss), 2N values.      */
int gabi_rhs(gabi_ctx *ctx, double *b);
int gabi_rhs_dev(gabi_ctx *ctx, double *b_dev);

/* y = A u of (eqdbef1)/(eqdbef2), u and y of length 2N, in the requested
 * gabi_precision.  The j = i self term is omitted (Section 2.2).            */
int gabi_matvec(gabi_ctx *ctx, int precision, const double *u, double *y);
int gabi_matvec_dev(gabi_ctx *ctx, int precision, const double *u_dev,
                    double *y_dev);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the FP64
 * product of gabi_matvec_dev, y = A u, with no allocation of any kind.
 * The element data come from the caller's device array elem_dev (32-byte
 * aligned, 8 n doubles): n records (cx, cy, cz, area), then n records
 * (nx, ny, nz, 0) of unit outward normals; it is not validated (the caller
 * vouches for distinct centroids and unit normals).  eps1, eps2, kappa are
 * the context's (gabi_set_params); the context's surface, slot and batch
 * are not used.  u_dev, y_dev: 2n doubles each, device memory.  Work goes
 * on the context's stream; the call returns once it is enqueued.  Weights,
 * partial sums, lists and counters live in a 32 MiB library-owned device
 * array per GPU (held until the process ends), so 1 <= n <= 65,536
 * (GABI_EINVAL otherwise); every call rewrites it from the start.  Calls on
 * one GPU share that array: calls that overlap in time on one GPU (other
 * streams, other contexts, other threads) race and give wrong results.
 * Errors: GABI_ESTATE (no parameters), GABI_EINVAL (size, null or
 * misaligned pointer), GABI_EDEVICE.  Results equal gabi_matvec_dev's at
 * GABI_FP64 up to the grouping of partial sums: bit for bit where the
 * context takes the symmetric scheme in one pass (8,192 <= n <= 20,480 with
 * the shipped tuning table and the default partial-sum budget; below 8,192
 * the table picks the split scheme).                                       */
int gabi_matvec_noalloc(gabi_ctx *ctx, int64_t n, const double *elem_dev,
                        const double *u_dev, double *y_dev);

/* Solve A u = b with b from gabi_rhs.  opts may be null (defaults).  x0
 * (length 2N) is the initial guess, null for zero (Section 2.4).  u receives
 * the solution (length 2N); info may be null.  Returns GABI_OK,
 * GABI_NOT_CONVERGED (u and info still valid) or an error.  The solution is
 * kept on the device for gabi_energy(ctx, NULL, ...).                       */
int gabi_solve(gabi_ctx *ctx, const gabi_solve_opts *opts, const double *x0,
               double *u, gabi_solve_info *info);
int gabi_solve_dev(gabi_ctx *ctx, const gabi_solve_opts *opts,
                   const double *x0_dev, double *u_dev, gabi_solve_info *info);

/* Electrostatic solvation energy (Section 2.3, eq. (solvation_energy)) in
 * kcal/mol for the surface values u (length 2N, host for gabi_energy,
 * device for gabi_energy_dev), or for the last solution if u is null (then
 * the value the solve's final step evaluated is returned without device
 * work).  Always evaluated in FP64.                                         */
int gabi_energy(gabi_ctx *ctx, const double *u, double *e_kcal_per_mol);
int gabi_energy_dev(gabi_ctx *ctx, const double *u_dev,
                    double *e_kcal_per_mol);

/* Reaction potential phi_reac(y_k) at every charge (Section 2.3), nc
 * values written to the host array phi (potential units e/Angstrom with
 * the 1/(4 pi) of G0), for u as in gabi_energy.                             */
int gabi_reaction_potential(gabi_ctx *ctx, const double *u, double *phi);

/* Device memory held by the context in bytes.                               */
int64_t gabi_device_bytes(const gabi_ctx *ctx);

/* Average device duration (milliseconds) per product of the pair-kernel
 * launches of products made since the last reset, measured with HIP events
 * on the context's stream when timing is enabled (from before a product's
 * first pair launch to after its last, folds between passes included;
 * event-record nodes inside a captured round); count receives the number
 * of products.  precision GABI_TIMING_TREE gives the treecode products
 * (all three of their kernels).  Timing adds two event records per product. */
#define GABI_TIMING_TREE 2
int gabi_set_kernel_timing(gabi_ctx *ctx, int enable);
int gabi_kernel_time(gabi_ctx *ctx, int precision, double *avg_ms,
                     int64_t *count, int reset);

/* ------------------------------------------------------------------------ */
/* Decomposition of the product (tuning table).                             */
/* ------------------------------------------------------------------------ */

/* Two decompositions of the product over targets i and sources j != i:
 *
 * GABI_SCHEME_SPLIT      row blocks of 256 * rows_per_thread targets times
 *                        source splits: the last tail_pieces * 64 sources
 *                        form splits of 64 sources each, the sources before
 *                        them splits of whole 256-source tiles sized so that
 *                        about target_blocks workgroups run.  Every ordered
 *                        pair (i, j) is evaluated on its own.
 * GABI_SCHEME_SYMMETRIC  blocks of 256 elements; a workgroup takes a block
 *                        pair (I, J), I < J, and evaluates each unordered
 *                        pair once: the separation, 1/rho, e^{-kappa rho}
 *                        and the A, B factors are shared by the (i, j) and
 *                        (j, i) terms (K1 is symmetric; K2..K4 differ only
 *                        in which normal and weights they use).  Diagonal
 *                        blocks (I, I) evaluate their ordered pairs.  The
 *                        block pairs are taken in the rounds of a
 *                        round-robin tournament (each block once per
 *                        round), and each round leaves one partial sum per
 *                        row.  When a product's rounds need more partial
 *                        sums than the partial-sum budget holds
 *                        (gabi_set_part_budget), it runs as several passes
 *                        of at most that many rounds, each pass folded into
 *                        an FP64 accumulator before the next.
 *                        rows_per_thread must be 1; target_blocks and
 *                        tail_pieces are not used.
 *
 * Work items are taken longest first.  A row's partial sums are added in
 * a fixed order, and the decomposition depends only on N, the precision,
 * this table and the partial-sum budget, so set them before creating
 * contexts or servers: every solve made under one table and budget is
 * bitwise reproducible, alone or batched.  The
 * table holds one entry per precision and N bucket (bucket = floor(log2 N),
 * 0..39).  rows_per_thread is 1 or 2; target_blocks in [1, 2^20];
 * tail_pieces in [0, 4096].  GABI_EINVAL otherwise.                          */
typedef enum { GABI_SCHEME_SPLIT = 0, GABI_SCHEME_SYMMETRIC = 1 } gabi_scheme;
int gabi_tune_set(int precision, int bucket, int scheme, int rows_per_thread,
                  int target_blocks, int tail_pieces);
int gabi_tune_get(int precision, int bucket, int *scheme, int *rows_per_thread,
                  int *target_blocks, int *tail_pieces);

/* Partial-sum budget: bytes one molecule's partial row sums of one
 * precision may take (default 512 MiB).  The symmetric scheme keeps
 * min(nbk, budget / (2 N x 8 bytes FP64, x 4 bytes FP32 pair)) slots per
 * row, nbk = ceil(N / 256), so a molecule's device memory is O(N) for a
 * given budget (the paper keeps O(N) device memory, Section 2.4).  Applies
 * to contexts, batches and servers whose molecules are sized after the
 * call.  bytes >= 1; GABI_EINVAL otherwise.                                 */
int gabi_set_part_budget(int64_t bytes);
int64_t gabi_get_part_budget(void);

/* ------------------------------------------------------------------------ */
/* Molecular surfaces and charges from files (host only).                   */
/* ------------------------------------------------------------------------ */

/* The paper's host reads the molecule (atom coordinates, radii, charges)
 * and the MSMS triangulation of its surface (Section 2.4, table tb_GPU).
 * MSMS files: <name>.vert (a count line, then "x y z nx ny nz ..." per
 * vertex, the vertex normal pointing out) and <name>.face (a count line,
 * then "v1 v2 v3 ..." per triangle, 1-based); lines starting with '#' are
 * comments.  PQR files: ATOM/HETATM records whose last five fields are
 * x y z charge radius.  Paths are NUL-terminated; arrays are caller-owned
 * host memory.  Unreadable file: GABI_EINVAL; malformed record, index out
 * of range or count mismatch: GABI_EMESH.                                   */
int gabi_msms_counts(const char *vert_path, const char *face_path, int64_t *nv, int64_t *nf);
/* xyz: 3 nv doubles; vnormal: 3 nv doubles or null; tri: 3 nf 0-based
 * vertex indices (as gabi_set_surface_mesh takes them).                    */
int gabi_msms_read(const char *vert_path, const char *face_path, int64_t nv, double *xyz,
                   double *vnormal, int64_t nf, int32_t *tri);
/* Rewinds every triangle whose right-hand normal points against the mean of
 * its vertex normals, so that all are counter-clockwise seen from outside
 * (the orientation gabi_set_surface_mesh assumes); *flipped receives how
 * many were rewound.                                                        */
int gabi_msms_orient(int64_t nv, const double *xyz, const double *vnormal, int64_t nf,
                     int32_t *tri, int64_t *flipped);
int gabi_pqr_count(const char *path, int64_t *natoms);
/* xyz: 3 natoms doubles, q: natoms charges (e), radius: natoms or null.     */
int gabi_pqr_read(const char *path, int64_t natoms, double *xyz, double *q, double *radius);

/* ------------------------------------------------------------------------ */
/* Treecode approximation of the product.                                   */
/* ------------------------------------------------------------------------ */

/* The paper evaluates the product by direct summation, O(N^2), and names
 * tree codes, O(N log N), as the route to larger surfaces (Section 1;
 * Section 4).  This is the barycentric Lagrange treecode of Wang, Krasny and
 * Tlupova (Commun. Comput. Phys. 28, 2020), particle-cluster form with
 * target batches, in FP64:
 *   - the centroids are split recursively (minimal boxes, cut at the box
 *     midpoint in every dimension of at least 1/sqrt 2 of the largest
 *     extent) down to leaves of at most leaf_size elements, the batches;
 *   - a cluster C acts on a batch B through (degree+1)^3 proxy points (the
 *     tensor Chebyshev points of the second kind of its box, carrying
 *     weights interpolated from its elements with barycentric Lagrange
 *     bases) when (r_B + r_C) < theta R (radii of the boxes, R the distance
 *     of their centres) and C has more elements than proxies; directly when
 *     the criterion holds and it has fewer; else through its children (a
 *     leaf directly).
 * theta in [0, 1) (0: every pair directly, the exact product up to
 * summation order), degree in [1, 8], leaf_size in [1, 256], precision
 * GABI_FP64 or GABI_FP32_PAIR; GABI_EINVAL otherwise.  The tree is built on the host at the first product after the
 * surface or the options change and kept on the device.                    */
typedef struct {
    double theta;
    int32_t degree;
    int32_t leaf_size;
    int32_t precision;  /* GABI_FP64: every pair term in FP64; GABI_FP32_PAIR:
                           pair terms in FP32 on coordinates relative to the
                           centre of the surface's bounding box, each staged
                           chunk of at most 256 sources summed in FP32 and
                           added to FP64 sums (as the FP32-pair product) */
    int32_t reserved;   /* 0                                                 */
} gabi_tree_opts;

typedef struct {
    int64_t leaves;                 /* target batches                        */
    int64_t clusters_with_proxies;  /* clusters acting through proxies       */
    int64_t far_entries, near_entries;  /* interaction-list entries          */
    int64_t far_pairs, near_pairs;  /* (target, proxy) and (target, element)
                                       pairs per product (near pairs include
                                       each batch's own diagonal)            */
    int64_t device_bytes;           /* device memory of the tree data        */
} gabi_tree_info;

/* y = A u approximated by the treecode, as gabi_matvec (host vectors of 2N
 * doubles) and gabi_matvec_dev (device vectors, on the context's stream).
 * Needs the surface and the parameters (GABI_ESTATE otherwise).           */
int gabi_tree_matvec(gabi_ctx *ctx, const gabi_tree_opts *opts, const double *u,
                     double *y);
int gabi_tree_matvec_dev(gabi_ctx *ctx, const gabi_tree_opts *opts,
                         const double *u_dev, double *y_dev);
/* Statistics of the context's tree for these options (builds it).          */
int gabi_tree_info_get(gabi_ctx *ctx, const gabi_tree_opts *opts, gabi_tree_info *out);
/* The same statistics from centroids alone, on the host (no device).       */
int gabi_tree_plan(int64_t n, const double *cx, const double *cy, const double *cz,
                   const gabi_tree_opts *opts, gabi_tree_info *out);

/* ------------------------------------------------------------------------ */
/* Self-test of device arithmetic.                                          */
/* ------------------------------------------------------------------------ */

/* The FP64 e^{-t} the pair kernels use (the exponential of the screened
 * Coulomb kernel, Section 2.1 eq. (eq_potential), in K1..K4 of eq. (Eq_Ls)),
 * evaluated on `device` at n host values 0 <= t (finite) into out (host);
 * for accuracy tests.  GABI_EINVAL for bad arguments.                       */
int gabi_selftest_exp_neg(int device, int64_t n, const double *t, double *out);

/* ------------------------------------------------------------------------ */
/* Many molecules at once.                                                  */
/* ------------------------------------------------------------------------ */

/* One solve request: a surface as element arrays (as gabi_set_surface), the
 * charges (as gabi_set_charges) and the parameters (as gabi_set_params).
 * All arrays are host memory read during the call that takes the problem.
 * u_out: optional host buffer of 2N doubles that receives the solution; the
 * caller keeps it valid until the result has been returned.  tag: any
 * caller value, copied into the result (tags need not be unique; the
 * result's ticket identifies the request).                                 */
typedef struct {
    int64_t n;
    const double *cx, *cy, *cz, *nx, *ny, *nz, *area;
    int64_t nc;
    const double *px, *py, *pz, *q;
    double eps1, eps2, kappa;
    double *u_out;
    int64_t tag;
} gabi_problem;

typedef struct {
    int64_t tag;
    int32_t status;        /* GABI_OK, GABI_NOT_CONVERGED or an error code */
    double energy;         /* E_sol, kcal/mol                              */
    gabi_solve_info info;
    double t_submit;       /* seconds, monotonic clock of the server       */
    double t_admit;        /* admitted to the device                       */
    double t_done;         /* result ready                                 */
    int64_t device_bytes;  /* device memory the solve held                 */
    int64_t ticket;        /* the server's sequence number of the request
                              (gabi_server_submit); the problem index in
                              gabi_batch_solve                              */
} gabi_result;

/* Device bytes one solve of n elements and nc charges holds with GMRES(m)
 * (the unit of admission; the paper's own count is 11N + 6Nc doubles,
 * Section 2.4, for its host-driven GMRES).                                 */
int64_t gabi_solve_footprint(int64_t n, int64_t nc, int32_t restart);

/* Solve nprob problems together on `device`: every kernel launch covers all
 * molecules still iterating (one batched product over a tile queue per
 * Arnoldi step); a molecule leaves the batch when it converges or reaches
 * maxit.  Each molecule is decomposed and reduced exactly as when it is
 * solved alone, so results[k] is bitwise the result of a batch of one.
 * opts as gabi_solve (shared by all problems).  results: nprob records,
 * filled in problem order.  Returns GABI_OK when every problem was
 * processed (per-problem status in results), or an error for the call.   */
int gabi_batch_solve(int device, int64_t nprob, const gabi_problem *probs,
                     const gabi_solve_opts *opts, gabi_result *results);

/* Serving: a worker thread owns one device, an arena of budget_bytes of
 * device memory and a FIFO queue.  A request is admitted when it is at the
 * head of the queue, fewer than max_slots solves are active and its
 * footprint fits in the free arena; admitted requests join the running
 * batch at the next round boundary (continuous batching) and leave it when
 * done, freeing their memory for the queue.  device = -1 runs the same
 * scheduler against a host-only executor that performs no arithmetic
 * (rounds take `mock_round_seconds`, a request finishes after
 * ceil(N / 4096) rounds) so admission can be exercised without a GPU.     */
typedef struct gabi_server gabi_server;

typedef struct {
    int64_t submitted, admitted, completed, failed;
    int64_t queued;          /* waiting for admission                      */
    int64_t active;          /* on the device                              */
    int64_t rounds;          /* batched rounds run                         */
    int64_t max_active;      /* most solves on the device at once          */
    int64_t bytes_in_use;    /* arena bytes held by active solves          */
    int64_t peak_bytes;
    int64_t budget_bytes;
} gabi_server_stats;

int gabi_server_create(gabi_server **out, int device, int64_t budget_bytes,
                       int32_t max_slots, const gabi_solve_opts *opts,
                       double mock_round_seconds);
/* Copies the problem and queues it; *ticket (may be null) receives a
 * sequence number.  GABI_EINVAL for bad data, GABI_ENOMEM if its footprint
 * exceeds the whole budget (it could never be admitted).                   */
int gabi_server_submit(gabi_server *srv, const gabi_problem *p, int64_t *ticket);
/* Moves up to max finished results (completion order) into out; *count
 * receives how many.  Never blocks.                                        */
int gabi_server_poll(gabi_server *srv, gabi_result *out, int32_t max, int32_t *count);
/* Blocks until every submitted request has finished or timeout_s elapses;
 * GABI_EBUSY on timeout.                                                   */
int gabi_server_drain(gabi_server *srv, double timeout_s);
/* Round cap, for latency of the largest requests: each round runs the
 * oldest active request and, in admission order, each further one whose
 * work (N^2) keeps the round's total within
 * max((1 + slack) x the oldest's work, floor_elements^2); the others wait a
 * round.  slack < 0 (the default) runs every active request every round.
 * Results do not depend on it (a request's arithmetic is the same in any
 * round).  Takes effect from the next round.  GABI_EINVAL for a non-finite
 * slack or a negative floor.                                                */
int gabi_server_set_round_cap(gabi_server *srv, double slack, int64_t floor_elements);
int gabi_server_stats_get(gabi_server *srv, gabi_server_stats *out);
/* Seconds on the server's monotonic clock (the clock of gabi_result).      */
double gabi_server_clock(gabi_server *srv);
const char *gabi_server_last_error(gabi_server *srv);
/* Stops the worker after the current round; unfinished requests are
 * dropped.  Frees the arena.                                               */
void gabi_server_destroy(gabi_server *srv);

#ifdef __cplusplus
}
#endif

#endif /* GABI_H */
