// Allocation-free FP64 product y = A u (Section 2.2, eqs. (eqdbef1)/(eqdbef2))
// for callers that cannot allocate device memory: code under HIP graph
// capture, tight serving loops, harnesses that forbid hipMalloc.
//
// It runs the kernels of gabi_matvec_dev at GABI_FP64 (weights, symmetric
// pair tiles, folds, finish) on element data the caller already holds on the
// device.  Everything else those kernels need -- the molecule descriptor, the
// block and tile lists, the tile-queue counters, the weights, the partial
// sums and the FP64 accumulator of a product taken in several passes -- lives
// in one file-scope device array, `scratch`, of kScratchBytes.  Its address
// on each device is looked up once (hipGetSymbolAddress, on the first call
// on that device, with that device current) and only that address is
// handed to kernels: in host code the array's name is a host stand-in, not a
// device address.
//
// Every call first runs a set-up kernel that writes the descriptor, the
// lists (the round-robin tile schedule of the symmetric scheme, generated on
// the device) and zero counters into the scratch, so nothing carries over
// between calls.  The number of partial-sum slots per pass is the most that
// fit beside the fixed parts; a product needs more passes than the context's
// (whose slots follow the partial-sum budget) when N is large, and the
// context takes the tuned decomposition (the split scheme at small N), so
// the two entry points may add the same terms in a different grouping:
// equal up to rounding, bit for bit only where both take the symmetric
// scheme in the same passes.  Calls on one device share its scratch and
// must not overlap (one stream, or synchronised streams).
#include <mutex>

#include "gabi_internal.h"

namespace gabi {

constexpr int64_t kScratchBytes = int64_t(32) << 20;  // per device
constexpr int64_t kNoallocMaxN = 65536;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) char scratch[kScratchBytes];

namespace {

std::mutex g_scratch_mu;
char *g_scratch_ptr[kMaxDevices] = {nullptr};

// Device address of this device's scratch (the device must be current).
int scratch_address(int device, char **out, std::string &msg) {
    if (device < 0 || device >= kMaxDevices) {
        msg = "device ordinal out of range";
        return GABI_EINVAL;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            msg = std::string("hipGetSymbolAddress(scratch) failed: ") + hipGetErrorString(e);
            return GABI_EDEVICE;
        }
        g_scratch_ptr[device] = static_cast<char *>(p);
    }
    *out = g_scratch_ptr[device];
    return GABI_OK;
}

// Byte offsets of the scratch parts for n elements, and the pass structure.
struct NoallocPlan {
    int64_t o_mol = 0, o_elem = 0, o_blas = 0, o_tiles = 0, o_xoff = 0, o_cnt = 0, o_wgt = 0,
            o_acc = 0, o_part = 0, total = 0;
    int nbk = 0, n_elem = 0, n_blas = 0, ntiles = 0, slots = 0, passes = 0, last = 0;
};

int64_t al256(int64_t v) { return (v + 255) & ~int64_t(255); }

// Tiles of round r and their first index in round order (sym_schedule.h:
// nbk odd, every round has (nbk + 1)/2 tiles; nbk even, the first nbk - 1
// rounds have nbk/2 and the diagonal round nbk).
__host__ __device__ inline int round_tiles(int nbk, int r) {
    if (nbk % 2) return (nbk + 1) / 2;
    return r == nbk - 1 ? nbk : nbk / 2;
}
__host__ __device__ inline int round_first(int nbk, int r) {
    return nbk % 2 ? r * ((nbk + 1) / 2) : r * (nbk / 2);
}

NoallocPlan noalloc_plan(int64_t n) {
    NoallocPlan P;
    P.nbk = (int)((n + kTile - 1) / kTile);
    P.n_elem = P.nbk;
    P.n_blas = blas_blocks(n);
    P.ntiles = P.nbk * (P.nbk + 1) / 2;
    int64_t off = 0;
    auto take = [&](int64_t bytes) {
        off = al256(off);
        const int64_t at = off;
        off += std::max<int64_t>(1, bytes);
        return at;
    };
    P.o_mol = take(sizeof(Mol));
    P.o_elem = take(sizeof(int2) * (int64_t)P.n_elem);
    P.o_blas = take(sizeof(int2) * (int64_t)P.n_blas);
    P.o_tiles = take(sizeof(int4) * (int64_t)P.ntiles);
    P.o_xoff = take(sizeof(int) * (int64_t)(kXcdLists + 1) * P.nbk);  // passes <= nbk
    P.o_cnt = take(256);
    P.o_wgt = take(sizeof(double4) * n);
    P.o_acc = take(sizeof(double) * 2 * n);
    P.o_part = al256(off);
    // FP64 partial sums: 2n doubles per slot
    const int64_t slot_bytes_ = 16 * n;
    const int64_t fit = (kScratchBytes - P.o_part) / slot_bytes_;
    sym_passes(P.nbk, fit, P.passes, P.slots);
    P.last = P.nbk - (P.passes - 1) * P.slots;
    P.total = P.o_part + slot_bytes_ * P.slots;
    return P;
}

}  // namespace

// Writes the descriptor, the element and reduction block lists, the
// symmetric tiles of every round (round order; round r writes slot r mod S
// in pass r / S), the cut of each pass into the symmetric kernel's lists
// (equal counts, in round order) and zero tile-queue counters into the
// scratch.
__global__ __launch_bounds__(kBlock) void noalloc_setup_kernel(Mol M, char *base, NoallocPlan P) {
    const int g = (int)(blockIdx.x * kBlock + threadIdx.x);
    const int nbk = P.nbk;
    if (g == 0) *reinterpret_cast<Mol *>(base + P.o_mol) = M;
    if (g < 64) reinterpret_cast<int *>(base + P.o_cnt)[g] = 0;
    if (g < P.n_elem) reinterpret_cast<int2 *>(base + P.o_elem)[g] = make_int2(0, g);
    if (g < P.n_blas) reinterpret_cast<int2 *>(base + P.o_blas)[g] = make_int2(0, g);
    if (g < P.passes * (kXcdLists + 1)) {
        const int p = g / (kXcdLists + 1), x = g % (kXcdLists + 1);
        const int r0 = p * P.slots, r1 = min(r0 + P.slots, nbk);
        const int len = (r1 == nbk ? P.ntiles : round_first(nbk, r1)) - round_first(nbk, r0);
        reinterpret_cast<int *>(base + P.o_xoff)[g] = len * x / kXcdLists;
    }
    if (g >= nbk * nbk) return;
    const int r = g / nbk, k = g % nbk;
    if (k >= round_tiles(nbk, r)) return;
    int a, b;
    if (nbk % 2) {
        // blocks rotate around a dummy; block r meets it (its diagonal tile)
        if (k == 0) {
            a = b = r;
        } else {
            a = (r + k) % nbk;
            b = (r - k + nbk) % nbk;
        }
    } else if (r == nbk - 1) {
        a = b = k;  // the diagonal round
    } else {
        const int m = nbk - 1;  // block nbk - 1 stays fixed
        if (k == 0) {
            a = r;
            b = nbk - 1;
        } else {
            a = (r + k) % m;
            b = (r - k + m) % m;
        }
    }
    const int I = a < b ? a : b, J = a < b ? b : a;
    const int w = (r % P.slots) | ((r / P.slots) << 16);
    reinterpret_cast<int4 *>(base + P.o_tiles)[round_first(nbk, r) + k] = make_int4(0, I, J, w);
}

}  // namespace gabi

using namespace gabi;

extern "C" {

int gabi_matvec_noalloc(gabi_ctx *ctx, int64_t n, const double *elem_dev, const double *u_dev,
                        double *y_dev) {
    if (!ctx) return GABI_EINVAL;
    if (!ctx->params_set) return fail(ctx, GABI_ESTATE, "parameters not set");
    if (n < 1 || n > kNoallocMaxN)
        return fail(ctx, GABI_EINVAL,
                    "gabi_matvec_noalloc: n = " + std::to_string(n) + " outside [1, " +
                        std::to_string(kNoallocMaxN) + "] (its scratch holds " +
                        std::to_string(kScratchBytes >> 20) + " MiB)");
    if (!elem_dev || !u_dev || !y_dev) return fail(ctx, GABI_EINVAL, "null device pointer");
    if (reinterpret_cast<uintptr_t>(elem_dev) % 32 != 0)
        return fail(ctx, GABI_EINVAL, "elem_dev must be 32-byte aligned");
    GABI_HIP(ctx, hipSetDevice(ctx->device));
    char *base = nullptr;
    std::string msg;
    int rc = scratch_address(ctx->device, &base, msg);
    if (rc) return fail(ctx, rc, msg);
    const NoallocPlan P = noalloc_plan(n);
    if (P.total > kScratchBytes || P.passes > kMaxPasses || P.slots < 1)
        return fail(ctx, GABI_EINVAL, "gabi_matvec_noalloc: n = " + std::to_string(n) +
                                          " does not fit the scratch");
    // the descriptor: the caller's elements and vectors, the rest in scratch
    Mol M{};
    PairLaunch L;
    L.scheme = GABI_SCHEME_SYMMETRIC;
    L.rows_per_thread = 1;
    L.row_blocks = P.nbk;
    L.splits = P.slots;
    L.passes = P.passes;
    L.last = P.last;
    M.n = (int32_t)n;
    M.nb = P.n_blas;
    M.mode = kModeFP64;
    mol_decomposition(M, n, L, L);
    mol_set_params(M, ctx->eps1, ctx->eps2, ctx->kappa);
    M.pos = reinterpret_cast<const double4 *>(elem_dev);
    M.nrm = M.pos + n;
    M.wgt = reinterpret_cast<double4 *>(base + P.o_wgt);
    M.part = reinterpret_cast<double *>(base + P.o_part);
    M.acc = reinterpret_cast<double *>(base + P.o_acc);
    M.u = const_cast<double *>(u_dev);  // read only (weights and diagonal)
    M.y = y_dev;
    // a batch of one whose device arrays are the scratch's
    Batch b;
    b.d_mols = reinterpret_cast<Mol *>(base + P.o_mol);
    b.d_elem = reinterpret_cast<int2 *>(base + P.o_elem);
    b.n_elem = P.n_elem;
    b.d_blas = reinterpret_cast<int2 *>(base + P.o_blas);
    b.n_blas = P.n_blas;
    b.d_tiles64 = reinterpret_cast<int4 *>(base + P.o_tiles);
    b.d_xoff64 = reinterpret_cast<int *>(base + P.o_xoff);
    b.n_tiles64[2] = P.ntiles;
    b.n_pass64 = P.passes;
    for (int p = 0; p <= P.passes; ++p) {
        const int r = std::min(p * P.slots, P.nbk);
        b.sym_off64[p] = r == P.nbk ? P.ntiles : round_first(P.nbk, r);
    }
    b.d_counter = reinterpret_cast<int *>(base + P.o_cnt);
    b.persistent = true;
    pair_grids(b.grid64, b.grid32);
    const int setup_threads =
        std::max({P.nbk * P.nbk, P.n_elem, P.n_blas, 64, P.passes * (kXcdLists + 1)});
    hipLaunchKernelGGL(noalloc_setup_kernel, dim3((setup_threads + kBlock - 1) / kBlock),
                       dim3(kBlock), 0, ctx->stream, M, base, P);
    launch_prep(b, ctx->stream, GABI_FP64, kPrepU, 0, false);
    launch_pair(b, ctx->stream, GABI_FP64, false, nullptr);
    launch_finish(b, ctx->stream, GABI_FP64, kFinishY, 0, false);
    GABI_HIP(ctx, hipGetLastError());
    return GABI_OK;
}

}  // extern "C"
