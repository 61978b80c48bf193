// C ABI of libgabi for a single molecule (declared in include/gabi.h):
// contexts, validation of element and charge data, and the host/device
// entry points.  A context owns one slot (the molecule's device buffers) and
// runs it as a batch of one through the same kernels the batched solver and
// the server use.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <numeric>
#include <unordered_map>

#include "gabi_internal.h"

namespace gabi {

int fail(gabi_ctx *ctx, int code, const std::string &msg) {
    if (ctx) ctx->err = msg;
    return code;
}

int hip_fail(gabi_ctx *ctx, hipError_t e, const char *what) {
    return fail(ctx, e == hipErrorOutOfMemory ? GABI_ENOMEM : GABI_EDEVICE,
                std::string(what) + ": " + hipGetErrorString(e));
}

}  // namespace gabi

using namespace gabi;

namespace {

struct Key {
    double x, y, z;
    bool operator==(const Key &o) const { return x == o.x && y == o.y && z == o.z; }
};
struct KeyHash {
    size_t operator()(const Key &k) const {
        uint64_t a, b, c;
        std::memcpy(&a, &k.x, 8);
        std::memcpy(&b, &k.y, 8);
        std::memcpy(&c, &k.z, 8);
        uint64_t h = a * 0x9E3779B97F4A7C15ull;
        h ^= b + 0x7F4A7C159E3779B9ull + (h << 6) + (h >> 2);
        h ^= c + 0x94D049BB133111EBull + (h << 6) + (h >> 2);
        return (size_t)h;
    }
};

bool is_finite(double v) { return std::isfinite(v); }

}  // namespace

namespace gabi {

// Shared validation (also used by the batched solver and the server).
int validate_surface(int64_t n, const double *cx, const double *cy, const double *cz,
                     const double *nx, const double *ny, const double *nz,
                     const double *area, std::string &msg) {
    if (!cx || !cy || !cz || !nx || !ny || !nz || !area) {
        msg = "null surface array";
        return GABI_EINVAL;
    }
    if (n < 4) {
        msg = "a closed surface needs at least 4 elements";
        return GABI_EMESH;
    }
    if (n > (int64_t)INT32_MAX / 4) {
        msg = "too many elements";
        return GABI_EINVAL;
    }
    for (int64_t i = 0; i < n; ++i) {
        if (!is_finite(cx[i]) || !is_finite(cy[i]) || !is_finite(cz[i]) || !is_finite(nx[i]) ||
            !is_finite(ny[i]) || !is_finite(nz[i]) || !is_finite(area[i])) {
            msg = "non-finite element data at " + std::to_string(i);
            return GABI_EMESH;
        }
        if (!(area[i] > 0.0)) {
            msg = "element " + std::to_string(i) + " has area <= 0";
            return GABI_EMESH;
        }
        const double nn = std::sqrt(nx[i] * nx[i] + ny[i] * ny[i] + nz[i] * nz[i]);
        if (std::fabs(nn - 1.0) > 1e-6) {
            msg = "normal of element " + std::to_string(i) + " is not unit";
            return GABI_EMESH;
        }
    }
    std::vector<int64_t> idx((size_t)n);
    std::iota(idx.begin(), idx.end(), (int64_t)0);
    std::sort(idx.begin(), idx.end(), [&](int64_t a, int64_t b) {
        if (cx[a] != cx[b]) return cx[a] < cx[b];
        if (cy[a] != cy[b]) return cy[a] < cy[b];
        return cz[a] < cz[b];
    });
    for (int64_t t = 1; t < n; ++t) {
        const int64_t a = idx[t - 1], b = idx[t];
        if (cx[a] == cx[b] && cy[a] == cy[b] && cz[a] == cz[b]) {
            msg = "elements " + std::to_string(a) + " and " + std::to_string(b) +
                  " share a centroid";
            return GABI_EMESH;
        }
    }
    return GABI_OK;
}

int validate_charges(int64_t nc, const double *px, const double *py, const double *pz,
                     const double *q, std::string &msg) {
    if (nc < 0) {
        msg = "negative charge count";
        return GABI_EINVAL;
    }
    if (nc > 0 && (!px || !py || !pz || !q)) {
        msg = "null charge array";
        return GABI_EINVAL;
    }
    if (nc > (int64_t)INT32_MAX / 4) {
        msg = "too many charges";
        return GABI_EINVAL;
    }
    for (int64_t k = 0; k < nc; ++k)
        if (!is_finite(px[k]) || !is_finite(py[k]) || !is_finite(pz[k]) || !is_finite(q[k])) {
            msg = "non-finite charge data at " + std::to_string(k);
            return GABI_EINVAL;
        }
    return GABI_OK;
}

// A charge exactly on a centroid makes a source term singular.
// Centroid i is (c[i * cs], c[i * cs + off_y], c[i * cs + off_z]).  The
// charges (usually far fewer than the elements) go into the hash table and
// every centroid is looked up, so a call costs O(N + Nc) with a small table;
// the error names the lowest-numbered charge that coincides with a centroid.
static int charges_on_centroids(int64_t n, const double *cx, const double *cy,
                                const double *cz, int64_t cs, int64_t nc, const double *px,
                                const double *py, const double *pz, std::string &msg) {
    if (n == 0 || nc == 0) return GABI_OK;
    std::unordered_map<Key, int64_t, KeyHash> chg;
    chg.reserve((size_t)nc * 2);
    for (int64_t k = nc - 1; k >= 0; --k) chg[Key{px[k], py[k], pz[k]}] = k;  // lowest k wins
    int64_t hit = -1;
    for (int64_t i = 0; i < n; ++i) {
        const auto it = chg.find(Key{cx[i * cs], cy[i * cs], cz[i * cs]});
        if (it != chg.end() && (hit < 0 || it->second < hit)) hit = it->second;
    }
    if (hit >= 0) {
        msg = "charge " + std::to_string(hit) + " lies exactly on an element centroid";
        return GABI_EINVAL;
    }
    return GABI_OK;
}

int check_charges_vs_centroids(int64_t n, const double *cx, const double *cy,
                               const double *cz, int64_t nc, const double *px,
                               const double *py, const double *pz, std::string &msg) {
    return charges_on_centroids(n, cx, cy, cz, 1, nc, px, py, pz, msg);
}

int params_valid(double eps1, double eps2, double kappa) {
    return eps1 > 0.0 && eps2 > 0.0 && kappa >= 0.0 && std::isfinite(eps1) &&
           std::isfinite(eps2) && std::isfinite(kappa);
}

int opts_check(const gabi_solve_opts *in, gabi_solve_opts *o, std::string &msg) {
    gabi_default_opts(o);
    if (in) *o = *in;
    if (o->restart < 1 || o->restart > kMaxRestart) {
        msg = "restart must be in [1, 64]";
        return GABI_EINVAL;
    }
    if (o->maxit < 0) {
        msg = "maxit must be >= 0";
        return GABI_EINVAL;
    }
    if (!(o->tol > 0.0) || !std::isfinite(o->tol)) {
        msg = "tol must be > 0";
        return GABI_EINVAL;
    }
    if (o->mode != GABI_SOLVE_FP64 && o->mode != GABI_SOLVE_MIXED_IR &&
        o->mode != GABI_SOLVE_TREE_IR) {
        msg = "unknown solve mode";
        return GABI_EINVAL;
    }
    if (o->mode != GABI_SOLVE_FP64 &&
        (!(o->inner_tol > 0.0) || !(o->inner_tol < 1.0) || o->max_outer < 1)) {
        msg = "need 0 < inner_tol < 1 and max_outer >= 1";
        return GABI_EINVAL;
    }
    if (o->mode == GABI_SOLVE_TREE_IR &&
        (!(o->tree_theta >= 0.0 && o->tree_theta < 1.0) || o->tree_degree < 1 ||
         o->tree_degree > 8 || o->tree_leaf < 1 || o->tree_leaf > kBlock ||
         (o->tree_precision != GABI_FP64 && o->tree_precision != GABI_FP32_PAIR))) {
        msg = "treecode options: theta in [0, 1), degree in [1, 8], leaf in [1, 256], "
              "precision GABI_FP64 or GABI_FP32_PAIR";
        return GABI_EINVAL;
    }
    if (o->x0_previous != 0 && o->x0_previous != 1) {
        msg = "x0_previous must be 0 or 1";
        return GABI_EINVAL;
    }
    return GABI_OK;
}

// Upload of staged host data into a carved slot (synchronous on stream s).
int upload_geometry(Slot &sl, const double4 *pos, const double4 *nrm, const float4 *geo32,
                    hipStream_t s) {
    const int64_t n = sl.mol.n;
    hipError_t e = hipMemcpyAsync((void *)sl.mol.pos, pos, sizeof(double4) * n,
                                  hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync((void *)sl.mol.nrm, nrm, sizeof(double4) * n, hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync((void *)sl.mol.pos32, geo32, sizeof(float4) * 2 * n,
                           hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    return e == hipSuccess ? GABI_OK : GABI_EDEVICE;
}

int upload_charges(Slot &sl, const double *chg4, hipStream_t s) {
    if (sl.mol.nc == 0) return GABI_OK;
    hipError_t e = hipMemcpyAsync((void *)sl.mol.chg, chg4, sizeof(double4) * sl.mol.nc,
                                  hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    return e == hipSuccess ? GABI_OK : GABI_EDEVICE;
}

void stage_surface(int64_t n, const double *cx, const double *cy, const double *cz,
                   const double *nx, const double *ny, const double *nz, const double *area,
                   std::vector<double4> &pos, std::vector<double4> &nrm,
                   std::vector<float4> &geo32) {
    pos.resize((size_t)n);
    nrm.resize((size_t)n);
    geo32.resize((size_t)(2 * n));
    // FP32 coordinates for the mixed product are taken relative to the centre
    // of the bounding box, which keeps their magnitude (and so their
    // rounding error) as small as a single origin allows.
    double lo[3] = {cx[0], cy[0], cz[0]}, hi[3] = {cx[0], cy[0], cz[0]};
    for (int64_t i = 1; i < n; ++i) {
        lo[0] = std::min(lo[0], cx[i]), hi[0] = std::max(hi[0], cx[i]);
        lo[1] = std::min(lo[1], cy[i]), hi[1] = std::max(hi[1], cy[i]);
        lo[2] = std::min(lo[2], cz[i]), hi[2] = std::max(hi[2], cz[i]);
    }
    const double ox = 0.5 * (lo[0] + hi[0]), oy = 0.5 * (lo[1] + hi[1]),
                 oz = 0.5 * (lo[2] + hi[2]);
    for (int64_t i = 0; i < n; ++i) {
        pos[i] = make_double4(cx[i], cy[i], cz[i], area[i]);
        nrm[i] = make_double4(nx[i], ny[i], nz[i], 0.0);
        geo32[i] = make_float4((float)(cx[i] - ox), (float)(cy[i] - oy), (float)(cz[i] - oz),
                               0.0f);
        geo32[n + i] = make_float4((float)nx[i], (float)ny[i], (float)nz[i], 0.0f);
    }
}

}  // namespace gabi

namespace {

int use_device(gabi_ctx *ctx) {
    GABI_HIP(ctx, hipSetDevice(ctx->device));
    return GABI_OK;
}

void free_slot(gabi_ctx *ctx) {
    if (ctx->slot.mem) (void)hipFree(ctx->slot.mem);
    ctx->slot.mem = nullptr;
    ctx->slot.bytes = 0;
    ctx->slot_n = ctx->slot_nc = -1;
    ctx->m_alloc = 0;
    ctx->batch_dirty = true;
}

// Make the slot match the staged data (sizes, restart length), upload what
// changed and rebuild the batch of one.
int ensure_slot(gabi_ctx *ctx, int m) {
    int rc = use_device(ctx);
    if (rc) return rc;
    m = std::max(m, std::max(ctx->m_alloc, 10));
    if (!ctx->slot.mem || ctx->slot_n != ctx->n || ctx->slot_nc != ctx->nc || m > ctx->m_alloc) {
        if (ctx->stream) GABI_HIP(ctx, hipStreamSynchronize(ctx->stream));
        free_slot(ctx);
        const int64_t bytes = slot_bytes(ctx->n, ctx->nc, m);
        hipError_t e = hipMalloc(&ctx->slot.mem, bytes);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            ctx->slot.mem = nullptr;
            return fail(ctx, GABI_ENOMEM, "device allocation of " + std::to_string(bytes) +
                                              " bytes failed");
        }
        ctx->slot.bytes = bytes;
        slot_carve(ctx->slot, ctx->n, ctx->nc, m);
        ctx->slot_n = ctx->n;
        ctx->slot_nc = ctx->nc;
        ctx->m_alloc = m;
        ctx->geom_dirty = ctx->chg_dirty = true;
        ctx->have_solution = false;
        ctx->prev_solution = false;
        ctx->batch_dirty = true;
    }
    if (ctx->geom_dirty) {
        if (upload_geometry(ctx->slot, ctx->host_pos.data(), ctx->host_nrm.data(),
                            ctx->host_geo32.data(), ctx->stream))
            return fail(ctx, GABI_EDEVICE, "geometry upload failed");
        ctx->geom_dirty = false;
    }
    if (ctx->chg_dirty) {
        if (upload_charges(ctx->slot, ctx->host_charges.data(), ctx->stream))
            return fail(ctx, GABI_EDEVICE, "charge upload failed");
        ctx->chg_dirty = false;
    }
    slot_set_params(ctx->slot, ctx->eps1, ctx->eps2, ctx->kappa);
    return GABI_OK;
}

int sync_batch(gabi_ctx *ctx) {
    if (!ctx->batch_dirty && ctx->batch.d_mem &&
        std::memcmp(&ctx->uploaded, &ctx->slot.mol, sizeof(Mol)) == 0)
        return GABI_OK;  // descriptor unchanged: keep the batch and its graph
    ctx->batch.slots.assign(1, &ctx->slot);
    ctx->batch.mode = ctx->slot.mol.mode;
    std::string err;
    int rc = batch_build(ctx->batch, ctx->stream, err);
    if (rc) return fail(ctx, rc, err);
    ctx->uploaded = ctx->slot.mol;
    ctx->batch_dirty = false;
    return GABI_OK;
}

int require_state(gabi_ctx *ctx, bool need_charges) {
    if (!ctx) return GABI_EINVAL;
    if (ctx->n == 0) return fail(ctx, GABI_ESTATE, "surface not set");
    if (!ctx->params_set) return fail(ctx, GABI_ESTATE, "parameters not set");
    if (need_charges && !ctx->charges_set) return fail(ctx, GABI_ESTATE, "charges not set");
    return GABI_OK;
}

int prepare(gabi_ctx *ctx, bool need_charges, int m) {
    int rc = require_state(ctx, need_charges);
    if (rc) return rc;
    if ((rc = ensure_slot(ctx, m))) return rc;
    return sync_batch(ctx);
}

Timer make_timer(gabi_ctx *ctx) {
    Timer t;
    if (ctx->timing) {
        t.pending[0] = &ctx->pending[0];
        t.pending[1] = &ctx->pending[1];
    }
    return t;
}

int read_status(gabi_ctx *ctx) {
    enqueue_gather(ctx->batch, ctx->stream);
    GABI_HIP(ctx, hipGetLastError());
    GABI_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return GABI_OK;
}

}  // namespace

extern "C" {

void gabi_default_opts(gabi_solve_opts *o) {
    if (!o) return;
    o->restart = 20;
    o->maxit = 100;
    o->tol = 1e-6;
    o->mode = GABI_SOLVE_FP64;
    o->inner_tol = 3e-6;
    o->max_outer = 20;
    o->use_graph = 1;
    o->x0_previous = 0;
    o->tree_theta = 0.6;   // the refinement's inner products need ~1e-6 only:
    o->tree_degree = 4;    // at N = 327,680 these settings solve 10% faster
    o->tree_leaf = 128;    // than (0.7, 5, 256), with as many products
    o->tree_precision = GABI_FP32_PAIR;
}

int gabi_create(gabi_ctx **out, int device) {
    if (!out) return GABI_EINVAL;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) {
        (void)hipGetLastError();
        return GABI_EDEVICE;
    }
    if (hipSetDevice(device) != hipSuccess) return GABI_EDEVICE;
    gabi_ctx *ctx = new (std::nothrow) gabi_ctx();
    if (!ctx) return GABI_ENOMEM;
    ctx->device = device;
    if (hipStreamCreateWithFlags(&ctx->capture, hipStreamNonBlocking) != hipSuccess) {
        (void)hipGetLastError();
        ctx->capture = nullptr;  // graphs unavailable; rounds run eagerly
    }
    *out = ctx;
    return GABI_OK;
}

void gabi_destroy(gabi_ctx *ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    else (void)hipDeviceSynchronize();
    for (int p = 0; p < 3; ++p)
        for (auto &ev : ctx->pending[p]) {
            (void)hipEventDestroy(ev.first);
            (void)hipEventDestroy(ev.second);
        }
    batch_free(ctx->batch);
    free_slot(ctx);
    tree_free(ctx->tree);
    if (ctx->tree_u) (void)hipFree(ctx->tree_u);
    if (ctx->capture) (void)hipStreamDestroy(ctx->capture);
    delete ctx;
}

const char *gabi_last_error(const gabi_ctx *ctx) {
    return ctx ? ctx->err.c_str() : "null context";
}

int gabi_set_stream(gabi_ctx *ctx, void *stream) {
    if (!ctx) return GABI_EINVAL;
    ctx->stream = (hipStream_t)stream;
    return GABI_OK;
}

int gabi_mesh_elements(int64_t nv, const double *xyz, int64_t nf,
                       const int32_t *tri, double *cx, double *cy, double *cz,
                       double *nx, double *ny, double *nz, double *area) {
    if (nv < 3 || nf < 1 || !xyz || !tri || !cx || !cy || !cz || !nx || !ny ||
        !nz || !area)
        return GABI_EINVAL;
    for (int64_t f = 0; f < nf; ++f) {
        const int32_t ia = tri[3 * f], ib = tri[3 * f + 1], ic = tri[3 * f + 2];
        if (ia < 0 || ib < 0 || ic < 0 || ia >= nv || ib >= nv || ic >= nv)
            return GABI_EMESH;
        const double *a = xyz + 3 * (int64_t)ia, *b = xyz + 3 * (int64_t)ib,
                     *c = xyz + 3 * (int64_t)ic;
        const double e1x = b[0] - a[0], e1y = b[1] - a[1], e1z = b[2] - a[2];
        const double e2x = c[0] - a[0], e2y = c[1] - a[1], e2z = c[2] - a[2];
        const double px = e1y * e2z - e1z * e2y;
        const double py = e1z * e2x - e1x * e2z;
        const double pz = e1x * e2y - e1y * e2x;
        const double len = std::sqrt(px * px + py * py + pz * pz);
        if (!(len > 0.0) || !std::isfinite(len)) return GABI_EMESH;
        cx[f] = (a[0] + b[0] + c[0]) / 3.0;
        cy[f] = (a[1] + b[1] + c[1]) / 3.0;
        cz[f] = (a[2] + b[2] + c[2]) / 3.0;
        nx[f] = px / len;
        ny[f] = py / len;
        nz[f] = pz / len;
        area[f] = 0.5 * len;
    }
    return GABI_OK;
}

int gabi_set_surface(gabi_ctx *ctx, int64_t n, const double *cx,
                     const double *cy, const double *cz, const double *nx,
                     const double *ny, const double *nz, const double *area) {
    if (!ctx) return GABI_EINVAL;
    std::string msg;
    int rc = validate_surface(n, cx, cy, cz, nx, ny, nz, area, msg);
    if (rc) return fail(ctx, rc, msg);
    if (ctx->nc > 0) {
        const double *q = ctx->host_charges.data();
        std::vector<double> px(ctx->nc), py(ctx->nc), pz(ctx->nc);
        for (int64_t k = 0; k < ctx->nc; ++k) {
            px[k] = q[4 * k];
            py[k] = q[4 * k + 1];
            pz[k] = q[4 * k + 2];
        }
        rc = check_charges_vs_centroids(n, cx, cy, cz, ctx->nc, px.data(), py.data(),
                                        pz.data(), msg);
        if (rc) return fail(ctx, rc, msg);
    }
    stage_surface(n, cx, cy, cz, nx, ny, nz, area, ctx->host_pos, ctx->host_nrm,
                  ctx->host_geo32);
    ctx->host_centroids.resize((size_t)(3 * n));
    for (int64_t i = 0; i < n; ++i) {
        ctx->host_centroids[3 * i] = cx[i];
        ctx->host_centroids[3 * i + 1] = cy[i];
        ctx->host_centroids[3 * i + 2] = cz[i];
    }
    ctx->n = n;
    ctx->geom_dirty = true;
    ctx->geom_version++;
    ctx->have_solution = false;
    return GABI_OK;
}

int gabi_set_surface_mesh(gabi_ctx *ctx, int64_t nv, const double *xyz,
                          int64_t nf, const int32_t *tri) {
    if (!ctx) return GABI_EINVAL;
    if (nf < 4) return fail(ctx, GABI_EMESH, "a closed surface needs at least 4 elements");
    std::vector<double> a((size_t)(7 * nf));
    double *p = a.data();
    int rc = gabi_mesh_elements(nv, xyz, nf, tri, p, p + nf, p + 2 * nf, p + 3 * nf,
                                p + 4 * nf, p + 5 * nf, p + 6 * nf);
    if (rc == GABI_EINVAL) return fail(ctx, rc, "bad mesh arguments");
    if (rc == GABI_EMESH)
        return fail(ctx, rc, "mesh has an out-of-range vertex index or a zero-area triangle");
    return gabi_set_surface(ctx, nf, p, p + nf, p + 2 * nf, p + 3 * nf, p + 4 * nf,
                            p + 5 * nf, p + 6 * nf);
}

int gabi_set_charges(gabi_ctx *ctx, int64_t nc, const double *px,
                     const double *py, const double *pz, const double *q) {
    if (!ctx) return GABI_EINVAL;
    std::string msg;
    int rc = validate_charges(nc, px, py, pz, q, msg);
    if (rc) return fail(ctx, rc, msg);
    if (ctx->n > 0 && nc > 0) {
        const double *c = ctx->host_centroids.data();  // x, y, z per element
        rc = charges_on_centroids(ctx->n, c, c + 1, c + 2, 3, nc, px, py, pz, msg);
        if (rc) return fail(ctx, rc, msg);
    }
    ctx->host_charges.resize((size_t)(4 * nc));
    for (int64_t k = 0; k < nc; ++k) {
        ctx->host_charges[4 * k] = px[k];
        ctx->host_charges[4 * k + 1] = py[k];
        ctx->host_charges[4 * k + 2] = pz[k];
        ctx->host_charges[4 * k + 3] = q[k];
    }
    ctx->nc = nc;
    ctx->charges_set = true;
    ctx->chg_dirty = true;
    ctx->have_solution = false;
    return GABI_OK;
}

int gabi_set_params(gabi_ctx *ctx, double eps1, double eps2, double kappa) {
    if (!ctx) return GABI_EINVAL;
    if (!params_valid(eps1, eps2, kappa))
        return fail(ctx, GABI_EINVAL, "need eps1 > 0, eps2 > 0, kappa >= 0, all finite");
    ctx->eps1 = eps1;
    ctx->eps2 = eps2;
    ctx->kappa = kappa;
    ctx->params_set = true;
    ctx->have_solution = false;
    return GABI_OK;
}

int gabi_rhs_dev(gabi_ctx *ctx, double *b_dev) {
    int rc = prepare(ctx, true, 0);
    if (rc) return rc;
    if (!b_dev) return fail(ctx, GABI_EINVAL, "null output");
    launch_rhs(ctx->batch, ctx->stream);
    GABI_HIP(ctx, hipMemcpyAsync(b_dev, ctx->slot.mol.rhs_dst, sizeof(double) * 2 * ctx->n,
                                 hipMemcpyDeviceToDevice, ctx->stream));
    GABI_HIP(ctx, hipGetLastError());
    return GABI_OK;
}

int gabi_rhs(gabi_ctx *ctx, double *b) {
    int rc = prepare(ctx, true, 0);
    if (rc) return rc;
    if (!b) return fail(ctx, GABI_EINVAL, "null output");
    launch_rhs(ctx->batch, ctx->stream);
    GABI_HIP(ctx, hipGetLastError());
    GABI_HIP(ctx, hipMemcpyAsync(b, ctx->slot.mol.rhs_dst, sizeof(double) * 2 * ctx->n,
                                 hipMemcpyDeviceToHost, ctx->stream));
    GABI_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return GABI_OK;
}

static int matvec_impl(gabi_ctx *ctx, int precision, const void *u, double *y,
                       hipMemcpyKind in_kind, hipMemcpyKind out_kind) {
    int rc = prepare(ctx, false, 0);
    if (rc) return rc;
    if (precision != GABI_FP64 && precision != GABI_FP32_PAIR)
        return fail(ctx, GABI_EINVAL, "unknown precision");
    if (!u || !y) return fail(ctx, GABI_EINVAL, "null vector");
    const size_t bytes = sizeof(double) * 2 * ctx->n;
    GABI_HIP(ctx, hipMemcpyAsync(ctx->slot.mol.u, u, bytes, in_kind, ctx->stream));
    Timer t = make_timer(ctx);
    launch_prep(ctx->batch, ctx->stream, precision, kPrepU, 0, false);
    launch_pair(ctx->batch, ctx->stream, precision, false, &t);
    launch_finish(ctx->batch, ctx->stream, precision, kFinishY, 0, false);
    GABI_HIP(ctx, hipGetLastError());
    GABI_HIP(ctx, hipMemcpyAsync(y, ctx->slot.mol.y, bytes, out_kind, ctx->stream));
    if (out_kind == hipMemcpyDeviceToHost) GABI_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return GABI_OK;
}

int gabi_matvec_dev(gabi_ctx *ctx, int precision, const double *u_dev, double *y_dev) {
    return matvec_impl(ctx, precision, u_dev, y_dev, hipMemcpyDeviceToDevice,
                       hipMemcpyDeviceToDevice);
}

int gabi_matvec(gabi_ctx *ctx, int precision, const double *u, double *y) {
    return matvec_impl(ctx, precision, u, y, hipMemcpyHostToDevice, hipMemcpyDeviceToHost);
}

static int solve_impl(gabi_ctx *ctx, const gabi_solve_opts *opts, const void *x0,
                      hipMemcpyKind x0_kind, double *u, hipMemcpyKind u_kind,
                      gabi_solve_info *info) {
    const auto t0 = std::chrono::steady_clock::now();
    gabi_solve_opts o;
    std::string msg;
    int rc = require_state(ctx, true);
    if (rc) return rc;
    if ((rc = opts_check(opts, &o, msg))) return fail(ctx, rc, msg);
    if ((rc = ensure_slot(ctx, o.restart))) return rc;
    Slot &sl = ctx->slot;
    const bool tree = o.mode == GABI_SOLVE_TREE_IR;
    // the treecode refinement runs the mixed solver's rounds with treecode
    // cycle products
    const int mode = o.mode == GABI_SOLVE_FP64 ? kModeFP64 : kModeMixed;
    slot_set_mode(sl, mode);
    set_solve_targets(sl, o.tol, o.inner_tol, o.maxit);
    sl.mol.m = o.restart;
    if (tree) {
        const gabi_tree_opts to{o.tree_theta, o.tree_degree, o.tree_leaf, o.tree_precision, 0};
        if ((rc = tree_for_solve(ctx, &to))) return rc;
    }
    if ((rc = sync_batch(ctx))) return rc;
    Batch &b = ctx->batch;
    {
        // a round captured with other cycle products (or another tree) is
        // recorded again
        const TreeState *tr = tree ? ctx->tree : nullptr;
        const int64_t gen = tr ? tree_generation(*tr) : -1;
        const bool f32 = tree && o.tree_precision == GABI_FP32_PAIR;
        if (b.tree != tr || b.tree_gen != gen || b.tree_f32 != f32) {
            release_graph(b);
            b.tree = tr;
            b.tree_gen = gen;
            b.tree_f32 = f32;
        }
    }
    Timer t = make_timer(ctx);
    const bool graph = o.use_graph != 0;
    const size_t bytes = sizeof(double) * 2 * ctx->n;
    // the previous solution is still in the slot's solution buffer: nothing
    // but a solve writes it, and a new slot clears prev_solution
    const bool previous = !x0 && o.x0_previous && ctx->prev_solution;
    if (x0)
        GABI_HIP(ctx, hipMemcpyAsync(sl.mol.res_x, x0, bytes, x0_kind, ctx->stream));
    else if (previous)
        GABI_HIP(ctx, hipMemcpyAsync(sl.mol.res_x, sl.mol.sol, bytes, hipMemcpyDeviceToDevice,
                                     ctx->stream));
    const bool warm = x0 != nullptr || previous;
    enqueue_init(b, ctx->stream, warm, &t);
    if ((rc = read_status(ctx))) return rc;
    int rounds = 0;
    for (;;) {
        const KrylovStatus &st = b.h_status[0];
        if (st.converged || st.iters >= st.maxit) break;
        if (mode == kModeMixed && rounds >= o.max_outer) break;
        if ((rc = run_round(b, ctx->stream, ctx->capture, &t, graph, msg)))
            return fail(ctx, rc, msg);
        if ((rc = read_status(ctx))) return rc;
        if (graph && ctx->timing) graph_round_times(b, ctx->total_ms, ctx->count);
        ++rounds;
    }
    enqueue_finalize(b, ctx->stream);  // solution to sol, reaction potential, energy
    if (u) GABI_HIP(ctx, hipMemcpyAsync(u, sl.mol.sol, bytes, u_kind, ctx->stream));
    if ((rc = read_status(ctx))) return rc;
    const KrylovStatus &st = b.h_status[0];
    gabi_solve_info out{};
    out.iterations = st.iters;
    out.restarts = rounds;
    const int64_t extra = warm ? 1 : 0;
    if (mode == kModeMixed) {
        (tree ? out.matvecs_tree : out.matvecs_fp32) = st.iters;
        out.matvecs_fp64 = rounds + extra;
        out.outer = rounds;
    } else {
        out.matvecs_fp64 = st.iters + rounds + extra;
    }
    out.rel_residual = st.beta0 > 0 ? st.rnorm / st.beta0 : 0.0;
    out.converged = st.converged;
    out.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    out.warm_start = warm ? 1 : 0;
    if (info) *info = out;
    ctx->have_solution = true;
    ctx->solution_energy = st.energy;  // enqueue_finalize evaluated it
    ctx->solution_energy_valid = true;
    ctx->prev_solution = true;
    return out.converged ? GABI_OK : GABI_NOT_CONVERGED;
}

int gabi_solve_dev(gabi_ctx *ctx, const gabi_solve_opts *opts,
                   const double *x0_dev, double *u_dev, gabi_solve_info *info) {
    return solve_impl(ctx, opts, x0_dev, hipMemcpyDeviceToDevice, u_dev,
                      hipMemcpyDeviceToDevice, info);
}

int gabi_solve(gabi_ctx *ctx, const gabi_solve_opts *opts, const double *x0,
               double *u, gabi_solve_info *info) {
    return solve_impl(ctx, opts, x0, hipMemcpyHostToDevice, u, hipMemcpyDeviceToHost, info);
}

static int energy_impl(gabi_ctx *ctx, const void *u, hipMemcpyKind kind, double *e,
                       double *phi_host) {
    int rc = prepare(ctx, true, 0);
    if (rc) return rc;
    if (!u && ctx->have_solution && ctx->solution_energy_valid) {
        // the solve's final step left E and phi_reac of its solution
        if (phi_host && ctx->nc) {
            GABI_HIP(ctx, hipMemcpyAsync(phi_host, ctx->slot.mol.phi, sizeof(double) * ctx->nc,
                                         hipMemcpyDeviceToHost, ctx->stream));
            GABI_HIP(ctx, hipStreamSynchronize(ctx->stream));
        }
        if (e) *e = ctx->solution_energy;
        return GABI_OK;
    }
    if (u) {
        ctx->solution_energy_valid = false;  // phi_reac and E now belong to u
        GABI_HIP(ctx, hipMemcpyAsync(ctx->slot.mol.u, u, sizeof(double) * 2 * ctx->n, kind,
                                     ctx->stream));
    } else if (!ctx->have_solution) {
        return fail(ctx, GABI_ESTATE, "no solution to evaluate");
    }
    launch_reaction(ctx->batch, ctx->stream, u == nullptr);
    if (phi_host && ctx->nc)
        GABI_HIP(ctx, hipMemcpyAsync(phi_host, ctx->slot.mol.phi, sizeof(double) * ctx->nc,
                                     hipMemcpyDeviceToHost, ctx->stream));
    if ((rc = read_status(ctx))) return rc;
    if (e) *e = ctx->batch.h_status[0].energy;
    if (!u) {
        ctx->solution_energy = ctx->batch.h_status[0].energy;
        ctx->solution_energy_valid = true;
    }
    return GABI_OK;
}

int gabi_energy_dev(gabi_ctx *ctx, const double *u_dev, double *e) {
    if (ctx && !e) return fail(ctx, GABI_EINVAL, "null output");
    return energy_impl(ctx, u_dev, hipMemcpyDeviceToDevice, e, nullptr);
}

int gabi_energy(gabi_ctx *ctx, const double *u, double *e) {
    if (ctx && !e) return fail(ctx, GABI_EINVAL, "null output");
    return energy_impl(ctx, u, hipMemcpyHostToDevice, e, nullptr);
}

int gabi_reaction_potential(gabi_ctx *ctx, const double *u, double *phi) {
    if (ctx && !phi && ctx->nc) return fail(ctx, GABI_EINVAL, "null output");
    return energy_impl(ctx, u, hipMemcpyHostToDevice, nullptr, phi);
}

int64_t gabi_device_bytes(const gabi_ctx *ctx) {
    return ctx ? ctx->slot.bytes + ctx->batch.cap_bytes : 0;
}

int gabi_set_kernel_timing(gabi_ctx *ctx, int enable) {
    if (!ctx) return GABI_EINVAL;
    ctx->timing = enable != 0;
    return GABI_OK;
}

int gabi_kernel_time(gabi_ctx *ctx, int precision, double *avg_ms,
                     int64_t *count, int reset) {
    if (!ctx) return GABI_EINVAL;
    if (precision != GABI_FP64 && precision != GABI_FP32_PAIR && precision != GABI_TIMING_TREE)
        return fail(ctx, GABI_EINVAL, "unknown precision");
    const int p = precision == GABI_FP64 ? 0 : precision == GABI_FP32_PAIR ? 1 : 2;
    for (auto &ev : ctx->pending[p]) {
        GABI_HIP(ctx, hipEventSynchronize(ev.second));
        float ms = 0.0f;
        GABI_HIP(ctx, hipEventElapsedTime(&ms, ev.first, ev.second));
        ctx->total_ms[p] += ms;
        ctx->count[p] += 1;
        (void)hipEventDestroy(ev.first);
        (void)hipEventDestroy(ev.second);
    }
    ctx->pending[p].clear();
    if (avg_ms) *avg_ms = ctx->count[p] ? ctx->total_ms[p] / (double)ctx->count[p] : 0.0;
    if (count) *count = ctx->count[p];
    if (reset) {
        ctx->total_ms[p] = 0.0;
        ctx->count[p] = 0;
    }
    return GABI_OK;
}

}  // extern "C"
