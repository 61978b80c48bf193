// C ABI of libgabi (declared in include/gabi.h): contexts, validation of the
// element and charge data, device buffers, and the host/device entry points
// around the kernels.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <unordered_set>

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

int dev_alloc(gabi_ctx *ctx, void **p, size_t bytes) {
    *p = nullptr;
    if (bytes == 0) bytes = 8;
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return fail(ctx, GABI_ENOMEM,
                    "device allocation of " + std::to_string(bytes) + " bytes failed: " +
                        hipGetErrorString(e));
    }
    ctx->bytes += (int64_t)bytes;
    return GABI_OK;
}

void dev_free(gabi_ctx *ctx, void **p, size_t bytes) {
    if (*p) {
        (void)hipFree(*p);
        ctx->bytes -= (int64_t)(bytes == 0 ? 8 : bytes);
    }
    *p = nullptr;
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

int use_device(gabi_ctx *ctx) {
    GABI_HIP(ctx, hipSetDevice(ctx->device));
    return GABI_OK;
}

// A charge exactly on a centroid makes a source term singular.
int check_charges_vs_surface(gabi_ctx *ctx) {
    if (ctx->n == 0 || ctx->nc == 0) return GABI_OK;
    std::unordered_set<Key, KeyHash> cent;
    cent.reserve((size_t)ctx->n * 2);
    const double *c = ctx->host_centroids.data();
    for (int64_t i = 0; i < ctx->n; ++i) cent.insert(Key{c[3 * i], c[3 * i + 1], c[3 * i + 2]});
    const double *q = ctx->host_charges.data();
    for (int64_t k = 0; k < ctx->nc; ++k) {
        if (cent.count(Key{q[4 * k], q[4 * k + 1], q[4 * k + 2]}))
            return fail(ctx, GABI_EINVAL,
                        "charge " + std::to_string(k) + " lies exactly on an element centroid");
    }
    return GABI_OK;
}

void free_surface(gabi_ctx *ctx) {
    const int64_t n = ctx->n, len = 2 * n;
    dev_free(ctx, (void **)&ctx->pos, sizeof(double4) * n);
    dev_free(ctx, (void **)&ctx->nrm, sizeof(double4) * n);
    dev_free(ctx, (void **)&ctx->nrm32, sizeof(float4) * n);
    dev_free(ctx, (void **)&ctx->wgt, sizeof(double4) * n);
    dev_free(ctx, (void **)&ctx->wgt32, sizeof(float4) * n);
    dev_free(ctx, (void **)&ctx->part, sizeof(double) * ctx->part_len);
    ctx->part_len = 0;
    dev_free(ctx, (void **)&ctx->vec_u, sizeof(double) * len);
    dev_free(ctx, (void **)&ctx->vec_y, sizeof(double) * len);
    dev_free(ctx, (void **)&ctx->vec_b, sizeof(double) * len);
    dev_free(ctx, (void **)&ctx->vec_in, sizeof(double) * len);
    if (ctx->V) {
        const int m = ctx->kry_m;
        dev_free(ctx, (void **)&ctx->V, sizeof(double) * len * (m + 1));
        dev_free(ctx, (void **)&ctx->H, sizeof(double) * (m + 1) * m);
        dev_free(ctx, (void **)&ctx->givens, sizeof(double) * (4 * m + 1));
        ctx->kry_m = 0;
    }
    double **vs[] = {&ctx->gm_b, &ctx->gm_x, &ctx->gm_r, &ctx->gm_w, &ctx->ir_x, &ctx->ir_r};
    for (double **p : vs) dev_free(ctx, (void **)p, sizeof(double) * len);
    ctx->n = 0;
    ctx->have_solution = false;
    ctx->host_centroids.clear();
}

void free_charges(gabi_ctx *ctx) {
    dev_free(ctx, (void **)&ctx->chg, sizeof(double4) * ctx->nc);
    dev_free(ctx, (void **)&ctx->phi_dev, sizeof(double) * ctx->nc);
    dev_free(ctx, (void **)&ctx->phi_part, sizeof(double) * ctx->phi_part_len);
    ctx->phi_part_len = 0;
    ctx->nc = 0;
    ctx->host_charges.clear();
}

int require_state(gabi_ctx *ctx, bool need_charges) {
    if (!ctx) return GABI_EINVAL;
    if (ctx->n == 0) return fail(ctx, GABI_ESTATE, "surface not set");
    if (!ctx->params_set) return fail(ctx, GABI_ESTATE, "parameters not set");
    if (need_charges && !ctx->charges_set) return fail(ctx, GABI_ESTATE, "charges not set");
    return use_device(ctx);
}

bool is_finite(double v) { return std::isfinite(v); }

}  // namespace

extern "C" {

void gabi_default_opts(gabi_solve_opts *o) {
    if (!o) return;
    o->restart = 10;
    o->maxit = 100;
    o->tol = 1e-6;
    o->mode = GABI_SOLVE_FP64;
    o->inner_tol = 1e-5;
    o->max_outer = 10;
    o->use_graph = 1;
}

int gabi_create(gabi_ctx **out, int device) {
    if (!out) return GABI_EINVAL;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) {
        (void)hipGetLastError();
        return GABI_EDEVICE;
    }
    gabi_ctx *ctx = new (std::nothrow) gabi_ctx();
    if (!ctx) return GABI_ENOMEM;
    ctx->device = device;
    if (hipSetDevice(device) != hipSuccess) {
        delete ctx;
        return GABI_EDEVICE;
    }
    if (dev_alloc(ctx, (void **)&ctx->red, sizeof(double) * 2 * kBlasBlocksMax) ||
        dev_alloc(ctx, (void **)&ctx->scalars, sizeof(double) * 16)) {
        gabi_destroy(ctx);
        return GABI_ENOMEM;
    }
    *out = ctx;
    return GABI_OK;
}

void gabi_destroy(gabi_ctx *ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    else (void)hipDeviceSynchronize();
    for (int p = 0; p < 2; ++p)
        for (auto &ev : ctx->timing.pending[p]) {
            (void)hipEventDestroy(ev.first);
            (void)hipEventDestroy(ev.second);
        }
    free_surface(ctx);
    free_charges(ctx);
    dev_free(ctx, (void **)&ctx->red, 0);
    dev_free(ctx, (void **)&ctx->scalars, 0);
    dev_free(ctx, (void **)&ctx->status, 0);
    if (ctx->status_host) (void)hipHostFree(ctx->status_host);
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
    if (!cx || !cy || !cz || !nx || !ny || !nz || !area)
        return fail(ctx, GABI_EINVAL, "null surface array");
    if (n < 4) return fail(ctx, GABI_EMESH, "a closed surface needs at least 4 elements");
    if (n > (int64_t)INT32_MAX / 2)
        return fail(ctx, GABI_EINVAL, "too many elements");
    for (int64_t i = 0; i < n; ++i) {
        if (!is_finite(cx[i]) || !is_finite(cy[i]) || !is_finite(cz[i]) || !is_finite(nx[i]) ||
            !is_finite(ny[i]) || !is_finite(nz[i]) || !is_finite(area[i]))
            return fail(ctx, GABI_EMESH, "non-finite element data at " + std::to_string(i));
        if (!(area[i] > 0.0))
            return fail(ctx, GABI_EMESH, "element " + std::to_string(i) + " has area <= 0");
        const double nn = std::sqrt(nx[i] * nx[i] + ny[i] * ny[i] + nz[i] * nz[i]);
        if (std::fabs(nn - 1.0) > 1e-6)
            return fail(ctx, GABI_EMESH, "normal of element " + std::to_string(i) + " is not unit");
    }
    {   // duplicate centroids: lexicographic sort, compare neighbours
        std::vector<int64_t> idx((size_t)n);
        std::iota(idx.begin(), idx.end(), (int64_t)0);
        std::sort(idx.begin(), idx.end(), [&](int64_t a, int64_t b) {
            if (cx[a] != cx[b]) return cx[a] < cx[b];
            if (cy[a] != cy[b]) return cy[a] < cy[b];
            return cz[a] < cz[b];
        });
        for (int64_t t = 1; t < n; ++t) {
            const int64_t a = idx[t - 1], b = idx[t];
            if (cx[a] == cx[b] && cy[a] == cy[b] && cz[a] == cz[b])
                return fail(ctx, GABI_EMESH, "elements " + std::to_string(a) + " and " +
                                                 std::to_string(b) + " share a centroid");
        }
    }
    std::vector<double> cent((size_t)(3 * n));
    for (int64_t i = 0; i < n; ++i) {
        cent[3 * i] = cx[i];
        cent[3 * i + 1] = cy[i];
        cent[3 * i + 2] = cz[i];
    }
    if (ctx->nc > 0) {
        std::swap(ctx->host_centroids, cent);
        const int64_t keep = ctx->n;
        ctx->n = n;
        int rc = check_charges_vs_surface(ctx);
        ctx->n = keep;
        std::swap(ctx->host_centroids, cent);
        if (rc) return rc;
    }
    int rc = use_device(ctx);
    if (rc) return rc;

    // host staging in the device layout
    std::vector<double4> hp((size_t)n), hn((size_t)n);
    std::vector<float4> hn32((size_t)n);
    for (int64_t i = 0; i < n; ++i) {
        hp[i] = make_double4(cx[i], cy[i], cz[i], area[i]);
        hn[i] = make_double4(nx[i], ny[i], nz[i], 0.0);
        hn32[i] = make_float4((float)nx[i], (float)ny[i], (float)nz[i], 0.0f);
    }
    if (ctx->stream) GABI_HIP(ctx, hipStreamSynchronize(ctx->stream));
    free_surface(ctx);
    const int64_t len = 2 * n;
    const PairLaunch L64 = pair_launch(n, GABI_FP64), L32 = pair_launch(n, GABI_FP32_PAIR);
    const int64_t part_len = 2 * n * (int64_t)std::max(L64.splits, L32.splits);
    if ((rc = dev_alloc(ctx, (void **)&ctx->pos, sizeof(double4) * n)) ||
        (rc = dev_alloc(ctx, (void **)&ctx->nrm, sizeof(double4) * n)) ||
        (rc = dev_alloc(ctx, (void **)&ctx->nrm32, sizeof(float4) * n)) ||
        (rc = dev_alloc(ctx, (void **)&ctx->wgt, sizeof(double4) * n)) ||
        (rc = dev_alloc(ctx, (void **)&ctx->wgt32, sizeof(float4) * n)) ||
        (rc = dev_alloc(ctx, (void **)&ctx->part, sizeof(double) * part_len)) ||
        (rc = dev_alloc(ctx, (void **)&ctx->vec_u, sizeof(double) * len)) ||
        (rc = dev_alloc(ctx, (void **)&ctx->vec_y, sizeof(double) * len)) ||
        (rc = dev_alloc(ctx, (void **)&ctx->vec_b, sizeof(double) * len)) ||
        (rc = dev_alloc(ctx, (void **)&ctx->vec_in, sizeof(double) * len))) {
        ctx->n = n;  // so that free_surface releases what was allocated
        ctx->part_len = part_len;
        free_surface(ctx);
        return rc;
    }
    ctx->n = n;
    ctx->part_len = part_len;
    GABI_HIP(ctx, hipMemcpy(ctx->pos, hp.data(), sizeof(double4) * n, hipMemcpyHostToDevice));
    GABI_HIP(ctx, hipMemcpy(ctx->nrm, hn.data(), sizeof(double4) * n, hipMemcpyHostToDevice));
    GABI_HIP(ctx, hipMemcpy(ctx->nrm32, hn32.data(), sizeof(float4) * n, hipMemcpyHostToDevice));
    ctx->host_centroids.swap(cent);
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
    if (nc < 0) return fail(ctx, GABI_EINVAL, "negative charge count");
    if (nc > 0 && (!px || !py || !pz || !q)) return fail(ctx, GABI_EINVAL, "null charge array");
    if (nc > (int64_t)INT32_MAX / 2) return fail(ctx, GABI_EINVAL, "too many charges");
    std::vector<double> h((size_t)(4 * nc));
    for (int64_t k = 0; k < nc; ++k) {
        if (!is_finite(px[k]) || !is_finite(py[k]) || !is_finite(pz[k]) || !is_finite(q[k]))
            return fail(ctx, GABI_EINVAL, "non-finite charge data at " + std::to_string(k));
        h[4 * k] = px[k];
        h[4 * k + 1] = py[k];
        h[4 * k + 2] = pz[k];
        h[4 * k + 3] = q[k];
    }
    if (ctx->n > 0 && nc > 0) {
        std::swap(ctx->host_charges, h);
        const int64_t keep = ctx->nc;
        ctx->nc = nc;
        int rc = check_charges_vs_surface(ctx);
        ctx->nc = keep;
        std::swap(ctx->host_charges, h);
        if (rc) return rc;
    }
    int rc = use_device(ctx);
    if (rc) return rc;
    if (ctx->stream) GABI_HIP(ctx, hipStreamSynchronize(ctx->stream));
    free_charges(ctx);
    if (nc > 0) {
        if ((rc = dev_alloc(ctx, (void **)&ctx->chg, sizeof(double4) * nc)) ||
            (rc = dev_alloc(ctx, (void **)&ctx->phi_dev, sizeof(double) * nc))) {
            ctx->nc = nc;
            free_charges(ctx);
            return rc;
        }
        GABI_HIP(ctx, hipMemcpy(ctx->chg, h.data(), sizeof(double4) * nc, hipMemcpyHostToDevice));
    }
    ctx->nc = nc;
    ctx->host_charges.swap(h);
    ctx->charges_set = true;
    ctx->have_solution = false;
    return GABI_OK;
}

int gabi_set_params(gabi_ctx *ctx, double eps1, double eps2, double kappa) {
    if (!ctx) return GABI_EINVAL;
    if (!(eps1 > 0.0) || !(eps2 > 0.0) || !(kappa >= 0.0) || !is_finite(eps1) ||
        !is_finite(eps2) || !is_finite(kappa))
        return fail(ctx, GABI_EINVAL, "need eps1 > 0, eps2 > 0, kappa >= 0, all finite");
    ctx->eps1 = eps1;
    ctx->eps2 = eps2;
    ctx->kappa = kappa;
    ctx->params_set = true;
    ctx->have_solution = false;
    return GABI_OK;
}

int gabi_rhs_dev(gabi_ctx *ctx, double *b_dev) {
    int rc = require_state(ctx, true);
    if (rc) return rc;
    if (!b_dev) return fail(ctx, GABI_EINVAL, "null output");
    launch_rhs(ctx, b_dev);
    GABI_HIP(ctx, hipGetLastError());
    return GABI_OK;
}

int gabi_rhs(gabi_ctx *ctx, double *b) {
    int rc = require_state(ctx, true);
    if (rc) return rc;
    if (!b) return fail(ctx, GABI_EINVAL, "null output");
    launch_rhs(ctx, ctx->vec_y);
    GABI_HIP(ctx, hipGetLastError());
    GABI_HIP(ctx, hipMemcpyAsync(b, ctx->vec_y, sizeof(double) * 2 * ctx->n,
                                 hipMemcpyDeviceToHost, ctx->stream));
    GABI_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return GABI_OK;
}

int gabi_matvec_dev(gabi_ctx *ctx, int precision, const double *u_dev,
                    double *y_dev) {
    int rc = require_state(ctx, false);
    if (rc) return rc;
    if (precision != GABI_FP64 && precision != GABI_FP32_PAIR)
        return fail(ctx, GABI_EINVAL, "unknown precision");
    if (!u_dev || !y_dev) return fail(ctx, GABI_EINVAL, "null vector");
    return matvec_device(ctx, precision, u_dev, y_dev);
}

int gabi_matvec(gabi_ctx *ctx, int precision, const double *u, double *y) {
    int rc = require_state(ctx, false);
    if (rc) return rc;
    if (!u || !y) return fail(ctx, GABI_EINVAL, "null vector");
    const size_t bytes = sizeof(double) * 2 * ctx->n;
    GABI_HIP(ctx, hipMemcpyAsync(ctx->vec_in, u, bytes, hipMemcpyHostToDevice, ctx->stream));
    if ((rc = gabi_matvec_dev(ctx, precision, ctx->vec_in, ctx->vec_y))) return rc;
    GABI_HIP(ctx, hipMemcpyAsync(y, ctx->vec_y, bytes, hipMemcpyDeviceToHost, ctx->stream));
    GABI_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return GABI_OK;
}

static int check_opts(gabi_ctx *ctx, const gabi_solve_opts *in, gabi_solve_opts *o) {
    gabi_default_opts(o);
    if (in) *o = *in;
    if (o->restart < 1 || o->restart > 64)
        return fail(ctx, GABI_EINVAL, "restart must be in [1, 64]");
    if (o->maxit < 0) return fail(ctx, GABI_EINVAL, "maxit must be >= 0");
    if (!(o->tol > 0.0) || !is_finite(o->tol)) return fail(ctx, GABI_EINVAL, "tol must be > 0");
    if (o->mode != GABI_SOLVE_FP64 && o->mode != GABI_SOLVE_MIXED_IR)
        return fail(ctx, GABI_EINVAL, "unknown solve mode");
    if (o->mode == GABI_SOLVE_MIXED_IR &&
        (!(o->inner_tol > 0.0) || !(o->inner_tol < 1.0) || o->max_outer < 1))
        return fail(ctx, GABI_EINVAL, "need 0 < inner_tol < 1 and max_outer >= 1");
    return GABI_OK;
}

int gabi_solve_dev(gabi_ctx *ctx, const gabi_solve_opts *opts,
                   const double *x0_dev, double *u_dev, gabi_solve_info *info) {
    int rc = require_state(ctx, true);
    if (rc) return rc;
    gabi_solve_opts o;
    if ((rc = check_opts(ctx, opts, &o))) return rc;
    return solve_device(ctx, o, x0_dev, u_dev, info);
}

int gabi_solve(gabi_ctx *ctx, const gabi_solve_opts *opts, const double *x0,
               double *u, gabi_solve_info *info) {
    int rc = require_state(ctx, true);
    if (rc) return rc;
    gabi_solve_opts o;
    if ((rc = check_opts(ctx, opts, &o))) return rc;
    const size_t bytes = sizeof(double) * 2 * ctx->n;
    if (x0)
        GABI_HIP(ctx, hipMemcpyAsync(ctx->vec_in, x0, bytes, hipMemcpyHostToDevice, ctx->stream));
    rc = solve_device(ctx, o, x0 ? ctx->vec_in : nullptr, nullptr, info);
    if (rc < 0) return rc;
    if (u) {
        GABI_HIP(ctx, hipMemcpyAsync(u, ctx->vec_u, bytes, hipMemcpyDeviceToHost, ctx->stream));
        GABI_HIP(ctx, hipStreamSynchronize(ctx->stream));
    }
    return rc;
}

static int energy_impl(gabi_ctx *ctx, const double *u_dev, double *e, double *phi_host) {
    if (!u_dev) {
        if (!ctx->have_solution) return fail(ctx, GABI_ESTATE, "no solution to evaluate");
        u_dev = ctx->vec_u;
    }
    launch_prep(ctx, GABI_FP64, u_dev, nullptr, nullptr, nullptr);
    int rc = launch_reaction(ctx, ctx->nc ? ctx->phi_dev : nullptr, ctx->scalars);
    if (rc) return rc;
    if (e)
        GABI_HIP(ctx, hipMemcpyAsync(e, ctx->scalars, sizeof(double), hipMemcpyDeviceToHost,
                                     ctx->stream));
    if (phi_host && ctx->nc)
        GABI_HIP(ctx, hipMemcpyAsync(phi_host, ctx->phi_dev, sizeof(double) * ctx->nc,
                                     hipMemcpyDeviceToHost, ctx->stream));
    GABI_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return GABI_OK;
}

int gabi_energy_dev(gabi_ctx *ctx, const double *u_dev, double *e) {
    int rc = require_state(ctx, true);
    if (rc) return rc;
    if (!e) return fail(ctx, GABI_EINVAL, "null output");
    return energy_impl(ctx, u_dev, e, nullptr);
}

int gabi_energy(gabi_ctx *ctx, const double *u, double *e) {
    int rc = require_state(ctx, true);
    if (rc) return rc;
    if (!e) return fail(ctx, GABI_EINVAL, "null output");
    if (u)
        GABI_HIP(ctx, hipMemcpyAsync(ctx->vec_in, u, sizeof(double) * 2 * ctx->n,
                                     hipMemcpyHostToDevice, ctx->stream));
    return energy_impl(ctx, u ? ctx->vec_in : nullptr, e, nullptr);
}

int gabi_reaction_potential(gabi_ctx *ctx, const double *u, double *phi) {
    int rc = require_state(ctx, true);
    if (rc) return rc;
    if (!phi && ctx->nc) return fail(ctx, GABI_EINVAL, "null output");
    if (u)
        GABI_HIP(ctx, hipMemcpyAsync(ctx->vec_in, u, sizeof(double) * 2 * ctx->n,
                                     hipMemcpyHostToDevice, ctx->stream));
    return energy_impl(ctx, u ? ctx->vec_in : nullptr, nullptr, phi);
}

int64_t gabi_device_bytes(const gabi_ctx *ctx) { return ctx ? ctx->bytes : 0; }

int gabi_set_kernel_timing(gabi_ctx *ctx, int enable) {
    if (!ctx) return GABI_EINVAL;
    ctx->timing.enabled = enable != 0;
    return GABI_OK;
}

int gabi_kernel_time(gabi_ctx *ctx, int precision, double *avg_ms,
                     int64_t *count, int reset) {
    if (!ctx) return GABI_EINVAL;
    if (precision != GABI_FP64 && precision != GABI_FP32_PAIR)
        return fail(ctx, GABI_EINVAL, "unknown precision");
    const int p = precision == GABI_FP64 ? 0 : 1;
    Timing &t = ctx->timing;
    for (auto &ev : t.pending[p]) {
        GABI_HIP(ctx, hipEventSynchronize(ev.second));
        float ms = 0.0f;
        GABI_HIP(ctx, hipEventElapsedTime(&ms, ev.first, ev.second));
        t.total_ms[p] += ms;
        t.count[p] += 1;
        (void)hipEventDestroy(ev.first);
        (void)hipEventDestroy(ev.second);
    }
    t.pending[p].clear();
    if (avg_ms) *avg_ms = t.count[p] ? t.total_ms[p] / (double)t.count[p] : 0.0;
    if (count) *count = t.count[p];
    if (reset) {
        t.total_ms[p] = 0.0;
        t.count[p] = 0;
    }
    return GABI_OK;
}

}  // extern "C"
