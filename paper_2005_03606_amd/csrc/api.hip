// C ABI entry points: argument validation, hierarchy objects, dispatch.
#include <math.h>
#include <stdio.h>

#include "common.h"

int store_set_base(mgd_hier *h, OpSet &o, const float *eps_c, hipStream_t st);

static const int64_t kMaxCoarseDofs = 1500;
void solve_cache_free(mgd_ctx *ctx);


static int64_t ipow(int64_t b, int e)
{
    int64_t r = 1;
    for (int i = 0; i < e; ++i) r *= b;
    return r;
}

int hier_alloc_levels(mgd_hier *h)
{
    mgd_ctx *ctx = h->ctx;
    h->H = n_half(h->dim);
    int nlev = 0, nn = h->n;
    h->nl[nlev++] = nn;
    while (nn % 2 == 0 && nn / 2 >= h->coarsest && nlev < MGD_MAXLEV) {
        nn /= 2;
        h->nl[nlev++] = nn;
    }
    h->nlev = nlev;
    for (int l = 0; l < nlev; ++l) h->NV[l] = ipow(h->nl[l] + 1, h->dim);
    h->m_coarse = ipow(h->nl[nlev - 1] - 1, h->dim);
    if (h->m_coarse > kMaxCoarseDofs)
        return mgd_fail(ctx, MGD_EINVAL, "coarsest grid has %lld interior vertices (limit %lld): n must be "
                        "divisible by 2 down to a small grid", (long long)h->m_coarse, (long long)kMaxCoarseDofs);
    int rc = opset_alloc(h, h->ops);
    if (rc) return rc;
    size_t vb = h->vec_bytes();
    for (int l = 0; l < nlev; ++l) {
        size_t b = (size_t)h->NV[l] * vb;
        if ((rc = dev_alloc(ctx, &h->u[l], b)) || (rc = dev_alloc(ctx, &h->f[l], b)) ||
            (rc = dev_alloc(ctx, &h->r[l], b)) || (rc = dev_alloc(ctx, &h->t[l], b)))
            return rc;
        HIPCHK(ctx, hipMemset(h->u[l], 0, b));
        HIPCHK(ctx, hipMemset(h->f[l], 0, b));
        HIPCHK(ctx, hipMemset(h->r[l], 0, b));
        HIPCHK(ctx, hipMemset(h->t[l], 0, b));
    }
    int64_t nb = (h->NV[0] + 255) / 256 + (h->nl[0] + 1) / 4 + 64;
    h->partial_cap = 2 * nb > h->m_coarse + 64 ? 2 * nb : h->m_coarse + 64;
    if ((rc = dev_alloc(ctx, (void **)&h->partial, (size_t)h->partial_cap * 8))) return rc;
    if ((rc = dev_alloc(ctx, (void **)&h->scal, 64 * 8))) return rc;
    HIPCHK(ctx, hipMemset(h->scal, 0, 64 * 8));
    if ((rc = dev_alloc(ctx, (void **)&h->partial2, (size_t)h->partial_cap * 8))) return rc;
    if (hipHostMalloc((void **)&h->host_scal, 64 * 8, hipHostMallocDefault) != hipSuccess)
        return mgd_fail(ctx, MGD_ENOMEM, "pinned allocation failed");
    // coherent: kernel stores bypass the GPU caches on their way to the host
    if (hipHostMalloc((void **)&h->host_part, kHostParts * 8, hipHostMallocCoherent) != hipSuccess)
        return mgd_fail(ctx, MGD_ENOMEM, "pinned allocation failed");
    for (int i = 0; i < kHostParts; ++i) h->host_part[i] = 0.0;
    HIPCHK(ctx, hipHostGetDevicePointer((void **)&h->host_part_dev, h->host_part, 0));
    // the clears above run on the null stream, which work on the caller's
    // non-blocking streams does not wait for: finish them before returning
    HIPCHK(ctx, hipDeviceSynchronize());
    return MGD_OK;
}

// working buffers of mgd_compress_stencils (the surplus [H][NV] and the
// vertex tiers), allocated on its first call on a hierarchy; the solver
// allocates them with its workspace
int hier_compress_buffers(mgd_hier *h)
{
    int rc;
    if (!h->delta && (rc = dev_alloc(h->ctx, (void **)&h->delta, (size_t)h->NV[0] * h->H * 4))) return rc;
    if (!h->vtier && (rc = dev_alloc(h->ctx, (void **)&h->vtier, (size_t)h->NV[0]))) return rc;
    return MGD_OK;
}

void hier_free(mgd_hier *h)
{
    opset_free(h->ops);
    for (int l = 0; l < MGD_MAXLEV; ++l) {
        dev_free(h->u[l]); dev_free(h->f[l]); dev_free(h->r[l]); dev_free(h->t[l]);
        h->u[l] = h->f[l] = h->r[l] = h->t[l] = nullptr;
    }
    dev_free(h->delta); dev_free(h->vtier);
    h->delta = nullptr;
    h->vtier = nullptr;
    dev_free(h->partial); dev_free(h->scal);
    h->partial = nullptr;
    h->scal = nullptr;
    h->partial_cap = 0;
    if (h->host_scal) (void)hipHostFree(h->host_scal);
    h->host_scal = nullptr;
    dev_free(h->partial2);
    h->partial2 = nullptr;
    if (h->host_part) (void)hipHostFree(h->host_part);
    h->host_part = h->host_part_dev = nullptr;
}

// ------------------------------------------------------------ validation
static int check_grid(mgd_ctx *ctx, int dim, int n)
{
    if (dim != 2 && dim != 3) return mgd_fail(ctx, MGD_EINVAL, "dim must be 2 or 3 (got %d)", dim);
    if (n < 1) return mgd_fail(ctx, MGD_EINVAL, "n must be >= 1 (got %d)", n);
    double nv = pow((double)n + 1, dim);
    if (nv > 4.0e9) return mgd_fail(ctx, MGD_EINVAL, "grid too large");
    return MGD_OK;
}

static int check_s(mgd_ctx *ctx, int s)
{
    if (s != 1 && s != 2 && s != 4 && s != 8 && s != 16)
        return mgd_fail(ctx, MGD_EINVAL, "s must be 1, 2, 4, 8 or 16 (got %d)", s);
    return MGD_OK;
}

static int check_eps(mgd_ctx *ctx, const mgd_eps *e, int dim, bool samples_ok)
{
    if (!e) return mgd_fail(ctx, MGD_EINVAL, "eps is NULL");
    if (e->kind < MGD_EPS_CONST || e->kind > MGD_EPS_SAMPLES)
        return mgd_fail(ctx, MGD_EINVAL, "unknown eps kind %d", e->kind);
    if (e->kind == MGD_EPS_SAMPLES && !samples_ok)
        return mgd_fail(ctx, MGD_EINVAL, "sample matrices are accepted by mgd_assemble_cells only");
    if (e->dim != dim) return mgd_fail(ctx, MGD_EINVAL, "eps.dim %d differs from dim %d", e->dim, dim);
    bool needs_data = e->kind >= MGD_EPS_BALLS;
    if (needs_data && !e->data) return mgd_fail(ctx, MGD_EINVAL, "eps.data is NULL");
    if ((e->kind == MGD_EPS_BALLS || e->kind == MGD_EPS_BOXES) && e->count < 0)
        return mgd_fail(ctx, MGD_EINVAL, "eps.count < 0");
    if (e->kind == MGD_EPS_LATTICE && e->count < 1) return mgd_fail(ctx, MGD_EINVAL, "lattice needs count >= 1");
    return MGD_OK;
}

// ------------------------------------------------------------ ABI
extern "C" {

const char *mgd_version(void) { return "mgdelay gfx950 1.0"; }

int mgd_create(mgd_ctx **out, int device)
{
    if (!out) return MGD_EINVAL;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return MGD_EINVAL;
    mgd_ctx *ctx = new mgd_ctx();
    ctx->device = device;
    if (hipSetDevice(device) != hipSuccess) { delete ctx; return MGD_EHIP; }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess) ctx->num_cu = prop.multiProcessorCount;
    if (hipStreamCreateWithFlags(&ctx->s_asm, hipStreamNonBlocking) != hipSuccess) { delete ctx; return MGD_EHIP; }
    if (scratch_init(ctx) != MGD_OK) {
        (void)hipStreamDestroy(ctx->s_asm);
        delete ctx;
        return MGD_EHIP;
    }
    *out = ctx;
    return MGD_OK;
}

int mgd_destroy(mgd_ctx *ctx)
{
    if (!ctx) return MGD_OK;
    (void)hipSetDevice(ctx->device);
    if (ctx->s_asm) (void)hipStreamSynchronize(ctx->s_asm);
    solve_cache_free(ctx);
    if (ctx->s_asm) (void)hipStreamDestroy(ctx->s_asm);
    delete ctx;
    return MGD_OK;
}

const char *mgd_last_error(const mgd_ctx *ctx) { return ctx ? ctx->err : "no context"; }

int mgd_assemble_cells(mgd_ctx *ctx, int32_t dim, int32_t n, int32_t s, const int64_t *cells, int64_t count,
                       const mgd_eps *eps, int32_t mode, void *K_out, const void *K_old, double C,
                       double *rel_out, uint8_t *done_out, hipStream_t stream)
{
    if (!ctx) return MGD_EINVAL;
    int rc;
    if ((rc = check_grid(ctx, dim, n)) || (rc = check_s(ctx, s)) || (rc = check_eps(ctx, eps, dim, true))) return rc;
    if (mode != MGD_FP64 && mode != MGD_MIXED) return mgd_fail(ctx, MGD_EINVAL, "mode must be MGD_FP64 or MGD_MIXED");
    int64_t ncell = ipow(n, dim);
    if (count == 0) return MGD_OK;
    if (!cells && count != ncell) return mgd_fail(ctx, MGD_EINVAL, "cells == NULL needs count == n^d");
    if (count < 0 || count > ncell) return mgd_fail(ctx, MGD_EINVAL, "bad count %lld", (long long)count);
    if (!K_out && count > 0) return mgd_fail(ctx, MGD_EINVAL, "K_out is NULL");
    if (K_old && K_old == K_out) return mgd_fail(ctx, MGD_EINVAL, "K_old must not alias K_out");
    if (!(C >= 0.0)) return mgd_fail(ctx, MGD_EINVAL, "C must be >= 0");
    HIPCHK(ctx, hipSetDevice(ctx->device));
    return launch_assemble(ctx, dim, n, s, cells, count, eps, mode, K_out, K_old, 0, C, rel_out, done_out,
                           nullptr, stream);
}

int mgd_ladder_step_keep(mgd_ctx *ctx, int32_t dim, int32_t n, int32_t s, const int64_t *cells, int64_t count,
                         const mgd_eps *eps, double *K, double C, double *rel_out, uint8_t *done_out,
                         hipStream_t stream)
{
    if (!ctx) return MGD_EINVAL;
    int rc;
    if ((rc = check_grid(ctx, dim, n)) || (rc = check_eps(ctx, eps, dim, false))) return rc;
    if (s < 1 || s > 16) return mgd_fail(ctx, MGD_EINVAL, "s must be in 1..16 (got %d)", s);
    int64_t ncell = ipow(n, dim);
    if (count == 0) return MGD_OK;
    if (!cells && count != ncell) return mgd_fail(ctx, MGD_EINVAL, "cells == NULL needs count == n^d");
    if (count < 0 || count > ncell) return mgd_fail(ctx, MGD_EINVAL, "bad count %lld", (long long)count);
    if (!K) return mgd_fail(ctx, MGD_EINVAL, "K is NULL");
    if (!(C >= 0.0)) return mgd_fail(ctx, MGD_EINVAL, "C must be >= 0");
    HIPCHK(ctx, hipSetDevice(ctx->device));
    // rows by cell id, read and rewritten in place by the lane that owns the cell
    return launch_assemble(ctx, dim, n, s, cells, count, eps, MGD_FP64, K, K, 1, C, rel_out, done_out, nullptr,
                           stream, 1);
}

int mgd_p3_encode(mgd_ctx *ctx, int32_t dim, const double *K, const double *K1, int64_t count, double tau,
                  uint8_t *p3_out, uint8_t *bytes_out, hipStream_t stream)
{
    if (!ctx) return MGD_EINVAL;
    if (dim != 2 && dim != 3) return mgd_fail(ctx, MGD_EINVAL, "dim must be 2 or 3 (got %d)", dim);
    if (count < 0) return mgd_fail(ctx, MGD_EINVAL, "bad count %lld", (long long)count);
    if (!(tau >= 0.0)) return mgd_fail(ctx, MGD_EINVAL, "tau must be >= 0");
    if (count == 0) return MGD_OK;
    if (!K || !K1 || !p3_out || !bytes_out) return mgd_fail(ctx, MGD_EINVAL, "NULL buffer");
    HIPCHK(ctx, hipSetDevice(ctx->device));
    return launch_p3_encode(ctx, dim, K, K1, count, tau, p3_out, bytes_out, stream);
}

int mgd_centre_samples(mgd_ctx *ctx, int32_t dim, int32_t n, const mgd_eps *eps, float *eps_c_out,
                       hipStream_t stream)
{
    if (!ctx) return MGD_EINVAL;
    int rc;
    if ((rc = check_grid(ctx, dim, n)) || (rc = check_eps(ctx, eps, dim, false))) return rc;
    if (!eps_c_out) return mgd_fail(ctx, MGD_EINVAL, "eps_c_out is NULL");
    HIPCHK(ctx, hipSetDevice(ctx->device));
    return launch_centre_eps(ctx, dim, n, eps, eps_c_out, stream);
}

int mgd_gather_stencils(mgd_ctx *ctx, int32_t dim, int32_t n, const void *K, int32_t k_mode, void *S_out,
                        int32_t s_mode, hipStream_t stream)
{
    if (!ctx) return MGD_EINVAL;
    int rc;
    if ((rc = check_grid(ctx, dim, n))) return rc;
    if (!K || !S_out) return mgd_fail(ctx, MGD_EINVAL, "null buffer");
    if ((k_mode != MGD_FP64 && k_mode != MGD_MIXED) || (s_mode != MGD_FP64 && s_mode != MGD_MIXED))
        return mgd_fail(ctx, MGD_EINVAL, "bad mode");
    HIPCHK(ctx, hipSetDevice(ctx->device));
    return launch_gather(ctx, dim, n, K, k_mode, S_out, s_mode, stream);
}

int mgd_hier_create(mgd_ctx *ctx, const mgd_hier_desc *d, mgd_hier **out)
{
    if (!ctx || !d || !out) return MGD_EINVAL;
    *out = nullptr;
    int rc;
    if ((rc = check_grid(ctx, d->dim, d->n))) return rc;
    if (d->n < 2) return mgd_fail(ctx, MGD_EINVAL, "n must be >= 2");
    if (d->precision != MGD_FP64 && d->precision != MGD_MIXED) return mgd_fail(ctx, MGD_EINVAL, "bad precision");
    if (d->transfer != MGD_GEOMETRIC && d->transfer != MGD_BOXMG) return mgd_fail(ctx, MGD_EINVAL, "bad transfer");
    if (d->coarsest < 2) return mgd_fail(ctx, MGD_EINVAL, "coarsest must be >= 2");
    if (d->store_path < MGD_STORE_AUTO || d->store_path > MGD_STORE_COPY)
        return mgd_fail(ctx, MGD_EINVAL, "bad store_path");
    HIPCHK(ctx, hipSetDevice(ctx->device));
    mgd_hier *h = new mgd_hier();
    h->ctx = ctx;
    h->dim = d->dim; h->n = d->n; h->precision = d->precision; h->transfer = d->transfer; h->coarsest = d->coarsest;
    h->store_path = d->store_path;
    rc = hier_alloc_levels(h);
    if (rc) { hier_free(h); delete h; return rc; }
    *out = h;
    return MGD_OK;
}

int mgd_hier_destroy(mgd_hier *h)
{
    if (!h) return MGD_OK;
    (void)hipSetDevice(h->ctx->device);
    (void)hipDeviceSynchronize();
    hier_free(h);
    delete h;
    return MGD_OK;
}

int mgd_hier_levels(const mgd_hier *h) { return h ? h->nlev : MGD_EINVAL; }
int mgd_hier_level_n(const mgd_hier *h, int level)
{
    return (h && level >= 0 && level < h->nlev) ? h->nl[level] : MGD_EINVAL;
}

int mgd_hier_set_fine(mgd_ctx *ctx, mgd_hier *h, const double *S, hipStream_t stream)
{
    if (!ctx || !h || !S) return MGD_EINVAL;
    if (h->precision != MGD_FP64) return mgd_fail(ctx, MGD_EINVAL, "set_fine needs an FP64 hierarchy");
    h->ops.dz_ok = 0;
    HIPCHK(ctx, hipMemcpyAsync(h->ops.S64[0], S, (size_t)h->NV[0] * h->H * 8, hipMemcpyDeviceToDevice, stream));
    return MGD_OK;
}

int mgd_compress_stencils(mgd_ctx *ctx, mgd_hier *h, const float *S32, const float *eps_c,
                          const mgd_tier_policy *pol, hipStream_t stream)
{
    if (!ctx || !h || !S32 || !eps_c || !pol) return MGD_EINVAL;
    if (h->precision != MGD_MIXED) return mgd_fail(ctx, MGD_EINVAL, "compress needs a MGD_MIXED hierarchy");
    if (pol->min_tier < 1 || pol->max_tier > 3 || pol->min_tier > pol->max_tier)
        return mgd_fail(ctx, MGD_EINVAL, "tiers must satisfy 1 <= min_tier <= max_tier <= 3");
    if (!(pol->tau_abs >= 0.0) || !(pol->tau_rel >= 0.0)) return mgd_fail(ctx, MGD_EINVAL, "tau must be >= 0");
    HIPCHK(ctx, hipSetDevice(ctx->device));
    int rc = hier_compress_buffers(h);
    if (rc) return rc;
    return compress_into(h, h->ops, S32, eps_c, pol, h->delta, h->vtier, stream);
}

int mgd_tier0_items(mgd_ctx *ctx, mgd_hier *h, int64_t *items, int64_t *tier0, hipStream_t stream)
{
    if (!ctx || !h || !items || !tier0) return MGD_EINVAL;
    if (h->dim != 3 || h->precision != MGD_MIXED)
        return mgd_fail(ctx, MGD_EINVAL, "tier-0 items exist for a 3D mixed hierarchy only");
    HIPCHK(ctx, hipSetDevice(ctx->device));
    return item_mask_count(h, items, tier0, stream);
}

int mgd_weight_tiles(mgd_ctx *ctx, const mgd_hier *h, int32_t level, int64_t *ntile, int64_t *geo_tiles)
{
    if (!ctx || !h || !ntile || !geo_tiles) return MGD_EINVAL;
    if (h->dim != 3 || h->transfer != MGD_BOXMG) return mgd_fail(ctx, MGD_EINVAL, "weight tiles need a 3D BoxMG hierarchy");
    if (level < 0 || level + 1 >= h->nlev) return mgd_fail(ctx, MGD_EINVAL, "level %d has no coarser level", level);
    HIPCHK(ctx, hipSetDevice(ctx->device));
    const int64_t nt = (h->NV[level] + 63) / 64;
    std::vector<uint8_t> f((size_t)nt);
    HIPCHK(ctx, hipDeviceSynchronize());
    HIPCHK(ctx, hipMemcpy(f.data(), h->ops.wgeo[level], (size_t)nt, hipMemcpyDeviceToHost));
    int64_t g = 0;
    for (uint8_t b : f) g += b != 0;
    *ntile = nt;
    *geo_tiles = g;
    return MGD_OK;
}

int mgd_store_info(mgd_ctx *ctx, const mgd_hier *h, int64_t *ntile, int64_t *payload_bytes, int64_t tier_tiles[4])
{
    if (!ctx || !h) return MGD_EINVAL;
    if (h->precision != MGD_MIXED) return mgd_fail(ctx, MGD_EINVAL, "no compressed store in an FP64 hierarchy");
    HIPCHK(ctx, hipDeviceSynchronize());
    uint32_t units = 0;
    HIPCHK(ctx, hipMemcpy(&units, h->ops.units_total, 4, hipMemcpyDeviceToHost));
    if (ntile) *ntile = h->ops.ntile;
    if (payload_bytes) *payload_bytes = (int64_t)units * 64;
    if (tier_tiles) {
        std::vector<uint8_t> t(h->ops.ntile);
        HIPCHK(ctx, hipMemcpy(t.data(), h->ops.tier, h->ops.ntile, hipMemcpyDeviceToHost));
        for (int k = 0; k < 4; ++k) tier_tiles[k] = 0;
        for (uint8_t x : t) tier_tiles[x & 3]++;
    }
    return MGD_OK;
}

int mgd_store_export(mgd_ctx *ctx, const mgd_hier *h, uint8_t *tile_tier, uint32_t *tile_off, uint8_t *payload,
                     hipStream_t stream)
{
    if (!ctx || !h) return MGD_EINVAL;
    if (h->precision != MGD_MIXED) return mgd_fail(ctx, MGD_EINVAL, "no compressed store in an FP64 hierarchy");
    const OpSet &o = h->ops;
    if (tile_tier) HIPCHK(ctx, hipMemcpyAsync(tile_tier, o.tier, o.ntile, hipMemcpyDeviceToDevice, stream));
    if (tile_off) HIPCHK(ctx, hipMemcpyAsync(tile_off, o.toff, o.ntile * 4, hipMemcpyDeviceToDevice, stream));
    if (payload) {
        HIPCHK(ctx, hipStreamSynchronize(stream));
        uint32_t units = 0;
        HIPCHK(ctx, hipMemcpy(&units, o.units_total, 4, hipMemcpyDeviceToHost));
        HIPCHK(ctx, hipMemcpyAsync(payload, o.payload, (size_t)units * 64, hipMemcpyDeviceToDevice, stream));
    }
    return MGD_OK;
}

int mgd_coarsen(mgd_ctx *ctx, mgd_hier *h, hipStream_t stream)
{
    if (!ctx || !h) return MGD_EINVAL;
    HIPCHK(ctx, hipSetDevice(ctx->device));
    return coarsen_ops(h, h->ops, stream);
}

int mgd_level_stencils(mgd_ctx *ctx, const mgd_hier *h, int level, double *S_out, hipStream_t stream)
{
    if (!ctx || !h || !S_out) return MGD_EINVAL;
    if (level < 0 || level >= h->nlev) return mgd_fail(ctx, MGD_EINVAL, "level out of range");
    return decode_level_f64(const_cast<mgd_hier *>(h), h->ops, level, S_out, stream);
}

int mgd_level_weights(mgd_ctx *ctx, const mgd_hier *h, int level, double *W_out, hipStream_t stream)
{
    if (!ctx || !h || !W_out) return MGD_EINVAL;
    if (level < 0 || level + 1 >= h->nlev) return mgd_fail(ctx, MGD_EINVAL, "level has no coarser level");
    return weights_f64(const_cast<mgd_hier *>(h), h->ops, level, W_out, stream);
}

static int check_level(mgd_ctx *ctx, const mgd_hier *h, int level, bool need_coarser)
{
    if (!h) return MGD_EINVAL;
    if (level < 0 || level >= h->nlev || (need_coarser && level + 1 >= h->nlev))
        return mgd_fail(ctx, MGD_EINVAL, "level %d out of range", level);
    return MGD_OK;
}

int mgd_smooth(mgd_ctx *ctx, mgd_hier *h, int level, void *u, const void *f, int32_t sweeps, double omega,
               hipStream_t stream)
{
    if (!ctx) return MGD_EINVAL;
    int rc;
    if ((rc = check_level(ctx, h, level, false))) return rc;
    if (!u || !f || sweeps < 0) return mgd_fail(ctx, MGD_EINVAL, "bad smooth arguments");
    return cycle_smooth(h, h->ops, level, u, f, h->t[level], sweeps, omega, false, stream);
}

int mgd_presmooth(mgd_ctx *ctx, mgd_hier *h, int level, const void *u, const void *f, void *u_out, void *r_out,
                  double omega, hipStream_t stream)
{
    if (!ctx) return MGD_EINVAL;
    int rc;
    if ((rc = check_level(ctx, h, level, false))) return rc;
    if (!f || !u_out || !r_out || u_out == u || u_out == r_out || r_out == f)
        return mgd_fail(ctx, MGD_EINVAL, "bad presmooth arguments (null or aliased buffers)");
    if (h->dim == 2) return lev2_pre(h, h->ops, level, u, f, u_out, r_out, omega, stream);
    size_t b = h->NV[level] * h->vec_bytes();
    if (u) HIPCHK(ctx, hipMemcpyAsync(u_out, u, b, hipMemcpyDeviceToDevice, stream));
    if ((rc = cycle_smooth(h, h->ops, level, u_out, f, h->t[level], 2, omega, u == nullptr, stream))) return rc;
    return cycle_residual(h, h->ops, level, u_out, f, r_out, stream);
}

int mgd_presmooth_restrict(mgd_ctx *ctx, mgd_hier *h, int level, const void *u, const void *f, void *u_out,
                           void *fc, double omega, hipStream_t stream)
{
    if (!ctx) return MGD_EINVAL;
    int rc;
    if ((rc = check_level(ctx, h, level, true))) return rc;
    if (!f || !u_out || !fc || u_out == u || fc == f || fc == u_out)
        return mgd_fail(ctx, MGD_EINVAL, "bad presmooth_restrict arguments (null or aliased buffers)");
    if (!lev2_ok(h, level, 2, 2)) return mgd_fail(ctx, MGD_EINVAL, "presmooth_restrict needs a 2D hierarchy");
    return lev2_prer(h, h->ops, level, u, f, u_out, fc, omega, stream);
}

int mgd_residual(mgd_ctx *ctx, mgd_hier *h, int level, const void *u, const void *f, void *r, hipStream_t stream)
{
    if (!ctx) return MGD_EINVAL;
    int rc;
    if ((rc = check_level(ctx, h, level, false))) return rc;
    if (!u || !f || !r) return mgd_fail(ctx, MGD_EINVAL, "null vector");
    return cycle_residual(h, h->ops, level, u, f, r, stream);
}

int mgd_restrict(mgd_ctx *ctx, mgd_hier *h, int level, const void *r, void *fc, hipStream_t stream)
{
    if (!ctx) return MGD_EINVAL;
    int rc;
    if ((rc = check_level(ctx, h, level, true))) return rc;
    if (!r || !fc) return mgd_fail(ctx, MGD_EINVAL, "null vector");
    return cycle_restrict(h, h->ops, level, r, fc, stream);
}

int mgd_prolong_add(mgd_ctx *ctx, mgd_hier *h, int level, const void *ec, void *u, hipStream_t stream)
{
    if (!ctx) return MGD_EINVAL;
    int rc;
    if ((rc = check_level(ctx, h, level, true))) return rc;
    if (!ec || !u) return mgd_fail(ctx, MGD_EINVAL, "null vector");
    return cycle_prolong(h, h->ops, level, ec, u, stream);
}

int mgd_vcycle(mgd_ctx *ctx, mgd_hier *h, void *u, const void *f, const mgd_cycle_opts *opts, hipStream_t stream)
{
    if (!ctx || !h || !u || !f || !opts) return MGD_EINVAL;
    if (opts->nu1 < 0 || opts->nu2 < 0) return mgd_fail(ctx, MGD_EINVAL, "nu must be >= 0");
    return vcycle_ops(h, h->ops, u, f, opts->omega, opts->nu1, opts->nu2, false, stream);
}

int mgd_outer_residual(mgd_ctx *ctx, mgd_hier *h, const double *u, const double *f, double *r, hipStream_t stream)
{
    if (!ctx || !h || !u || !f || !r) return MGD_EINVAL;
    return outer_residual(h, h->ops, u, f, r, nullptr, stream);
}

}  // extern "C"
