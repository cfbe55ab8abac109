// mgd_solve: delayed (lazy) or up-front assembly feeding a multigrid solve
// (paper Sec. 5.1-5.4).  The ladder of sub-sample counts runs on the
// assembly stream; each completed rung is turned into a full operator set
// (stencils, surplus store, coarse operators) in the spare of two operator
// sets and published at a cycle boundary, where the solver switches sets.
#include <math.h>

#include <chrono>

#include "common.h"

int store_set_base(mgd_hier *h, OpSet &o, const float *eps_c, hipStream_t st);
int vec_cast_to_cycle(mgd_hier *h, const double *a, void *b, hipStream_t st);
int vec_add_cycle(mgd_hier *h, double *u, const void *e, hipStream_t st);
int pcg_beta(mgd_hier *h, const void *z, const double *r, const double *rold, double *s, hipStream_t st);
int pcg_matvec(mgd_hier *h, const OpSet &o, const void *z, const double *pold, double *pnew, double *Ap, double *s,
               hipStream_t st);
int pcg_update(mgd_hier *h, double *x, const double *p, double *r, double *rold, const double *Ap, double *s,
               hipStream_t st);
int vec_fill_f64(mgd_ctx *ctx, double *a, int64_t n, double v, hipStream_t st);

namespace {

struct Ladder {
    mgd_hier *h = nullptr;
    mgd_eps eps{};
    int s_fixed = 0, s_max = 1, R = 0;  // rungs 1..R use s = 2^r
    double C = 0.01;
    mgd_tier_policy tiers{};
    int64_t ncell = 0;
    void *K = nullptr;        // [ncell][U] current element matrices (in place)
    float *eps_c = nullptr;   // centre samples
    float *Sg = nullptr;      // gathered FP32 couplings (mixed)
    int64_t *act[2] = {nullptr, nullptr};
    int64_t *cnt_dev = nullptr;  // [2]
    uint8_t *done = nullptr;
    int32_t *blk = nullptr;
    int64_t *cnt_host = nullptr;  // pinned [8]: active cells at rung r
    int mode() const { return h->precision; }
};

void ladder_free(Ladder &L)
{
    dev_free(L.K); dev_free(L.eps_c); dev_free(L.Sg);
    dev_free(L.act[0]); dev_free(L.act[1]); dev_free(L.cnt_dev); dev_free(L.done); dev_free(L.blk);
    if (L.cnt_host) (void)hipHostFree(L.cnt_host);
}

int ladder_alloc(Ladder &L)
{
    mgd_ctx *ctx = L.h->ctx;
    int U = n_pairs(L.h->dim), rc;
    size_t kb = L.h->precision == MGD_FP64 ? 8 : 4;
    if ((rc = dev_alloc(ctx, &L.K, (size_t)L.ncell * U * kb))) return rc;
    if ((rc = dev_alloc(ctx, (void **)&L.eps_c, (size_t)L.ncell * 4))) return rc;
    if (L.h->precision == MGD_MIXED)
        if ((rc = dev_alloc(ctx, (void **)&L.Sg, (size_t)L.h->NV[0] * L.h->H * 4))) return rc;
    if (L.R >= 2) {
        if ((rc = dev_alloc(ctx, (void **)&L.act[0], (size_t)L.ncell * 8))) return rc;
        if ((rc = dev_alloc(ctx, (void **)&L.act[1], (size_t)L.ncell * 8))) return rc;
    }
    if ((rc = dev_alloc(ctx, (void **)&L.cnt_dev, 2 * 8))) return rc;
    if ((rc = dev_alloc(ctx, (void **)&L.done, (size_t)L.ncell))) return rc;
    if ((rc = dev_alloc(ctx, (void **)&L.blk, (size_t)((L.ncell + 255) / 256 + 1) * 4))) return rc;
    if (hipHostMalloc((void **)&L.cnt_host, 8 * 8, hipHostMallocDefault) != hipSuccess)
        return mgd_fail(ctx, MGD_ENOMEM, "pinned allocation failed");
    for (int r = 0; r < 8; ++r) L.cnt_host[r] = 0;
    return MGD_OK;
}

// rung 0: every cell at s_fixed (or the centre sample), plus centre samples
int rung0(Ladder &L, hipStream_t st)
{
    mgd_ctx *ctx = L.h->ctx;
    int s0 = L.s_fixed > 0 ? L.s_fixed : 1;
    int rc = launch_assemble(ctx, L.h->dim, L.h->n, s0, nullptr, L.ncell, &L.eps, L.mode(), L.K, nullptr, 0, 0.0,
                             nullptr, nullptr, nullptr, st);
    if (rc) return rc;
    L.cnt_host[0] = L.ncell;
    L.cnt_host[1] = L.R >= 1 ? L.ncell : 0;
    if (L.h->precision == MGD_MIXED) return launch_centre_eps(ctx, L.h->dim, L.h->n, &L.eps, L.eps_c, st);
    return MGD_OK;
}

// rung r >= 1: integrate the open cells at s = 2^r in place, criterion
// against the stored matrix, then compact the still-open cells for rung r+1
int rung(Ladder &L, int r, hipStream_t st)
{
    mgd_ctx *ctx = L.h->ctx;
    const int64_t *cells = r == 1 ? nullptr : L.act[r % 2];
    const int64_t *cnt = r == 1 ? nullptr : L.cnt_dev + (r % 2);
    int rc = launch_assemble(ctx, L.h->dim, L.h->n, 1 << r, cells, L.ncell, &L.eps, L.mode(), L.K, L.K, 1, L.C,
                             nullptr, L.done, cnt, st);
    if (rc) return rc;
    if (r < L.R) {
        rc = launch_compact_open(ctx, L.done, cells, cnt, L.ncell, L.blk, L.act[(r + 1) % 2],
                                 L.cnt_dev + ((r + 1) % 2), st);
        if (rc) return rc;
        HIPCHK(ctx, hipMemcpyAsync(L.cnt_host + r + 1, L.cnt_dev + ((r + 1) % 2), 8, hipMemcpyDeviceToHost, st));
    }
    return MGD_OK;
}

// operator set from the current element matrices
int build(Ladder &L, OpSet &o, bool base_only, hipStream_t st)
{
    mgd_hier *h = L.h;
    int rc;
    if (h->precision == MGD_FP64) {
        if ((rc = launch_gather(h->ctx, h->dim, h->n, L.K, MGD_FP64, o.S64[0], MGD_FP64, st))) return rc;
    } else if (base_only) {
        if ((rc = store_set_base(h, o, L.eps_c, st))) return rc;
    } else {
        if ((rc = launch_gather(h->ctx, h->dim, h->n, L.K, MGD_MIXED, L.Sg, MGD_MIXED, st))) return rc;
        if ((rc = compress_into(h, o, L.Sg, L.eps_c, &L.tiers, st))) return rc;
    }
    return coarsen_ops(h, o, st);
}

double now_ms()
{
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

}  // namespace

extern "C" int mgd_solve(mgd_ctx *ctx, int32_t dim, int32_t n, const mgd_eps *eps, const double *f, double *u,
                         const mgd_solve_opts *op, mgd_report *rep, hipStream_t stream)
{
    if (!ctx || !eps || !f || !u || !op || !rep) return MGD_EINVAL;
    double t0 = now_ms();
    memset(rep, 0, sizeof(*rep));
    if (dim != 2 && dim != 3) return mgd_fail(ctx, MGD_EINVAL, "dim must be 2 or 3");
    if (eps->kind < MGD_EPS_CONST || eps->kind > MGD_EPS_BOXES || eps->dim != dim)
        return mgd_fail(ctx, MGD_EINVAL, "eps must be a field descriptor of the same dimension");
    if (eps->kind >= MGD_EPS_BALLS && !eps->data) return mgd_fail(ctx, MGD_EINVAL, "eps.data is NULL");
    if (op->precision != MGD_FP64 && op->precision != MGD_MIXED) return mgd_fail(ctx, MGD_EINVAL, "bad precision");
    if (op->outer != MGD_STATIONARY && op->outer != MGD_PCG) return mgd_fail(ctx, MGD_EINVAL, "bad outer");
    if (op->schedule != MGD_UPFRONT && op->schedule != MGD_LAZY) return mgd_fail(ctx, MGD_EINVAL, "bad schedule");
    int sf = op->s_fixed;
    if (sf > 0 && sf != 1 && sf != 2 && sf != 4 && sf != 8 && sf != 16) return mgd_fail(ctx, MGD_EINVAL, "bad s_fixed");
    int sm = op->s_max;
    if (sf <= 0 && sm != 1 && sm != 2 && sm != 4 && sm != 8 && sm != 16) return mgd_fail(ctx, MGD_EINVAL, "bad s_max");
    if (op->nu1 < 0 || op->nu2 < 0 || op->max_cycles < 0 || !(op->tol >= 0.0) || !(op->div_factor > 0.0))
        return mgd_fail(ctx, MGD_EINVAL, "bad cycle options");
    if (op->precision == MGD_MIXED &&
        (op->tiers.min_tier < 1 || op->tiers.max_tier > 3 || op->tiers.min_tier > op->tiers.max_tier))
        return mgd_fail(ctx, MGD_EINVAL, "bad tier policy");
    HIPCHK(ctx, hipSetDevice(ctx->device));

    mgd_hier H;
    H.ctx = ctx;
    H.dim = dim; H.n = n; H.precision = op->precision; H.transfer = op->transfer;
    H.coarsest = op->coarsest < 2 ? 2 : op->coarsest;
    Ladder L;
    OpSet O1;
    int rc = MGD_OK;
    hipEvent_t ev_ready[8] = {}, ev_free = nullptr, ev_start = nullptr;
    double *r = nullptr, *rold = nullptr, *p[2] = {nullptr, nullptr}, *Ap = nullptr;
    bool lazy = op->schedule == MGD_LAZY && sf <= 0 && sm >= 2;
    int status = MGD_ENOCONV, k = 0, ncyc = 0;
    auto cleanup = [&]() {
        (void)hipStreamSynchronize(ctx->s_asm);
        (void)hipStreamSynchronize(stream);
        ladder_free(L);
        opset_free(O1);
        hier_free(&H);
        dev_free(r); dev_free(rold); dev_free(p[0]); dev_free(p[1]); dev_free(Ap);
        for (auto &e : ev_ready) if (e) (void)hipEventDestroy(e);
        if (ev_free) (void)hipEventDestroy(ev_free);
        if (ev_start) (void)hipEventDestroy(ev_start);
    };
#define TRY(x)                   \
    do {                         \
        if ((rc = (x))) {        \
            cleanup();           \
            return rc;           \
        }                        \
    } while (0)

    TRY(hier_alloc_levels(&H));
    if (lazy) TRY(opset_alloc(&H, O1));
    L.h = &H;
    L.eps = *eps;
    L.s_fixed = sf;
    L.s_max = sf > 0 ? sf : sm;
    L.R = 0;
    if (sf <= 0) while ((1 << L.R) < sm) ++L.R;
    L.C = op->C;
    L.tiers = op->tiers;
    L.ncell = 1;
    for (int m = 0; m < dim; ++m) L.ncell *= n;
    TRY(ladder_alloc(L));
    int64_t NV = H.NV[0];
    TRY(dev_alloc(ctx, (void **)&r, NV * 8));
    TRY(dev_alloc(ctx, (void **)&rold, NV * 8));
    TRY(dev_alloc(ctx, (void **)&p[0], NV * 8));
    TRY(dev_alloc(ctx, (void **)&p[1], NV * 8));
    TRY(dev_alloc(ctx, (void **)&Ap, NV * 8));
    TRY(vec_fill_f64(ctx, rold, NV, 0.0, stream));
    TRY(vec_fill_f64(ctx, p[0], NV, 0.0, stream));
    TRY(vec_fill_f64(ctx, p[1], NV, 0.0, stream));
    for (auto &e : ev_ready) HIPCHK(ctx, hipEventCreateWithFlags(&e, hipEventDisableTiming));
    HIPCHK(ctx, hipEventCreateWithFlags(&ev_free, hipEventDisableTiming));
    HIPCHK(ctx, hipEventCreateWithFlags(&ev_start, hipEventDisableTiming));

    OpSet *sets[2] = {&H.ops, &O1};
    int cur = 0;
    // ---- assembly
    TRY(rung0(L, stream));
    int published = 0, built = 0;  // highest rung published / whose build is enqueued
    bool ladder_done = L.R == 0;
    if (!lazy) {
        for (int rr = 1; rr <= L.R; ++rr) TRY(rung(L, rr, stream));
        TRY(build(L, H.ops, false, stream));
        published = built = L.R;
        ladder_done = true;
    } else {
        TRY(build(L, H.ops, true, stream));
        HIPCHK(ctx, hipEventRecord(ev_start, stream));
        HIPCHK(ctx, hipStreamWaitEvent(ctx->s_asm, ev_start, 0));
        TRY(rung(L, 1, ctx->s_asm));
        TRY(build(L, O1, false, ctx->s_asm));
        HIPCHK(ctx, hipEventRecord(ev_ready[1], ctx->s_asm));
        built = 1;
        if (L.R >= 2) TRY(rung(L, 2, ctx->s_asm));
    }

    // ---- cycles
    double *s = ctx->scal, r0 = 0.0, rk = 0.0, r_ref = 0.0;
    bool restart = true, pcg = op->outer == MGD_PCG;
    bool deterministic = op->publish == MGD_PUBLISH_DETERMINISTIC;
    double t_first = 0.0, t_loop0 = 0.0;
    int publishes = 0;
    for (k = 0;; ++k) {
        // publish a completed rung at this cycle boundary
        if (lazy && published < built) {
            int next = published + 1;
            bool ready;
            if (deterministic) {
                ready = ncyc >= next;
                if (ready) HIPCHK(ctx, hipEventSynchronize(ev_ready[next]));
            } else {
                hipError_t q = hipEventQuery(ev_ready[next]);
                ready = q == hipSuccess;
                if (q != hipSuccess && q != hipErrorNotReady) HIPCHK(ctx, q);
            }
            if (ready) {
                HIPCHK(ctx, hipStreamWaitEvent(stream, ev_ready[next], 0));
                int old = cur;
                cur = next % 2;
                HIPCHK(ctx, hipEventRecord(ev_free, stream));
                published = next;
                ++publishes;
                restart = true;
                // rung `next` is final when no cell stays open after it
                bool more = next < L.R && L.cnt_host[next + 1] > 0;
                if (more) {
                    HIPCHK(ctx, hipStreamWaitEvent(ctx->s_asm, ev_free, 0));
                    TRY(build(L, *sets[old], false, ctx->s_asm));
                    HIPCHK(ctx, hipEventRecord(ev_ready[next + 1], ctx->s_asm));
                    built = next + 1;
                    if (next + 2 <= L.R) TRY(rung(L, next + 2, ctx->s_asm));
                } else {
                    ladder_done = true;
                }
            }
        }
        const OpSet &O = *sets[cur];
        if (restart || !pcg) {
            TRY(outer_residual(&H, O, u, f, r, s + 4, stream));
            if (pcg) TRY(vec_fill_f64(ctx, s + 7, 1, 1.0, stream));
        }
        HIPCHK(ctx, hipMemcpyAsync(ctx->host_scal, s + 4, 8, hipMemcpyDeviceToHost, stream));
        HIPCHK(ctx, hipStreamSynchronize(stream));
        rk = sqrt(ctx->host_scal[0]);
        if (k == 0) {
            r0 = rk;
            t_first = now_ms() - t0;
            t_loop0 = now_ms();
        }
        if (k == 0 || restart) r_ref = rk > r0 ? rk : r0;
        double rel = r0 > 0.0 ? rk / r0 : 0.0;
        if (k < MGD_HIST) rep->hist[k] = rel;
        if (!(rk <= op->div_factor * r_ref)) { status = MGD_EDIVERGED; break; }
        if (rel <= op->tol) {
            if (ladder_done) { status = MGD_OK; break; }
            // starvation guard: the tolerance was met on a provisional
            // operator; in the asynchronous mode wait for the pending rung and
            // publish it at once, the deterministic mode keeps its schedule
            if (!deterministic && published < built) {
                HIPCHK(ctx, hipEventSynchronize(ev_ready[published + 1]));
                continue;
            }
        }
        if (ncyc >= op->max_cycles) { status = (rel <= op->tol) ? MGD_ESTARVED : MGD_ENOCONV; break; }
        TRY(vec_cast_to_cycle(&H, r, H.f[0], stream));
        TRY(vcycle_ops(&H, O, H.u[0], H.f[0], op->omega, op->nu1, op->nu2, true, stream));
        if (!pcg) {
            TRY(vec_add_cycle(&H, u, H.u[0], stream));
        } else {
            TRY(pcg_beta(&H, H.u[0], r, rold, s, stream));
            TRY(pcg_matvec(&H, O, H.u[0], p[0], p[1], Ap, s, stream));
            TRY(pcg_update(&H, u, p[1], r, rold, Ap, s, stream));
            double *t = p[0]; p[0] = p[1]; p[1] = t;
        }
        ++ncyc;
        restart = false;
    }
    HIPCHK(ctx, hipStreamSynchronize(stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->s_asm));
    double t_end = now_ms();
    rep->status = status;
    rep->cycles = ncyc;
    rep->checks = k + 1 < MGD_HIST ? k + 1 : MGD_HIST;
    rep->nlev = H.nlev;
    rep->publishes = publishes;
    rep->r0 = r0;
    rep->r_final = rk;
    rep->t_total_ms = t_end - t0;
    rep->t_first_cycle_ms = t_first;
    rep->t_cycles_ms = t_end - t_loop0;
    // cells per final s and cell integrations
    if (sf > 0) {
        int b = 0;
        while ((1 << b) < sf) ++b;
        rep->cells_at_s[b] = L.ncell;
        rep->integrations = L.ncell;
    } else {
        rep->integrations = L.ncell;
        for (int rr = 1; rr <= published && rr <= L.R; ++rr) {
            int64_t open_r = L.cnt_host[rr];
            int64_t open_next = rr < L.R ? L.cnt_host[rr + 1] : 0;
            rep->integrations += open_r;
            rep->cells_at_s[rr] = open_r - open_next;
        }
        if (L.R == 0) rep->cells_at_s[0] = L.ncell;
    }
    if (H.precision == MGD_MIXED) {
        const OpSet &O = *sets[cur];
        uint32_t units = 0;
        HIPCHK(ctx, hipMemcpy(&units, O.units_total, 4, hipMemcpyDeviceToHost));
        std::vector<uint8_t> t(O.ntile);
        HIPCHK(ctx, hipMemcpy(t.data(), O.tier, O.ntile, hipMemcpyDeviceToHost));
        for (uint8_t x : t) rep->tier_tiles[x & 3]++;
        // payload + tier byte and offset per tile + centre sample per cell
        rep->store_bytes = (double)units * 64 + (double)O.ntile * 5 + (double)L.ncell * 4;
    } else {
        rep->store_bytes = (double)NV * H.H * 8;
    }
    cleanup();
#undef TRY
    return status;
}
