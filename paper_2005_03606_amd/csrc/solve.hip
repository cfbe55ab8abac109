// Solve driver: delayed (lazy) or up-front assembly feeding a multigrid
// solve (paper Sec. 5.1-5.4).  The ladder of sub-sample counts runs on the
// assembly stream; completed rungs become full operator sets (stencils,
// surplus store, coarse operators) in the spare of two operator sets, which
// the solver switches to at a cycle boundary.  A solve is a resumable state
// machine (begin / step) so that several can be interleaved on one device;
// mgd_solve drives one to completion.
#include <math.h>

#include <chrono>

#include <cmath>

#include "common.h"
#include "solve.h"

int store_set_base(mgd_hier *h, OpSet &o, const float *eps_c, hipStream_t st);
int vec_cast_to_cycle(mgd_hier *h, const double *a, void *b, hipStream_t st);
int vec_add_cycle(mgd_hier *h, double *u, const void *e, hipStream_t st);
int vec_fill_f64(mgd_ctx *ctx, double *a, int64_t n, double v, hipStream_t st);

static double now_ms()
{
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// ------------------------------------------------------------ ladder
static void ladder_free(Ladder &L)
{
    dev_free(L.K); dev_free(L.eps_c); dev_free(L.Sg);
    dev_free(L.act[0]); dev_free(L.act[1]); dev_free(L.cnt_dev); dev_free(L.done); dev_free(L.blk);
    if (L.cnt_host) (void)hipHostFree(L.cnt_host);
    L = Ladder();
}

static int ladder_alloc(Ladder &L, mgd_hier *h)
{
    mgd_ctx *ctx = h->ctx;
    int U = n_pairs(h->dim), rc;
    L.h = h;
    L.ncell = 1;
    for (int m = 0; m < h->dim; ++m) L.ncell *= h->n;
    size_t kb = h->precision == MGD_FP64 ? 8 : 4;
    if ((rc = dev_alloc(ctx, &L.K, (size_t)L.ncell * U * kb))) return rc;
    if ((rc = dev_alloc(ctx, (void **)&L.eps_c, (size_t)L.ncell * 4))) return rc;
    if (h->precision == MGD_MIXED)
        if ((rc = dev_alloc(ctx, (void **)&L.Sg, (size_t)h->NV[0] * h->H * 4))) return rc;
    if ((rc = dev_alloc(ctx, (void **)&L.act[0], (size_t)L.ncell * 8))) return rc;
    if ((rc = dev_alloc(ctx, (void **)&L.act[1], (size_t)L.ncell * 8))) return rc;
    if ((rc = dev_alloc(ctx, (void **)&L.cnt_dev, 2 * 8))) return rc;
    if ((rc = dev_alloc(ctx, (void **)&L.done, (size_t)L.ncell))) return rc;
    if ((rc = dev_alloc(ctx, (void **)&L.blk, (size_t)((L.ncell + 255) / 256 + 1) * 4))) return rc;
    if (hipHostMalloc((void **)&L.cnt_host, 8 * 8, hipHostMallocDefault) != hipSuccess)
        return mgd_fail(ctx, MGD_ENOMEM, "pinned allocation failed");
    for (int r = 0; r < 8; ++r) L.cnt_host[r] = 0;
    return MGD_OK;
}

// rung 0: every cell at s_fixed (or the centre sample), plus centre samples
static int rung0(Ladder &L, hipStream_t st)
{
    mgd_ctx *ctx = L.h->ctx;
    int s0 = L.s_fixed > 0 ? L.s_fixed : 1;
    int rc = launch_assemble(ctx, L.h->dim, L.h->n, s0, nullptr, L.ncell, &L.eps, L.h->precision, L.K, nullptr, 0,
                             0.0, nullptr, nullptr, nullptr, st);
    if (rc) return rc;
    for (int r = 0; r < 8; ++r) L.cnt_host[r] = 0;
    L.cnt_host[0] = L.ncell;
    L.cnt_host[1] = L.R >= 1 ? L.ncell : 0;
    // centre samples: the mixed store's base, and the cell values of a lazy
    // solve's provisional geometric hierarchy
    return launch_centre_eps(ctx, L.h->dim, L.h->n, &L.eps, L.eps_c, st);
}

// rung r >= 1: integrate the open cells at s = 2^r in place, criterion
// against the stored matrix, then compact the still-open cells for rung r+1
static int rung(Ladder &L, int r, hipStream_t st)
{
    mgd_ctx *ctx = L.h->ctx;
    const int64_t *cells = r == 1 ? nullptr : L.act[r % 2];
    const int64_t *cnt = r == 1 ? nullptr : L.cnt_dev + (r % 2);
    int rc = launch_assemble(ctx, L.h->dim, L.h->n, 1 << r, cells, L.ncell, &L.eps, L.h->precision, L.K, L.K, 1,
                             L.C, nullptr, L.done, cnt, st);
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
static int build(Ladder &L, OpSet &o, hipStream_t st)
{
    mgd_hier *h = L.h;
    int rc;
    o.dz_ok = 0;
    if (h->precision == MGD_FP64) {
        if ((rc = launch_gather(h->ctx, h->dim, h->n, L.K, MGD_FP64, o.S64[0], MGD_FP64, st))) return rc;
    } else {
        if ((rc = launch_gather(h->ctx, h->dim, h->n, L.K, MGD_MIXED, L.Sg, MGD_MIXED, st))) return rc;
        if ((rc = compress_into(h, o, L.Sg, L.eps_c, &L.tiers, h->delta, h->vtier, st))) return rc;
    }
    return coarsen_ops(h, o, st);
}

// ------------------------------------------------------------ workspace
void solve_state_free(SolveState *S)
{
    if (!S) return;
    (void)hipSetDevice(S->ctx->device);
    if (S->s_asm) (void)hipStreamSynchronize(S->s_asm);
    (void)hipDeviceSynchronize();
    ladder_free(S->L);
    opset_free(S->O1);
    hier_free(&S->H);
    dev_free(S->r); dev_free(S->rold); dev_free(S->p[0]); dev_free(S->p[1]); dev_free(S->Ap);
    for (auto &e : S->ev_ready)
        if (e) (void)hipEventDestroy(e);
    for (hipEvent_t e : {S->ev_free, S->ev_start, S->ev_norm[0], S->ev_norm[1], S->ev_final, S->ev_verify})
        if (e) (void)hipEventDestroy(e);
    if (S->own_asm && S->s_asm) (void)hipStreamDestroy(S->s_asm);
    delete S;
}

void solve_cache_free(mgd_ctx *ctx)
{
    if (ctx && ctx->cache) {
        solve_state_free(ctx->cache);
        ctx->cache = nullptr;
    }
}

// allocate the device state of one solve shape
int solve_state_create(mgd_ctx *ctx, int dim, int n, int precision, int transfer, int coarsest, bool own_asm,
                       SolveState **out)
{
    *out = nullptr;
    size_t bytes0 = g_dev_alloc_bytes;
    SolveState *S = new SolveState();
    S->ctx = ctx;
    S->dim = dim; S->n = n; S->precision = precision; S->transfer = transfer; S->coarsest = coarsest;
    mgd_hier &H = S->H;
    H.ctx = ctx;
    H.dim = dim; H.n = n; H.precision = precision; H.transfer = transfer; H.coarsest = coarsest;
    int rc = MGD_OK;
#define CK(x)                      \
    do {                           \
        if ((rc = (x))) {          \
            solve_state_free(S);   \
            return rc;             \
        }                          \
    } while (0)
    CK(hier_alloc_levels(&H));
    if (precision == MGD_MIXED) CK(hier_compress_buffers(&H));
    CK(opset_alloc(&H, S->O1));
    CK(ladder_alloc(S->L, &H));
    int64_t NV = H.NV[0];
    CK(dev_alloc(ctx, (void **)&S->r, NV * 8));
    CK(dev_alloc(ctx, (void **)&S->rold, NV * 8));
    CK(dev_alloc(ctx, (void **)&S->p[0], NV * 8));
    CK(dev_alloc(ctx, (void **)&S->p[1], NV * 8));
    CK(dev_alloc(ctx, (void **)&S->Ap, NV * 8));
    for (auto &e : S->ev_ready)
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) CK(MGD_EHIP);
    for (hipEvent_t *e : {&S->ev_free, &S->ev_start, &S->ev_final})
        if (hipEventCreateWithFlags(e, hipEventDisableTiming) != hipSuccess) CK(MGD_EHIP);
    // the squared residual norms are written by a kernel straight into pinned
    // host memory: the check events release to system scope so the host sees them
    for (hipEvent_t *e : {&S->ev_norm[0], &S->ev_norm[1], &S->ev_verify})
        if (hipEventCreateWithFlags(e, hipEventDisableTiming | hipEventReleaseToSystem) != hipSuccess) CK(MGD_EHIP);
    if (own_asm) {
        if (hipStreamCreateWithFlags(&S->s_asm, hipStreamNonBlocking) != hipSuccess) CK(MGD_EHIP);
        S->own_asm = true;
    } else {
        S->s_asm = ctx->s_asm;
    }
#undef CK
    // null-stream clears of the new buffers must be done before any solve
    // stream (non-blocking) touches them
    if (hipDeviceSynchronize() != hipSuccess) {
        solve_state_free(S);
        return mgd_fail(ctx, MGD_EHIP, "device synchronisation failed");
    }
    S->bytes = g_dev_alloc_bytes - bytes0;
    *out = S;
    return MGD_OK;
}

bool solve_state_matches(const SolveState *S, int dim, int n, int precision, int transfer, int coarsest)
{
    return S && S->dim == dim && S->n == n && S->precision == precision && S->transfer == transfer &&
           S->coarsest == coarsest;
}

// ------------------------------------------------------------ state machine
int solve_validate(mgd_ctx *ctx, int32_t dim, int32_t n, const mgd_eps *eps, const double *f, const double *u,
                   const mgd_solve_opts *op)
{
    if (!eps || !f || !u || !op) return mgd_fail(ctx, MGD_EINVAL, "null argument");
    if (dim != 2 && dim != 3) return mgd_fail(ctx, MGD_EINVAL, "dim must be 2 or 3");
    if (n < 2) return mgd_fail(ctx, MGD_EINVAL, "n must be >= 2");
    if (eps->kind < MGD_EPS_CONST || eps->kind > MGD_EPS_BOXES || eps->dim != dim)
        return mgd_fail(ctx, MGD_EINVAL, "eps must be a field descriptor of the same dimension");
    if (eps->kind >= MGD_EPS_BALLS && !eps->data) return mgd_fail(ctx, MGD_EINVAL, "eps.data is NULL");
    if (op->precision != MGD_FP64 && op->precision != MGD_MIXED) return mgd_fail(ctx, MGD_EINVAL, "bad precision");
    if (op->transfer != MGD_GEOMETRIC && op->transfer != MGD_BOXMG) return mgd_fail(ctx, MGD_EINVAL, "bad transfer");
    if (op->outer != MGD_STATIONARY && op->outer != MGD_PCG) return mgd_fail(ctx, MGD_EINVAL, "bad outer");
    if (op->schedule != MGD_UPFRONT && op->schedule != MGD_LAZY) return mgd_fail(ctx, MGD_EINVAL, "bad schedule");
    if (op->publish < MGD_PUBLISH_ASYNC || op->publish > MGD_PUBLISH_EVERY)
        return mgd_fail(ctx, MGD_EINVAL, "bad publish mode");
    if (op->store_path < MGD_STORE_AUTO || op->store_path > MGD_STORE_COPY)
        return mgd_fail(ctx, MGD_EINVAL, "bad store_path");
    if (op->start != MGD_START_CARRY && op->start != MGD_START_BEST) return mgd_fail(ctx, MGD_EINVAL, "bad start");
    if (op->cycle < MGD_CYCLE_V || op->cycle > MGD_CYCLE_ADAFAC_JAC) return mgd_fail(ctx, MGD_EINVAL, "bad cycle");
    if (op->cycle != MGD_CYCLE_V && op->outer != MGD_STATIONARY)
        return mgd_fail(ctx, MGD_EINVAL, "the additive adaFAC cycles need the stationary outer iteration");
    int sf = op->s_fixed, sm = op->s_max;
    if (sf > 0 && sf != 1 && sf != 2 && sf != 4 && sf != 8 && sf != 16) return mgd_fail(ctx, MGD_EINVAL, "bad s_fixed");
    if (sf <= 0 && sm != 1 && sm != 2 && sm != 4 && sm != 8 && sm != 16) return mgd_fail(ctx, MGD_EINVAL, "bad s_max");
    if (op->nu1 < 0 || op->nu2 < 0 || op->max_cycles < 0 || !(op->tol >= 0.0) || !(op->div_factor > 0.0) ||
        !(op->prov_tol >= 0.0) || !(op->prov_growth >= 0.0))
        return mgd_fail(ctx, MGD_EINVAL, "bad cycle options");
    if (op->precision == MGD_MIXED &&
        (op->tiers.min_tier < 1 || op->tiers.max_tier > 3 || op->tiers.min_tier > op->tiers.max_tier ||
         !(op->tiers.tau_abs >= 0.0) || !(op->tiers.tau_rel >= 0.0)))
        return mgd_fail(ctx, MGD_EINVAL, "bad tier policy");
    return MGD_OK;
}

// enqueue residual check kq (outer residual after an operator change or for
// the stationary iteration, else the CG recursion's, whose partials the
// update kernel already left in h->partial); its squared norm lands in slot
// kq & 1, read by the host once ev_norm[kq & 1] has completed
static int enqueue_check(SolveState *S, int nparts)
{
    mgd_ctx *ctx = S->ctx;
    mgd_hier &H = S->H;
    int rc;
    const bool true_res = S->restart || !S->pcg || nparts == 0;
    S->chk_true[S->kq & 1] = true_res;
    if (true_res) {
        if ((rc = outer_residual(&H, *S->sets[S->cur], S->u, S->f, S->r, &nparts, S->stream))) return rc;
        if (S->pcg && S->restart && (rc = vec_fill_f64(ctx, H.scal + 7, 1, 1.0, S->stream))) return rc;
    }
    const int slot = S->kq & 1;
    if (S->restart && S->kq > 0 && S->op.start == MGD_START_BEST) {
        // an operator change under the optional start rule: the carried
        // iterate or the zero start (the CG direction and product vectors
        // restart too: free as scratch)
        if ((rc = restart_pick(&H, *S->sets[S->cur], nparts, slot, S->f, S->u, S->r, S->p[0], S->Ap, S->stream)))
            return rc;
    } else if ((rc = check_sum(&H, nparts, slot, S->stream))) {
        return rc;
    }
    HIPCHK(ctx, hipEventRecord(S->ev_norm[slot], S->stream));
    S->kq++;
    return MGD_OK;
}

static int boundary_publish(SolveState *S, bool force_wait);
static void finish(SolveState *S);

// one preconditioned cycle with the current operator and its residual check;
// `gated`: queued before the previous check was read, so the update is
// skipped on the device if that check met the tolerance
static int enqueue_cycle(SolveState *S, bool gated)
{
    mgd_hier &H = S->H;
    const mgd_solve_opts &op = S->op;
    const OpSet &O = *S->sets[S->cur];
    hipStream_t st = S->stream;
    int rc;
    // rhs of the correction cycle: the FP64 residual itself, or the FP32 copy
    // that the kernels producing r write beside it
    const void *rhs = H.precision == MGD_FP64 ? (const void *)S->r : (const void *)H.f[0];
    void *z = nullptr;
    bool dots_done = false;
    int nparts = 0;
    Lev2Dots dots{S->r, S->rold, H.scal};
    if (op.cycle != MGD_CYCLE_V) {
        if ((rc = adafac_ops(&H, O, rhs, op.omega, op.cycle, &z, st))) return rc;
    } else if ((rc = vcycle_ops(&H, O, H.u[0], rhs, op.omega, op.nu1, op.nu2, true, st, S->pcg ? &dots : nullptr,
                                &z, &dots_done))) {
        return rc;
    }
    if (!S->pcg) {
        if ((rc = vec_add_cycle(&H, S->u, z, st))) return rc;
    } else {
        if (!dots_done && (rc = pcg_dots(&H, z, S->r, S->rold, st))) return rc;
        CgScalars c{H.scal, H.p1, H.p1_n, 8 + (S->ncyc & 1), 8 + ((S->ncyc + 1) & 1)};
        if ((rc = pcg_matvec(&H, O, z, S->p[0], S->p[1], S->Ap, c, st))) return rc;
        if ((rc = pcg_update(&H, S->u, S->p[1], S->r, S->rold, S->Ap, c, gated ? S->kq - 1 : -1, S->thr, &nparts,
                             st)))
            return rc;
        double *t = S->p[0];
        S->p[0] = S->p[1];
        S->p[1] = t;
    }
    S->ncyc++;
    S->restart = false;
    if ((rc = boundary_publish(S, false))) return rc;
    return enqueue_check(S, nparts);
}

// switch the solver to operator set `set`, built for rung `rung_no`
static int publish(SolveState *S, int rung_no, int set, hipEvent_t ready)
{
    mgd_ctx *ctx = S->ctx;
    HIPCHK(ctx, hipStreamWaitEvent(S->stream, ready, 0));
    S->cur = set;
    HIPCHK(ctx, hipEventRecord(S->ev_free, S->stream));
    S->published = rung_no;
    S->publishes++;
    S->restart = true;
    return MGD_OK;
}

// per-rung schedules: after publishing rung r, start the build of rung r+1
static int chain_next(SolveState *S)
{
    Ladder &L = S->L;
    int r = S->published;
    bool more = r < L.R && L.cnt_host[r + 1] > 0;
    if (!more) {
        S->ladder_done = true;
        return MGD_OK;
    }
    int rc;
    HIPCHK(S->ctx, hipStreamWaitEvent(S->s_asm, S->ev_free, 0));
    if ((rc = build(L, *S->sets[1 - S->cur], S->s_asm))) return rc;
    HIPCHK(S->ctx, hipEventRecord(S->ev_ready[r + 1], S->s_asm));
    S->built = r + 1;
    if (r + 2 <= L.R && (rc = rung(L, r + 2, S->s_asm))) return rc;
    return MGD_OK;
}

// publish at a cycle boundary if the schedule allows it
static int boundary_publish(SolveState *S, bool force_wait)
{
    if (!S->lazy || S->ladder_done) return MGD_OK;
    mgd_ctx *ctx = S->ctx;
    int rc;
    if (S->publish_mode == MGD_PUBLISH_ASYNC) {
        if (force_wait) HIPCHK(ctx, hipEventSynchronize(S->ev_final));
        hipError_t q = hipEventQuery(S->ev_final);
        if (q == hipErrorNotReady) return MGD_OK;
        HIPCHK(ctx, q);
        if ((rc = publish(S, S->L.R, 1 - S->cur, S->ev_final))) return rc;
        S->ladder_done = true;
        return MGD_OK;
    }
    if (S->published >= S->built) return MGD_OK;
    int next = S->published + 1;
    bool ready;
    if (S->publish_mode == MGD_PUBLISH_DETERMINISTIC) {
        ready = S->ncyc >= next;
        if (ready) HIPCHK(ctx, hipEventSynchronize(S->ev_ready[next]));
    } else {
        if (force_wait) HIPCHK(ctx, hipEventSynchronize(S->ev_ready[next]));
        hipError_t q = hipEventQuery(S->ev_ready[next]);
        ready = q == hipSuccess;
        if (q != hipSuccess && q != hipErrorNotReady) HIPCHK(ctx, q);
    }
    if (!ready) return MGD_OK;
    if ((rc = publish(S, next, next % 2, S->ev_ready[next]))) return rc;
    return chain_next(S);
}

// the provisional operator has done its part: publish the pending one once
// it is built and measure the residual against it (2 while it is not built
// and the caller does not block)
static int await_publish(SolveState *S, bool blocking)
{
    mgd_ctx *ctx = S->ctx;
    hipEvent_t ev = S->publish_mode == MGD_PUBLISH_ASYNC ? S->ev_final : S->ev_ready[S->published + 1];
    if (blocking) {
        HIPCHK(ctx, hipEventSynchronize(ev));
    } else {
        hipError_t q = hipEventQuery(ev);
        if (q == hipErrorNotReady) {
            S->parked = true;
            return 2;
        }
        HIPCHK(ctx, q);
    }
    S->parked = false;
    int rc;
    if ((rc = boundary_publish(S, true))) return rc;
    S->k++;
    if ((rc = enqueue_check(S, 0))) return rc;
    return 0;
}


// The stopping rule is on f - A u (Sec. 6).  A CG convergence read from the
// recursion's residual, which drifts from f - A u by rounding, is confirmed
// with the residual itself (check slot 2); if that is still above the
// tolerance, CG restarts from it (beta = 0) and the iteration goes on.
static int verify_finish(SolveState *S, bool blocking)
{
    mgd_ctx *ctx = S->ctx;
    if (blocking) {
        hipError_t q;
        while ((q = hipEventQuery(S->ev_verify)) == hipErrorNotReady) {
        }
        HIPCHK(ctx, q);
    } else {
        hipError_t q = hipEventQuery(S->ev_verify);
        if (q == hipErrorNotReady) return 2;
        HIPCHK(ctx, q);
    }
    S->verifying = false;
    const double rr = S->H.host_part[2];
    if (rr <= S->thr) {
        S->rk = sqrt(rr);
        S->status = MGD_OK;
        finish(S);
        return 1;
    }
    // the recursion converged but f - A u did not: restart CG from the true
    // residual now in r (and its cycle-type copy); a check queued beyond the
    // converged one (a gated cycle's) is superseded by the next cycle's
    int rc;
    if ((rc = vec_fill_f64(ctx, S->H.scal + 7, 1, 1.0, S->stream))) return rc;
    S->kq = S->k + 1;
    S->k++;
    if (S->ncyc >= S->op.max_cycles) {
        S->k--;
        S->rk = sqrt(rr);
        S->status = MGD_ENOCONV;
        finish(S);
        return 1;
    }
    if ((rc = enqueue_cycle(S, false))) return rc;
    return 0;
}

static int verify_begin(SolveState *S, bool blocking)
{
    mgd_hier &H = S->H;
    int nparts = 0, rc;
    if ((rc = outer_residual(&H, *S->sets[S->cur], S->u, S->f, S->r, &nparts, S->stream))) return rc;
    if ((rc = check_sum(&H, nparts, 2, S->stream))) return rc;
    HIPCHK(S->ctx, hipEventRecord(S->ev_verify, S->stream));
    S->verifying = true;
    return verify_finish(S, blocking);
}


int solve_begin(SolveState *S, const mgd_eps *eps, const double *f, double *u, const mgd_solve_opts *op,
                mgd_report *rep, hipStream_t stream)
{
    mgd_ctx *ctx = S->ctx;
    S->t0 = now_ms();
    S->op = *op;
    S->eps = *eps;
    S->f = f;
    S->u = u;
    S->rep = rep;
    S->stream = stream;
    memset(rep, 0, sizeof(*rep));
    int sf = op->s_fixed, sm = op->s_max;
    S->lazy = op->schedule == MGD_LAZY && sf <= 0 && sm >= 2;
    S->pcg = op->outer == MGD_PCG;
    S->publish_mode = op->publish;
    S->H.store_path = op->store_path;
    S->sets[0] = &S->H.ops;
    S->sets[1] = &S->O1;
    S->cur = 0;
    S->published = S->built = 0;
    S->publishes = 0;
    S->ncyc = 0;
    S->k = 0;
    S->r0 = S->rk = S->r_ref = 0.0;
    S->status = MGD_ENOCONV;
    S->done = false;
    S->parked = false;
    S->verifying = false;
    S->spec = false;
    S->kq = 0;
    S->thr = 0.0;
    S->restart = true;
    S->t_first = S->t_loop0 = 0.0;
    Ladder &L = S->L;
    L.eps = *eps;
    L.s_fixed = sf;
    L.s_max = sf > 0 ? sf : sm;
    L.R = 0;
    if (sf <= 0)
        while ((1 << L.R) < sm) ++L.R;
    L.C = op->C;
    L.tiers = op->tiers;
    S->ladder_done = L.R == 0;
    int64_t NV = S->H.NV[0];
    int rc;
    if ((rc = vec_fill_f64(ctx, S->rold, NV, 0.0, stream)) || (rc = vec_fill_f64(ctx, S->p[0], NV, 0.0, stream)) ||
        (rc = vec_fill_f64(ctx, S->p[1], NV, 0.0, stream)))
        return rc;
    // the assembly stream may still hold work of an earlier solve on this state
    HIPCHK(ctx, hipEventRecord(S->ev_start, S->s_asm));
    HIPCHK(ctx, hipStreamWaitEvent(stream, S->ev_start, 0));
    if ((rc = rung0(L, stream))) return rc;
    if (!S->lazy) {
        for (int rr = 1; rr <= L.R; ++rr)
            if ((rc = rung(L, rr, stream))) return rc;
        if ((rc = build(L, S->H.ops, stream))) return rc;
        S->published = S->built = L.R;
        S->ladder_done = true;
    } else {
        // the provisional operator: the ladder rewrites the element matrices
        // in place, so it starts once the provisional stencils have read them
        // (FP64: the gather; mixed: the centre-sample base needs none) and
        // runs beside the provisional coarsening
        mgd_hier *h = L.h;
        S->H.ops.dz_ok = 0;
        if (h->precision == MGD_FP64)
            rc = launch_gather(ctx, h->dim, h->n, L.K, MGD_FP64, S->H.ops.S64[0], MGD_FP64, stream);
        else
            rc = store_set_base(h, S->H.ops, L.eps_c, stream);
        if (rc) return rc;
        HIPCHK(ctx, hipEventRecord(S->ev_start, stream));
        HIPCHK(ctx, hipStreamWaitEvent(S->s_asm, S->ev_start, 0));
        // geometric coarse levels and transfers for the provisional operator
        // (the cycle vector t[0] is free scratch before the first cycle)
        if ((rc = coarsen_geometric(h, S->H.ops, L.eps_c, (float *)S->H.t[0], stream))) return rc;
        if (S->publish_mode == MGD_PUBLISH_ASYNC) {
            // the whole ladder back to back, then one build of the final operator
            for (int rr = 1; rr <= L.R; ++rr)
                if ((rc = rung(L, rr, S->s_asm))) return rc;
            if ((rc = build(L, S->O1, S->s_asm))) return rc;
            HIPCHK(ctx, hipEventRecord(S->ev_final, S->s_asm));
            S->built = L.R;
        } else {
            if ((rc = rung(L, 1, S->s_asm))) return rc;
            if ((rc = build(L, S->O1, S->s_asm))) return rc;
            HIPCHK(ctx, hipEventRecord(S->ev_ready[1], S->s_asm));
            S->built = 1;
            if (L.R >= 2 && (rc = rung(L, 2, S->s_asm))) return rc;
        }
    }
    return enqueue_check(S, 0);
}

static void finish(SolveState *S)
{
    mgd_report *rep = S->rep;
    Ladder &L = S->L;
    double t_end = now_ms();
    rep->status = S->status;
    rep->cycles = S->ncyc;
    rep->checks = S->k + 1 < MGD_HIST ? S->k + 1 : MGD_HIST;
    rep->nlev = S->H.nlev;
    rep->publishes = S->publishes;
    rep->r0 = S->r0;
    rep->r_final = S->rk;
    rep->t_total_ms = t_end - S->t0;
    rep->t_first_cycle_ms = S->t_first;
    rep->t_cycles_ms = t_end - S->t_loop0;
    int sf = L.s_fixed;
    if (sf > 0) {
        int b = 0;
        while ((1 << b) < sf) ++b;
        rep->cells_at_s[b] = L.ncell;
        rep->integrations = L.ncell;
    } else {
        rep->integrations = L.ncell;
        int top = S->published < L.R ? S->published : L.R;
        for (int rr = 1; rr <= top; ++rr) {
            int64_t open_r = L.cnt_host[rr];
            int64_t open_next = rr < L.R ? L.cnt_host[rr + 1] : 0;
            rep->integrations += open_r;
            rep->cells_at_s[rr] = open_r - open_next;
        }
        if (L.R == 0) rep->cells_at_s[0] = L.ncell;
    }
    mgd_hier &H = S->H;
    const OpSet &O = *S->sets[S->cur];
    if (H.precision == MGD_MIXED) {
        uint32_t units = 0;
        (void)hipMemcpy(&units, O.units_total, 4, hipMemcpyDeviceToHost);
        std::vector<uint8_t> t(O.ntile);
        (void)hipMemcpy(t.data(), O.tier, O.ntile, hipMemcpyDeviceToHost);
        for (uint8_t x : t) rep->tier_tiles[x & 3]++;
        // payload + tier byte and offset per tile + centre sample per cell
        rep->store_bytes = (double)units * 64 + (double)O.ntile * 5 + (double)L.ncell * 4;
    } else {
        rep->store_bytes = (double)H.NV[0] * H.H * 8;
    }
    S->done = true;
}

// one cycle boundary: returns 1 when finished, 0 when more steps follow,
// 2 when the residual is not available yet (non-blocking), < 0 on error
int solve_step(SolveState *S, bool blocking)
{
    if (S->done) return 1;
    if (S->verifying) return verify_finish(S, blocking);
    if (S->parked) return await_publish(S, blocking);
    mgd_ctx *ctx = S->ctx;
    const mgd_solve_opts &op = S->op;
    int rc;
    // with the final operator in place, the next CG cycle is queued before
    // check k is read, so the device does not idle while the host decides;
    // its update is skipped on the device if check k has converged
    if (!S->spec && S->pcg && S->ladder_done && !S->restart && S->k >= 1 && S->kq == S->k + 1 &&
        S->ncyc < op.max_cycles) {
        if ((rc = enqueue_cycle(S, true))) return rc;
        S->spec = true;
    }
    hipEvent_t ev = S->ev_norm[S->k & 1];
    if (blocking) {
        // spin on the event: a sleeping wait wakes tens of microseconds late,
        // and every cycle passes through this point
        hipError_t q;
        while ((q = hipEventQuery(ev)) == hipErrorNotReady) {
        }
        HIPCHK(ctx, q);
    } else {
        hipError_t q = hipEventQuery(ev);
        if (q == hipErrorNotReady) return 2;
        HIPCHK(ctx, q);
    }
    const double rr = S->H.host_part[S->k & 1];
    S->rk = sqrt(rr);
    if (S->k == 0) {
        S->r0 = S->rk;
        S->thr = (op.tol * S->r0) * (op.tol * S->r0);
        S->t_first = now_ms() - S->t0;
        S->t_loop0 = now_ms();
    }
    if (S->k == 0 || S->restart) S->r_ref = S->rk > S->r0 ? S->rk : S->r0;
    double rel = S->r0 > 0.0 ? S->rk / S->r0 : 0.0;
    if (S->k < MGD_HIST) S->rep->hist[S->k] = rel;
    // the device gate of a queued cycle takes the same decision on the same value
    const bool conv = rr <= S->thr;
    // divergence guard of the stationary iteration; the CG residual norm is
    // not monotone (its transients grow with the condition number), so CG
    // stops only on a non-finite residual
    if (S->pcg ? !std::isfinite(S->rk) : !(S->rk <= op.div_factor * S->r_ref)) {
        S->status = MGD_EDIVERGED;
        finish(S);
        return 1;
    }
    if (conv && S->ladder_done) {
        if (S->spec) S->ncyc--;  // the queued cycle made no update
        S->spec = false;
        if (!S->chk_true[S->k & 1]) return verify_begin(S, blocking);
        S->status = MGD_OK;
        finish(S);
        return 1;
    }
    // on a provisional operator, the asynchronous modes stop cycling once the
    // tolerance (starvation guard) or the provisional target is met, or once
    // the cycles have raised the residual past the growth bound, wait for
    // the pending operator and publish it at once; the deterministic mode
    // keeps its schedule
    if (!S->ladder_done && S->publish_mode != MGD_PUBLISH_DETERMINISTIC &&
        (conv || (op.prov_tol > 0.0 && S->rk <= op.prov_tol * S->r_ref) ||
         (op.prov_growth > 0.0 && S->rk > op.prov_growth * S->r_ref)))
        return await_publish(S, blocking);
    S->k++;
    if (S->spec) {  // the next cycle and its check are queued already
        S->spec = false;
        return 0;
    }
    if (S->ncyc >= op.max_cycles) {
        S->k--;
        S->status = conv ? MGD_ESTARVED : MGD_ENOCONV;
        finish(S);
        return 1;
    }
    if ((rc = enqueue_cycle(S, false))) return rc;
    return 0;
}

int solve_end(SolveState *S)
{
    HIPCHK(S->ctx, hipStreamSynchronize(S->stream));
    HIPCHK(S->ctx, hipStreamSynchronize(S->s_asm));
    return MGD_OK;
}

extern "C" int mgd_solve(mgd_ctx *ctx, int32_t dim, int32_t n, const mgd_eps *eps, const double *f, double *u,
                         const mgd_solve_opts *op, mgd_report *rep, hipStream_t stream)
{
    if (!ctx || !rep) return MGD_EINVAL;
    int rc = solve_validate(ctx, dim, n, eps, f, u, op);
    if (rc) return rc;
    HIPCHK(ctx, hipSetDevice(ctx->device));
    double t0 = now_ms();
    int coarsest = op->coarsest < 2 ? 2 : op->coarsest;
    if (!solve_state_matches(ctx->cache, dim, n, op->precision, op->transfer, coarsest)) {
        solve_cache_free(ctx);
        SolveState *S = nullptr;
        if ((rc = solve_state_create(ctx, dim, n, op->precision, op->transfer, coarsest, false, &S))) return rc;
        ctx->cache = S;
    }
    SolveState *S = ctx->cache;
    if ((rc = solve_begin(S, eps, f, u, op, rep, stream))) return rc;
    S->t0 = t0;
    int st;
    while ((st = solve_step(S, true)) == 0) {
    }
    if (st < 0) return st;
    if ((rc = solve_end(S))) return rc;
    rep->t_total_ms = now_ms() - t0;
    return rep->status;
}

// device bytes a solve state of this shape allocates (mirrors the
// allocations of hier_alloc_levels, opset_alloc, ladder_alloc and the CG
// vectors), used for admission before anything is allocated
size_t solve_footprint(int dim, int n, int precision, int transfer, int coarsest)
{
    auto ipow = [](int64_t b, int e) { int64_t r = 1; for (int i = 0; i < e; ++i) r *= b; return r; };
    int H = n_half(dim), U = n_pairs(dim), nlw = 1 << dim;
    size_t vb = precision == MGD_FP64 ? 8 : 4;
    int nl[MGD_MAXLEV], nlev = 0, nn = n;
    nl[nlev++] = nn;
    while (nn % 2 == 0 && nn / 2 >= coarsest && nlev < MGD_MAXLEV) {
        nn /= 2;
        nl[nlev++] = nn;
    }
    int64_t NV0 = ipow(n + 1, dim), ncell = ipow(n, dim), m = ipow(nl[nlev - 1] - 1, dim);
    size_t ops = 0, vec = 0;
    for (int l = 0; l < nlev; ++l) {
        int64_t NV = ipow(nl[l] + 1, dim);
        ops += (size_t)NV * H * vb;
        if (transfer == MGD_BOXMG && l + 1 < nlev) ops += (size_t)NV * nlw * vb;
        if (dim == 3) ops += (size_t)NV * vb;  // zero-start diagonal
        if (dim == 3 && transfer == MGD_BOXMG && l + 1 < nlev) ops += (size_t)(NV + 63) / 64;  // d-linear tile flags
        vec += 4 * (size_t)NV * vb;
    }
    if (precision == MGD_MIXED) {
        int64_t ntile = (NV0 + 63) / 64;
        ops += (size_t)ntile * 5 + (size_t)ntile * (64 + 256 * H) + (size_t)ncell * 4 + 64;
        if (dim == 3 && items4_fit(3, n)) ops += (size_t)(n / 4) * (n + 1) * (n + 1);  // tier-0 item mask
    }
    ops += (size_t)(m > 0 ? m * m : 1) * 8;
    if (m <= kCinvMax) ops += (size_t)(m > 0 ? m * m : 1) * 8;
    size_t hier = ops + vec + (precision == MGD_MIXED ? (size_t)NV0 * H * 4 + NV0 : 0);
    int64_t nb = (NV0 + 255) / 256 + (n + 1) / 4 + 64;
    int64_t pcap = 2 * nb > m + 64 ? 2 * nb : m + 64;
    hier += 2 * (size_t)pcap * 8 + 64 * 8;  // two partial lists, device scalars
    size_t ladder = (size_t)ncell * U * vb + (size_t)ncell * 4 + (precision == MGD_MIXED ? (size_t)NV0 * H * 4 : 0) +
                    2 * (size_t)ncell * 8 + 16 + (size_t)ncell + ((size_t)(ncell + 255) / 256 + 1) * 4;
    size_t cg = 5 * (size_t)NV0 * 8;
    return hier + ops + ladder + cg;
}
