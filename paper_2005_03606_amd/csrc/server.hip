// Continuous-batching solve server: requests of any grid size and material
// are admitted in arrival order while a slot and device memory are free,
// each runs as a resumable solve on its own stream pair (solve + assembly),
// and all active solves advance together so their kernels overlap on the
// device.  Device state (hierarchy, ladder buffers, operator sets) stays
// resident in a pool and is reused by later requests of the same shape;
// idle states are evicted oldest-first when the memory budget needs room.
#include <algorithm>
#include <chrono>
#include <deque>
#include <unordered_map>
#include <vector>

#include "common.h"
#include "solve.h"

namespace {

double now_ms()
{
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct Request {
    int64_t id = 0;
    int dim = 0, n = 0;
    mgd_eps eps{};
    const double *f = nullptr;
    double *u = nullptr;
    mgd_solve_opts op{};
    mgd_report rep{};
    int state = 0;  // 0 waiting, 1 active, 2 done
    int rc = 0;
    double t_submit = 0, t_admit = 0, t_done = 0;
    SolveState *S = nullptr;
    hipStream_t stream = nullptr;
    hipEvent_t inputs = nullptr;  // recorded on the producer stream at submit
};

}  // namespace

size_t solve_footprint(int dim, int n, int precision, int transfer, int coarsest);

struct mgd_server {
    mgd_ctx *ctx = nullptr;
    int max_slots = 8;
    double budget = 0;
    size_t used = 0;  // bytes of all states (active and idle)
    int64_t next_id = 1;
    std::deque<int64_t> waiting;
    std::vector<int64_t> active;
    std::unordered_map<int64_t, Request> reqs;
    std::vector<SolveState *> idle;  // oldest first
    std::vector<hipStream_t> free_streams;
    std::vector<hipStream_t> all_streams;
    std::vector<hipEvent_t> events;  // free input events
    int64_t completed = 0;
};

static void release_event(mgd_server *sv, Request &r)
{
    if (r.inputs) sv->events.push_back(r.inputs);
    r.inputs = nullptr;
}

static int take_state(mgd_server *sv, Request &r, SolveState **out)
{
    int coarsest = r.op.coarsest < 2 ? 2 : r.op.coarsest;
    for (size_t i = 0; i < sv->idle.size(); ++i)
        if (solve_state_matches(sv->idle[i], r.dim, r.n, r.op.precision, r.op.transfer, coarsest)) {
            *out = sv->idle[i];
            sv->idle.erase(sv->idle.begin() + i);
            return MGD_OK;
        }
    size_t need = solve_footprint(r.dim, r.n, r.op.precision, r.op.transfer, coarsest);
    while (sv->used + need > sv->budget && !sv->idle.empty()) {
        SolveState *old = sv->idle.front();
        sv->idle.erase(sv->idle.begin());
        sv->used -= old->bytes;
        solve_state_free(old);
    }
    if (sv->used + need > sv->budget) return 1;  // not now
    SolveState *S = nullptr;
    int rc = solve_state_create(sv->ctx, r.dim, r.n, r.op.precision, r.op.transfer, coarsest, true, &S);
    if (rc) return rc;
    sv->used += S->bytes;
    *out = S;
    return MGD_OK;
}

static int admit(mgd_server *sv)
{
    while (!sv->waiting.empty() && (int)sv->active.size() < sv->max_slots && !sv->free_streams.empty()) {
        Request &r = sv->reqs[sv->waiting.front()];
        SolveState *S = nullptr;
        int rc = take_state(sv, r, &S);
        if (rc == 1 && sv->active.empty() && sv->idle.empty())
            rc = mgd_fail(sv->ctx, MGD_ENOMEM, "request %lld needs more than the whole budget", (long long)r.id);
        if (rc == 1) break;  // wait for memory
        sv->waiting.pop_front();
        if (rc) {
            release_event(sv, r);
            r.state = 2;
            r.rc = rc;
            r.t_done = now_ms();
            sv->completed++;
            continue;
        }
        r.S = S;
        r.stream = sv->free_streams.back();
        sv->free_streams.pop_back();
        r.t_admit = now_ms();
        rc = hipStreamWaitEvent(r.stream, r.inputs, 0) == hipSuccess
                 ? solve_begin(S, &r.eps, r.f, r.u, &r.op, &r.rep, r.stream)
                 : mgd_fail(sv->ctx, MGD_EHIP, "wait on the producer stream failed");
        if (rc) {
            (void)hipStreamSynchronize(r.stream);
            release_event(sv, r);
            r.state = 2;
            r.rc = rc;
            r.t_done = now_ms();
            sv->free_streams.push_back(r.stream);
            sv->idle.push_back(S);
            sv->completed++;
            continue;
        }
        r.state = 1;
        sv->active.push_back(r.id);
    }
    return MGD_OK;
}

extern "C" {

int mgd_server_create(mgd_ctx *ctx, const mgd_server_opts *o, mgd_server **out)
{
    if (!ctx || !o || !out) return MGD_EINVAL;
    *out = nullptr;
    if (o->max_slots < 1 || o->max_slots > 64 || !(o->hbm_budget_bytes > 0))
        return mgd_fail(ctx, MGD_EINVAL, "max_slots must be in [1,64] and the budget positive");
    HIPCHK(ctx, hipSetDevice(ctx->device));
    mgd_server *sv = new mgd_server();
    sv->ctx = ctx;
    sv->max_slots = o->max_slots;
    sv->budget = o->hbm_budget_bytes;
    for (int i = 0; i < o->max_slots; ++i) {
        hipStream_t s;
        if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
            mgd_server_destroy(sv);
            return mgd_fail(ctx, MGD_EHIP, "stream creation failed");
        }
        sv->all_streams.push_back(s);
        sv->free_streams.push_back(s);
    }
    *out = sv;
    return MGD_OK;
}

int mgd_server_destroy(mgd_server *sv)
{
    if (!sv) return MGD_OK;
    (void)hipSetDevice(sv->ctx->device);
    for (auto &kv : sv->reqs)
        if (kv.second.S) {
            (void)solve_end(kv.second.S);
            solve_state_free(kv.second.S);
            kv.second.S = nullptr;
        }
    for (SolveState *S : sv->idle) solve_state_free(S);
    for (auto &kv : sv->reqs) release_event(sv, kv.second);
    for (hipEvent_t e : sv->events) (void)hipEventDestroy(e);
    for (hipStream_t s : sv->all_streams) {
        (void)hipStreamSynchronize(s);
        (void)hipStreamDestroy(s);
    }
    delete sv;
    return MGD_OK;
}

int mgd_server_submit(mgd_server *sv, int32_t dim, int32_t n, const mgd_eps *eps, const double *f, double *u,
                      const mgd_solve_opts *op, hipStream_t producer, int64_t *ticket)
{
    if (!sv || !ticket) return MGD_EINVAL;
    int rc = solve_validate(sv->ctx, dim, n, eps, f, u, op);
    if (rc) return rc;
    hipEvent_t ev = nullptr;
    if (!sv->events.empty()) {
        ev = sv->events.back();
        sv->events.pop_back();
    } else if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
        return mgd_fail(sv->ctx, MGD_EHIP, "event creation failed");
    }
    if (hipEventRecord(ev, producer) != hipSuccess) {
        sv->events.push_back(ev);
        return mgd_fail(sv->ctx, MGD_EHIP, "event record on the producer stream failed");
    }
    Request r;
    r.inputs = ev;
    r.id = sv->next_id++;
    r.dim = dim;
    r.n = n;
    r.eps = *eps;
    r.f = f;
    r.u = u;
    r.op = *op;
    r.t_submit = now_ms();
    sv->reqs[r.id] = r;
    sv->waiting.push_back(r.id);
    *ticket = r.id;
    return admit(sv);
}

int mgd_server_poll(mgd_server *sv, int32_t *n_active, int32_t *n_waiting)
{
    if (!sv) return MGD_EINVAL;
    int finished = 0;
    for (size_t i = 0; i < sv->active.size();) {
        Request &r = sv->reqs[sv->active[i]];
        int st = solve_step(r.S, false);
        if (st == 0 || st == 2) {
            ++i;
            continue;
        }
        r.rc = st < 0 ? st : r.rep.status;
        (void)solve_end(r.S);
        release_event(sv, r);
        r.t_done = now_ms();
        r.state = 2;
        sv->idle.push_back(r.S);
        r.S = nullptr;
        sv->free_streams.push_back(r.stream);
        r.stream = nullptr;
        sv->active.erase(sv->active.begin() + i);
        sv->completed++;
        ++finished;
    }
    int rc = admit(sv);
    if (rc) return rc;
    if (n_active) *n_active = (int32_t)sv->active.size();
    if (n_waiting) *n_waiting = (int32_t)sv->waiting.size();
    return finished;
}

int mgd_server_result(mgd_server *sv, int64_t ticket, mgd_report *rep, double *times_ms)
{
    if (!sv) return MGD_EINVAL;
    auto it = sv->reqs.find(ticket);
    if (it == sv->reqs.end()) return mgd_fail(sv->ctx, MGD_EINVAL, "unknown ticket");
    Request &r = it->second;
    if (r.state != 2) return 0;
    if (rep) {
        *rep = r.rep;
        rep->status = r.rc;
    }
    if (times_ms) {
        times_ms[0] = r.t_submit;
        times_ms[1] = r.t_admit;
        times_ms[2] = r.t_done;
    }
    sv->reqs.erase(it);
    return 1;
}

int mgd_server_stats(const mgd_server *sv, int64_t *completed, double *resident_bytes, int32_t *idle_states)
{
    if (!sv) return MGD_EINVAL;
    if (completed) *completed = sv->completed;
    if (resident_bytes) *resident_bytes = (double)sv->used;
    if (idle_states) *idle_states = (int32_t)sv->idle.size();
    return MGD_OK;
}

int mgd_solve_footprint(int32_t dim, int32_t n, const mgd_solve_opts *op, double *bytes)
{
    if (!op || !bytes || (dim != 2 && dim != 3) || n < 2) return MGD_EINVAL;
    *bytes = (double)solve_footprint(dim, n, op->precision, op->transfer, op->coarsest < 2 ? 2 : op->coarsest);
    return MGD_OK;
}

}  // extern "C"
