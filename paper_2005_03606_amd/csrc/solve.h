// Per-solve device state and the resumable solve driver.
#pragma once
#include "common.h"

struct Ladder {
    mgd_hier *h = nullptr;
    mgd_eps eps{};
    int s_fixed = 0, s_max = 1, R = 0;  // rungs 1..R use s = 2^r
    double C = 0.01;
    mgd_tier_policy tiers{};
    int64_t ncell = 0;
    void *K = nullptr;            // [ncell][U] current element matrices (in place)
    float *eps_c = nullptr;       // centre samples
    float *Sg = nullptr;          // gathered FP32 couplings (mixed)
    int64_t *act[2] = {nullptr, nullptr};
    int64_t *cnt_dev = nullptr;   // [2]
    uint8_t *done = nullptr;
    int32_t *blk = nullptr;
    int64_t *cnt_host = nullptr;  // pinned [8]: open cells at rung r
};

struct SolveState {
    mgd_ctx *ctx = nullptr;
    int dim = 0, n = 0, precision = 0, transfer = 0, coarsest = 2;
    mgd_hier H;
    OpSet O1;
    Ladder L;
    double *r = nullptr, *rold = nullptr, *p[2] = {nullptr, nullptr}, *Ap = nullptr;
    hipEvent_t ev_ready[8] = {};
    hipEvent_t ev_free = nullptr, ev_start = nullptr, ev_final = nullptr;
    hipEvent_t ev_norm[2] = {nullptr, nullptr};  // residual check k completes ev_norm[k & 1]
    hipEvent_t ev_verify = nullptr;              // the true-residual confirmation completes it
    hipStream_t s_asm = nullptr, stream = nullptr;
    bool own_asm = false;
    size_t bytes = 0;
    // run
    mgd_solve_opts op{};
    mgd_eps eps{};
    const double *f = nullptr;
    double *u = nullptr;
    mgd_report *rep = nullptr;
    OpSet *sets[2] = {nullptr, nullptr};
    int cur = 0, published = 0, built = 0, publishes = 0, ncyc = 0, k = 0, status = 0, publish_mode = 0;
    int kq = 0;         // residual checks queued (check k is read when k < kq)
    bool spec = false;  // a cycle beyond the check being read is already queued
    double thr = 0.0;   // (tol r_0)^2: squared-norm convergence threshold
    bool lazy = false, pcg = false, ladder_done = false, restart = true, done = false;
    bool parked = false;  // done with the provisional operator, waiting for the pending one
    bool verifying = false;  // a CG convergence is being confirmed with f - A u
    bool chk_true[2] = {true, true};  // check k (slot k & 1) measured f - A u, not the CG recursion
    double r0 = 0, rk = 0, r_ref = 0, t0 = 0, t_first = 0, t_loop0 = 0;
};

int solve_validate(mgd_ctx *ctx, int32_t dim, int32_t n, const mgd_eps *eps, const double *f, const double *u,
                   const mgd_solve_opts *op);
int solve_state_create(mgd_ctx *ctx, int dim, int n, int precision, int transfer, int coarsest, bool own_asm,
                       SolveState **out);
void solve_state_free(SolveState *S);
bool solve_state_matches(const SolveState *S, int dim, int n, int precision, int transfer, int coarsest);
int solve_begin(SolveState *S, const mgd_eps *eps, const double *f, double *u, const mgd_solve_opts *op,
                mgd_report *rep, hipStream_t stream);
int solve_step(SolveState *S, bool blocking);
int solve_end(SolveState *S);
void solve_cache_free(mgd_ctx *ctx);
