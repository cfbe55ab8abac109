/*
 * mgdelay.h -- C ABI of the MI355X (gfx950) library for delayed approximate
 * matrix assembly in multigrid with dynamic precisions (Murray & Weinzierl,
 * arXiv:2005.03606).
 *
 * Problem: -div(eps grad u) = f on the unit square / cube, homogeneous
 * Dirichlet conditions, d-linear (Q1) finite elements on N^d equal cells
 * (Sec. 4: nodal Ritz-Galerkin, 9- / 27-point stencils).
 *
 * Conventions shared by every entry point
 *   - cell c = i + N (j + N k), vertex v = i + (N+1)(j + (N+1) k), x fastest;
 *     NV = (N+1)^d; vectors hold every vertex, boundary entries are 0;
 *   - local vertex a of a cell has bit m = offset along axis m;
 *   - element matrices are stored by their off-diagonal upper triangle,
 *     pairs (a,b), a < b, row-major: U = 6 (2D) or 28 (3D) entries per cell.
 *     Rows sum to zero (sum_a phi_a = 1), so K[a][a] = -sum_{b != a} K[a][b];
 *   - stencils are stored as upper-half couplings: for stencil offset index
 *     sum_m (o_m+1) 3^m above the centre (4 in 2D, 9 in 3D is the centre),
 *     H = 4 (2D) / 13 (3D) slots, slot-major arrays [H][NV]; the coupling
 *     of v to v - o is slot o of vertex v - o (symmetry), and the diagonal
 *     is minus the sum of all off-diagonal couplings of the row;
 *   - all pointers marked (dev) are device memory owned by the caller; the
 *     library keeps no reference to them after the call returns;
 *   - calls are asynchronous on the given stream unless stated otherwise;
 *   - every call returns MGD_OK (0) or a negative code; mgd_last_error()
 *     gives a message for the context's last failure.  Argument errors are
 *     detected before any work is enqueued.
 */
#ifndef MGDELAY_H
#define MGDELAY_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    MGD_OK = 0,
    MGD_EINVAL = -1,    /* bad argument: shape, size, mode or null pointer */
    MGD_ENOMEM = -2,    /* device allocation failed */
    MGD_EHIP = -3,      /* a HIP runtime call failed */
    MGD_ENOCONV = -4,   /* max_cycles reached before the tolerance */
    MGD_EDIVERGED = -5, /* stationary: residual above div_factor x reference; CG: non-finite */
    MGD_ESTARVED = -6   /* tolerance met but the assembly never completed */
};

enum { MGD_FP64 = 0, MGD_MIXED = 1 };          /* precision of a path */
enum { MGD_GEOMETRIC = 0, MGD_BOXMG = 1 };     /* transfer operators */
enum { MGD_STATIONARY = 0, MGD_PCG = 1 };      /* FP64 outer iteration */
enum { MGD_UPFRONT = 0, MGD_LAZY = 1 };        /* assembly schedule */
enum { MGD_PUBLISH_ASYNC = 0, MGD_PUBLISH_DETERMINISTIC = 1, MGD_PUBLISH_EVERY = 2 };
enum { MGD_STORE_AUTO = 0, MGD_STORE_DECODE = 1, MGD_STORE_COPY = 2 }; /* finest-level source */
enum { MGD_START_CARRY = 0, MGD_START_BEST = 1 }; /* iterate after an operator change */
enum { MGD_CYCLE_V = 0, MGD_CYCLE_ADAFAC_PI = 1, MGD_CYCLE_ADAFAC_JAC = 2 }; /* correction cycle */

typedef struct mgd_ctx mgd_ctx;   /* per-device context: streams, scratch */
typedef struct mgd_hier mgd_hier; /* device-resident multigrid hierarchy */

/* Context on HIP device `device`.  Owns the assembly stream of mgd_solve
 * and the cached workspace of the last mgd_solve shape; destroy with
 * mgd_destroy. */
int mgd_create(mgd_ctx **ctx, int device);
int mgd_destroy(mgd_ctx *ctx);
const char *mgd_last_error(const mgd_ctx *ctx);
/* library build identification (static string) */
const char *mgd_version(void);

/* ------------------------------------------------------------------------
 * Material description.  eps(x) is evaluated at sub-cell midpoints
 * x_q = ((i + (q_x + 1/2)/s)/N, ...), q = q_x + s (q_y + s q_z).
 *   MGD_EPS_CONST   eps = p0
 *   MGD_EPS_SINE    eps = 1 + p0 prod_m sin(2 pi x_m)
 *   MGD_EPS_THETA   eps = 1 + (0.3/d) prod_m exp(-p0 x_m) cos(pi p0 x_m)
 *                   (results section, eq. results:theta-setup)
 *   MGD_EPS_BALLS   eps = p1 inside any ball (|x-c|^2 <= r^2), else p0;
 *                   data (dev) = count rows (c_0..c_{d-1}, r)
 *   MGD_EPS_LATTICE eps = exp(p0 g(x)), g d-linear in lattice values on a
 *                   (count+1)^d vertex lattice of spacing 1/count, x fastest
 *   MGD_EPS_BOXES   eps = value of the last box with lo_m <= x_m < hi_m for
 *                   all m, else p0; data (dev) = count rows (lo.., hi.., eps)
 *   MGD_EPS_SAMPLES data (dev) = explicit samples [cells][s^d] (assemble
 *                   only; row i belongs to the i-th listed cell)
 * ---------------------------------------------------------------------- */
enum {
    MGD_EPS_CONST = 0, MGD_EPS_SINE = 1, MGD_EPS_THETA = 2, MGD_EPS_BALLS = 3,
    MGD_EPS_LATTICE = 4, MGD_EPS_BOXES = 5, MGD_EPS_SAMPLES = 6
};
typedef struct {
    int32_t kind, dim, count, pad;
    double p0, p1;
    const double *data;
} mgd_eps;

/* (1) Element integration, Sec. 4.2 eq. (mg:weak-form-of-assembly): eps held
 * constant on each of the s^d equal sub-cells (s = 1: one centre sample),
 * the gradient products integrated exactly on each sub-cell:
 *     K_c = sum_q eps(x_q) G_q.
 * dim 2 or 3; n >= 1 cells per axis; s in {1,2,4,8,16}.
 * cells (dev, int64 [count]) lists the cells, or NULL for all n^d in order.
 * mode MGD_FP64: FP64 samples and arithmetic, K_out double [count][U].
 * mode MGD_MIXED: eps split into bf16 hi+lo, contracted with the exactly
 *   split integer-scaled G table on MFMA with FP32 accumulation, K_out
 *   float [count][U].
 * Optional adaptive criterion, Sec. 5.2 eq. (termination criterion): when
 * K_old (dev, same type and layout as K_out) is given, rel_out[i] (dev
 * double, may be NULL) receives ||K_new - K_old||_max / ||K_old||_max over
 * the full 2^d x 2^d matrices and done_out[i] (dev uint8, may be NULL)
 * receives 1 if rel < C, else 0. */
int mgd_assemble_cells(mgd_ctx *ctx, int32_t dim, int32_t n, int32_t s,
                       const int64_t *cells, int64_t count, const mgd_eps *eps,
                       int32_t mode, void *K_out, const void *K_old, double C,
                       double *rel_out, uint8_t *done_out, hipStream_t stream);

/* (1p) The paper's own ladder step, n -> n + 1 (Sec. 5.2, with the older
 * matrix kept on convergence: the reading under which Table
 * memory-footprint's theta = 1 row stays at n = 1): for each listed cell c,
 * the element matrix with s^d samples (FP64, any s in 1..16) is compared
 * with the row K[c], which holds the cell's matrix with (s - 1)^d samples;
 * rel = ||K_new - K[c]||_max / ||K[c]||_max over the full 2^d x 2^d
 * matrices.  rel < C: the cell is done and K[c] keeps the older matrix;
 * else K[c] becomes K_new.  K (dev double [n^d][U], rows by cell id) is
 * read and written in place; cells (dev int64 [count], or NULL for all n^d
 * in order); rel_out (dev double [count], may be NULL); done_out (dev uint8
 * [count], may be NULL) gets 1 for done.  eps: any field kind but
 * explicit samples.  Errors: MGD_EINVAL for s outside 1..16 or a bad grid,
 * field or count. */
int mgd_ladder_step_keep(mgd_ctx *ctx, int32_t dim, int32_t n, int32_t s, const int64_t *cells,
                         int64_t count, const mgd_eps *eps, double *K, double C, double *rel_out,
                         uint8_t *done_out, hipStream_t stream);

/* (1q) The paper's flexible-precision format of the hierarchical surplus
 * (Sec. 5.5), cell by cell: E = K - K1 as a full 2^d x 2^d matrix (off the
 * diagonal from the stored pairs, E[a][b] = E[b][a] = K[p] - K1[p]; on it
 * minus the sum of its row's off-diagonal entries, taken in ascending
 * column order, as rows of a stiffness matrix sum to zero).  p3 = 0 when
 * the Frobenius norm of E (squares summed row by row) is below tau; else
 * the fewest bytes p in 2..7 whose encoding keeps every entry within tau of
 * it, or 8 (the double itself).  A p-byte datum (2 <= p <= 7): p - 1 bytes,
 * little-endian, holding the sign in the top bit and the leading
 * 8 (p - 1) - 1 bits of the IEEE fraction (truncated), then one byte with
 * the unbiased exponent as a signed char clamped to [-128, 127]; zero is
 * exponent -128 with a zero fraction.  K, K1: dev double [count][U];
 * p3_out: dev uint8 [count]; bytes_out: dev uint8 [count][2^d 2^d 8], of
 * which a cell's first 2^d 2^d p3 bytes (entries row by row) are written.
 * Errors: MGD_EINVAL for a bad dim, count or tau, or a NULL buffer. */
int mgd_p3_encode(mgd_ctx *ctx, int32_t dim, const double *K, const double *K1, int64_t count, double tau,
                  uint8_t *p3_out, uint8_t *bytes_out, hipStream_t stream);

/* Centre samples eps(x_c) of all n^d cells as FP32 (eps_c_out dev float
 * [n^d]): the s = 1 integration of Sec. 5.2 and the base of the
 * hierarchical surplus (Sec. 5.5) that mgd_compress_stencils subtracts. */
int mgd_centre_samples(mgd_ctx *ctx, int32_t dim, int32_t n, const mgd_eps *eps, float *eps_c_out,
                       hipStream_t stream);

/* (2a) Stencil gather, Sec. 4 (a stencil is one row of A_h): for every
 * vertex and upper slot, the coupling is the sum of K_c[loc v][loc v+o] over
 * the cells holding both, in ascending cell order.  K (dev) holds all n^d
 * cells in order; k_mode MGD_FP64 (double) or MGD_MIXED (float); S_out (dev)
 * [H][NV] in s_mode's type (double / float). */
int mgd_gather_stencils(mgd_ctx *ctx, int32_t dim, int32_t n, const void *K, int32_t k_mode,
                        void *S_out, int32_t s_mode, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Hierarchy.  precision MGD_FP64: every level FP64 half stencils, FP64
 * vectors.  MGD_MIXED: the finest level is the compressed store of (2b),
 * beside it the store's decode (base + surplus summed in FP64, rounded once
 * to FP32: the mixed operator), coarse levels are FP32 half stencils, cycle
 * vectors are FP32.
 * Levels: n_0 = n, halved while even and n/2 >= coarsest (>= 2).
 * store_path (MGD_MIXED, the finest level's sweeps, residuals and CG
 * product): MGD_STORE_DECODE decodes the compressed store in every pass,
 * MGD_STORE_COPY reads the FP32 decode.  MGD_STORE_AUTO (0): in 2D it decodes
 * the store when the finest level has at least 2^22 vertices (streamed from
 * HBM, where the store's fewer bytes set the pace) and reads the FP32 decode
 * on smaller levels (cache-resident between passes, bound by arithmetic); in
 * 3D with n % 4 == 0 the sweeps and residuals re-evaluate the couplings of
 * every four-vertex item whose coupling sources all lie in tier-0 tiles
 * (surplus 0, Sec. 5.5) from the cells' centre samples and read the FP32
 * decode for the other items, and the CG product reads the FP32 decode.
 * Every choice applies the same operator values in the same order and gives
 * the same results bit for bit.
 * ---------------------------------------------------------------------- */
typedef struct {
    int32_t dim, n, precision, transfer, coarsest, store_path;
} mgd_hier_desc;

int mgd_hier_create(mgd_ctx *ctx, const mgd_hier_desc *desc, mgd_hier **out);
int mgd_hier_destroy(mgd_hier *h);
int mgd_hier_levels(const mgd_hier *h);
int mgd_hier_level_n(const mgd_hier *h, int level);

/* FP64 form: install fine half stencils S (dev double [H][NV]). */
int mgd_hier_set_fine(mgd_ctx *ctx, mgd_hier *h, const double *S, hipStream_t stream);

/* (2b) Hierarchical surplus store, Sec. 5.5.  For a MGD_MIXED hierarchy:
 * S32 (dev float [H][NV]) are the gathered fine couplings, eps_c (dev float
 * [n^d]) the centre samples.  Per vertex v and slot j,
 *   base = ((sum of (double)eps_c over the cells holding v and v+o,
 *            ascending) * k(o)) * h^{d-2}
 * with k(o) the unit-eps Q1 coupling (2D -1/6 face, -1/3 diagonal; 3D 0
 * face, -1/12 edge and corner), and delta = (float)((double)S32 - base).
 * Tier per vertex: the cheapest of {0: nothing stored} u [min_tier,max_tier]
 * (1 FP8 E4M3FN, 2 binary16, 3 binary32) whose max error over the stencil
 * is <= tau = max(tau_abs, tau_rel * ref_v), ref_v = (sum of eps_c around v)
 * * h^{d-2}; falling back to max_tier.  Tiles of 64 consecutive vertices take
 * the largest tier of their vertices; each vertex is encoded at its tile's
 * tier with an E8M0 scale 2^e, e the smallest exponent with
 * max|delta| <= fmax(tier) 2^e (fmax 448 / 65504), round-to-nearest-even,
 * saturating.  Tile payload (tier > 0), 64-byte aligned: 64 scale bytes
 * (e + 127), then for each slot j the 64 entries of the tile (1/2/4 bytes
 * each).  Tile offsets are in 64-byte units, in tile order. */
typedef struct {
    int32_t min_tier, max_tier;
    double tau_abs, tau_rel;
} mgd_tier_policy;

int mgd_compress_stencils(mgd_ctx *ctx, mgd_hier *h, const float *S32, const float *eps_c,
                          const mgd_tier_policy *policy, hipStream_t stream);

/* Allocation-free variant of mgd_compress_stencils, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): same arguments, same store bit
 * for bit.  mgd_compress_stencils allocates its working buffers (surplus
 * [H][NV] FP32 and vertex tiers [NV], 4 H + 1 bytes per level-0 vertex) on
 * its first call on a hierarchy; this variant instead uses a static device
 * array of 64 MiB that every GPU the library runs on holds until the
 * process ends, and calls no allocating routine.  Level 0 may have about
 * 64 MiB / (4 H + 1) vertices at most (2D: 3.9 M, e.g. 1976^2 cells; 3D:
 * 1.26 M, e.g. 107^3 cells), else MGD_EINVAL before any work is enqueued.  All calls on one device share
 * the array (each call overwrites what it uses, nothing is carried over):
 * calls that overlap on one GPU, on different streams or host threads,
 * race and must be ordered by the caller. */
int mgd_compress_stencils_noalloc(mgd_ctx *ctx, mgd_hier *h, const float *S32, const float *eps_c,
                                  const mgd_tier_policy *policy, hipStream_t stream);

/* Transfer weights of a 3D BoxMG hierarchy level (coarsened): the number of
 * 64-vertex tiles of the level and of those whose operator-dependent
 * prolongation equals the d-linear one in every structurally nonzero weight
 * (hierarchical surplus P - P_geo = 0, Sec. 5.5); the restriction and
 * prolongation read no weights there.  Synchronous.  MGD_EINVAL for a 2D or
 * geometric hierarchy or a level without a coarser one. */
int mgd_weight_tiles(mgd_ctx *ctx, const mgd_hier *h, int32_t level, int64_t *ntile, int64_t *geo_tiles);

/* Items of the finest level of a 3D mixed hierarchy as the default sweep
 * takes them (four consecutive vertices of a grid row, x0 = 1 + 4c; n % 4
 * == 0) and how many of them re-evaluate their couplings from the centre
 * samples (Sec. 5.5: every coupling source in a tier-0 tile, i.e. no stored
 * surplus).  Built from the current store on `stream`; synchronous.  0 and 0
 * when n % 4 != 0 (the sweep then reads the decode for every vertex).
 * MGD_EINVAL for a 2D or FP64 hierarchy. */
int mgd_tier0_items(mgd_ctx *ctx, mgd_hier *h, int64_t *items, int64_t *tier0, hipStream_t stream);

/* Copy the compressed store out (dev buffers; pass NULL to skip one):
 * tile_tier uint8 [ntile], tile_off uint32 [ntile], payload (payload_bytes).
 * Host scalars ntile / payload_bytes are returned synchronously. */
int mgd_store_info(mgd_ctx *ctx, const mgd_hier *h, int64_t *ntile, int64_t *payload_bytes,
                   int64_t tier_tiles[4]);
int mgd_store_export(mgd_ctx *ctx, const mgd_hier *h, uint8_t *tile_tier, uint32_t *tile_off,
                     uint8_t *payload, hipStream_t stream);

/* (2c) Galerkin coarse operators A_{l+1} = P^T A_l P for all levels, Sec. 4,
 * with P d-linear (MGD_GEOMETRIC) or operator-dependent (MGD_BOXMG: coarse
 * values injected, other fine values from their own stencil row collapsed
 * onto the line / plane of the interpolating coarse points), R = P^T; then
 * the dense Cholesky factor of the coarsest interior matrix (FP64). */
int mgd_coarsen(mgd_ctx *ctx, mgd_hier *h, hipStream_t stream);

/* Decoded FP64 copy of a level's half stencils (dev double [H][NV_l]) and,
 * for levels above the coarsest, its prolongation weights (dev double
 * [2^d][NV_l], weight of v toward coarse vertex (v_m >> 1) + B_m). */
int mgd_level_stencils(mgd_ctx *ctx, const mgd_hier *h, int level, double *S_out, hipStream_t stream);
int mgd_level_weights(mgd_ctx *ctx, const mgd_hier *h, int level, double *W_out, hipStream_t stream);

/* (3) Multigrid pieces on one level (vectors of the hierarchy's cycle type:
 * double for MGD_FP64, float for MGD_MIXED; [NV_l], boundary entries 0).
 *   smooth:   sweeps x u <- u + omega D^{-1} (f - A u)  (damped Jacobi, Sec. 4.1)
 *   residual: r = f - A u on interior vertices
 *   restrict: fc = P^T r on interior coarse vertices  (level -> level+1)
 *   prolong:  u += P ec on interior fine vertices     (level+1 -> level)
 *   vcycle:   u <- V(nu1,nu2)(u; f) on the finest level: pre-smooth,
 *             residual, restrict, recurse from zero, coarsest dense solve,
 *             prolong, post-smooth (multiplicative correction scheme). */
typedef struct {
    double omega;
    int32_t nu1, nu2;
} mgd_cycle_opts;

int mgd_smooth(mgd_ctx *ctx, mgd_hier *h, int level, void *u, const void *f, int32_t sweeps,
               double omega, hipStream_t stream);
int mgd_residual(mgd_ctx *ctx, mgd_hier *h, int level, const void *u, const void *f, void *r,
                 hipStream_t stream);
int mgd_restrict(mgd_ctx *ctx, mgd_hier *h, int level, const void *r, void *fc, hipStream_t stream);
int mgd_prolong_add(mgd_ctx *ctx, mgd_hier *h, int level, const void *ec, void *u, hipStream_t stream);
int mgd_vcycle(mgd_ctx *ctx, mgd_hier *h, void *u, const void *f, const mgd_cycle_opts *opts,
               hipStream_t stream);
/* Pre-smoothing half of a V(2,.) level in one pass (Sec. 4.1): two damped
 * Jacobi sweeps from u (u = NULL: from zero) into u_out, then the residual
 * r_out = f - A u_out.  u_out must not alias u.  In 2D the level's operator,
 * rhs and iterate cross HBM once (halo-tiled in LDS); in 3D the separate
 * kernels run. */
int mgd_presmooth(mgd_ctx *ctx, mgd_hier *h, int level, const void *u, const void *f, void *u_out, void *r_out,
                  double omega, hipStream_t stream);
/* The same pass followed by the restriction (Sec. 4): fc = P^T (f - A u_out)
 * on level+1 (fc of the coarser level's vector type and size), instead of
 * writing the residual.  This is the finest-to-coarse half of a V(2,.)
 * level as the solver runs it; u_out must not alias u.  2D only. */
int mgd_presmooth_restrict(mgd_ctx *ctx, mgd_hier *h, int level, const void *u, const void *f, void *u_out,
                           void *fc, double omega, hipStream_t stream);

/* FP64 outer residual r = f - A u of the finest operator as stored (the
 * compressed store's decode for MGD_MIXED: base + surplus summed in FP64
 * and rounded once to FP32); u, f, r dev double, FP64 arithmetic. */
int mgd_outer_residual(mgd_ctx *ctx, mgd_hier *h, const double *u, const double *f, double *r,
                       hipStream_t stream);

/* (4) Solve.  Synchronous: returns when the run stops.
 * Assembly: s_fixed > 0 integrates every cell once with that s; otherwise
 * the adaptive ladder s = 1, 2, 4, .., s_max with threshold C (Sec. 5.2).
 * MGD_UPFRONT finishes every cell's ladder before the first cycle;
 * MGD_LAZY starts cycling on the centre-sample operator at once and runs the
 * ladder on a second stream; completed rungs are published (stencils
 * re-gathered, re-compressed, coarse operators recomputed) at cycle
 * boundaries: MGD_PUBLISH_ASYNC runs the whole ladder back to back and
 * publishes the final operator at the first boundary after it is built (one
 * switch); MGD_PUBLISH_EVERY publishes every rung as soon as it is built;
 * MGD_PUBLISH_DETERMINISTIC publishes rung k right before cycle k
 * (reproducible bit for bit).  The solver keeps its state (hierarchy,
 * ladder buffers) in the context between calls of the same shape.
 * Outer FP64 iteration: MGD_STATIONARY u += V(f - A u), or MGD_PCG
 * conjugate gradients with one V-cycle as preconditioner (Polak-Ribiere
 * beta, restarted at every publish).  Stops when every cell's ladder is final
 * and published and ||f - A u||_2 / ||r_0||_2 <= tol (interior vertices,
 * r_0 at cycle 0, Sec. 6); MGD_EDIVERGED when the residual of the
 * stationary iteration exceeds div_factor times the residual at the last
 * operator change, or when a CG residual is not finite (the CG residual
 * norm is not monotone: its transients grow with the condition number).
 * prov_tol (MGD_LAZY with MGD_PUBLISH_ASYNC or MGD_PUBLISH_EVERY): once the
 * residual on a provisional operator has dropped to prov_tol times the
 * residual at the last operator change, the solver stops cycling on it and
 * waits for the pending operator, leaving the device to the assembly stream
 * (a provisional operator's solution is no closer to the final one than the
 * operator is to the final operator); 0 cycles on until the publish.
 * prov_growth (same modes): once the residual on a provisional operator
 * exceeds prov_growth times the residual at the last operator change, the
 * solver likewise stops cycling on it and waits for the pending operator:
 * cycles that raise the residual only take compute units from the assembly
 * (a contrast the provisional operator's coarse levels cannot follow makes
 * its cycles diverge); the iterate is carried over as usual.  0 (the
 * default) keeps cycling; a value above 1 leaves room for the CG residual's
 * transients.
 * store_path: as for a hierarchy (MGD_MIXED).
 * start: the iterate after an operator change.  MGD_START_CARRY (0, the
 * paper's schedule, Sec. 5.1-5.3) carries it over; MGD_START_BEST keeps the
 * carried iterate unless its residual on the new operator exceeds that of
 * the zero start (interior set to zero, boundary values kept), and then
 * continues from the zero start (decided on the device).
 * cycle: the correction applied per outer iteration.  MGD_CYCLE_V is the
 * multiplicative V(nu1,nu2); MGD_CYCLE_ADAFAC_PI and MGD_CYCLE_ADAFAC_JAC are
 * the additive adaFAC-x cycle of Sec. 4.1 eq. (mg:adaFAC-x): the residual
 * restricted to every level, each level's damped Jacobi update minus an
 * auxiliary coarse step (PI: injection and P; Jac: the prolongation smoothed
 * by one damped Jacobi step and its transpose), exact coarsest solve, the
 * updates summed through the prolongations.  The additive cycles need
 * outer = MGD_STATIONARY (adaFAC-PI is not symmetric).
 * f (dev double [NV]) is the load vector; u (dev double [NV]) is the initial
 * guess on entry and the solution on return. */
typedef struct {
    int32_t precision, transfer, outer, schedule;
    int32_t publish, s_fixed, s_max, nu1;
    int32_t nu2, max_cycles, coarsest, store_path;
    double C, omega, tol, div_factor;
    mgd_tier_policy tiers;
    double prov_tol;
    int32_t start, cycle;
    double prov_growth;
} mgd_solve_opts;

#define MGD_HIST 512
typedef struct {
    int32_t status, cycles, nlev, publishes;
    int32_t checks, pad;     /* residual checks recorded in hist */
    double r0, r_final;
    int64_t cells_at_s[5];   /* cells whose final s is 1, 2, 4, 8, 16 */
    int64_t integrations;    /* cell integrations performed */
    int64_t tier_tiles[4];   /* fine store tiles per tier at the end */
    double store_bytes;      /* fine operator bytes at the end */
    double t_total_ms;       /* wall time of the call */
    double t_first_cycle_ms; /* wall time until the first cycle was enqueued */
    double t_cycles_ms;      /* wall time spent in the cycle loop */
    double hist[MGD_HIST];   /* normalised residual at the start of each cycle */
} mgd_report;

int mgd_solve(mgd_ctx *ctx, int32_t dim, int32_t n, const mgd_eps *eps, const double *f, double *u,
              const mgd_solve_opts *opts, mgd_report *report, hipStream_t stream);

/* Device bytes that mgd_solve keeps resident for a problem of this shape
 * (hierarchy, both operator sets, ladder buffers, outer vectors). */
int mgd_solve_footprint(int32_t dim, int32_t n, const mgd_solve_opts *opts, double *bytes);

/* ------------------------------------------------------------------------
 * Serving (continuous batching).  Requests of any shape and material are
 * admitted in arrival order whenever one of max_slots slots is free and the
 * device bytes of all resident solve states stay within hbm_budget_bytes;
 * each admitted request runs as an mgd_solve on its own streams and all
 * active ones advance on every mgd_server_poll, so their kernels overlap on
 * the device.  Solve states stay resident after completion and are reused
 * by later requests of the same shape (evicted oldest-first when the budget
 * needs room).  f and u are owned by the caller and must stay valid until
 * mgd_server_result reports the request finished.  Not thread-safe: one host
 * thread drives a server.
 * ---------------------------------------------------------------------- */
typedef struct mgd_server mgd_server;
typedef struct {
    int32_t max_slots, pad;
    double hbm_budget_bytes;
} mgd_server_opts;

int mgd_server_create(mgd_ctx *ctx, const mgd_server_opts *opts, mgd_server **out);
int mgd_server_destroy(mgd_server *srv);
/* Queue a solve (validated now; the descriptors are copied); *ticket
 * identifies it.  The solve runs on a server stream after everything queued
 * on `producer` so far (the writes of f, u and the eps data), so the caller
 * need not synchronise before submitting. */
int mgd_server_submit(mgd_server *srv, int32_t dim, int32_t n, const mgd_eps *eps, const double *f, double *u,
                      const mgd_solve_opts *opts, hipStream_t producer, int64_t *ticket);
/* advance every active solve without blocking, then admit waiting ones;
 * returns the number of solves that finished in this call (or < 0) */
int mgd_server_poll(mgd_server *srv, int32_t *n_active, int32_t *n_waiting);
/* 1 once finished: the report (report->status is the solve's outcome, an
 * MGD_* code such as MGD_ENOMEM for a request larger than the whole budget)
 * and times_ms[3] = submit, admit, done on the host's steady clock in ms;
 * the ticket is then forgotten.  0 while still queued or running; MGD_EINVAL
 * for an unknown ticket. */
int mgd_server_result(mgd_server *srv, int64_t ticket, mgd_report *report, double *times_ms);
int mgd_server_stats(const mgd_server *srv, int64_t *completed, double *resident_bytes, int32_t *idle_states);

#ifdef __cplusplus
}
#endif
#endif /* MGDELAY_H */
