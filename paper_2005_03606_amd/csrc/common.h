// Shared definitions of the gfx950 library: grid geometry, half-stencil
// layout, compressed-store decoding and the host-side objects.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>
#include <string>
#include <vector>

#include "../../include/mgdelay.h"

#define MGD_MAXLEV 24

// ----------------------------------------------------------------- errors
struct SolveState;
struct mgd_ctx {
    int device = 0;
    int num_cu = 256;
    hipStream_t s_asm = nullptr;  // assembly stream (default priority)
    char err[512] = {0};
    SolveState *cache = nullptr;  // device-resident workspace of the last solve shape
    unsigned char *scratch = nullptr;  // device address of this device's static scratch array
};

int mgd_fail(mgd_ctx *ctx, int code, const char *fmt, ...);
#define HIPCHK(ctx, x)                                                               \
    do {                                                                             \
        hipError_t e_ = (x);                                                         \
        if (e_ != hipSuccess)                                                        \
            return mgd_fail((ctx), MGD_EHIP, "%s failed: %s (%s:%d)", #x,           \
                            hipGetErrorString(e_), __FILE__, __LINE__);              \
    } while (0)

// ------------------------------------------------------------- geometry
__host__ __device__ constexpr int n_half(int D) { return D == 2 ? 4 : 13; }
__host__ __device__ constexpr int n_pairs(int D) { return D == 2 ? 6 : 28; }

// offset component m of half slot j (slot j = stencil index centre+1+j)
__host__ __device__ inline int half_off(int D, int j, int m)
{
    int i = (D == 2 ? 5 : 14) + j;
    for (int k = 0; k < m; ++k) i /= 3;
    return i % 3 - 1;
}

// linear vertex offset of half slot j on a grid with nv vertices per axis
__host__ __device__ inline int64_t half_lin(int D, int j, int64_t nv)
{
    int64_t s = half_off(D, j, 0) + half_off(D, j, 1) * nv;
    if (D == 3) s += (int64_t)half_off(D, j, 2) * nv * nv;
    return s;
}

// pair index of local vertices a < b among the upper off-diagonal entries
__host__ __device__ inline int pair_index(int D, int a, int b)
{
    int nl = 1 << D;
    if (a > b) { int t = a; a = b; b = t; }
    // row a holds nl-1-a entries; rows before a hold sum_{r<a} (nl-1-r)
    return a * (nl - 1) - a * (a - 1) / 2 + (b - a - 1);
}

// workgroups go to the 8 XCDs in turn (block b to XCD b mod 8); this order
// gives each XCD a contiguous range of vertices instead, so in 3D the plane
// below a block was read by the same XCD and its L2 may still hold it
__device__ inline int64_t xcd_block(int64_t b, int64_t nb)
{
    const int64_t q = nb / 8, r = nb % 8, x = b % 8, i = b / 8;
    return x < r ? x * (q + 1) + i : r * (q + 1) + (x - r) * q + i;
}

// the block's index in that order for 3D grids (plain order in 2D, whose
// row neighbours are near in any order)
template <int D> __device__ inline int64_t block_index()
{
    return D == 3 ? xcd_block(blockIdx.x, gridDim.x) : (int64_t)blockIdx.x;
}

// 3D work items of four consecutive vertices of a grid row, x0 = 1 + 4c
// .. x0 + 3, on grids with n % 4 == 0: a row's vertices 1..n are then
// exactly n/4 items (vertex 0 goes with the row's first item; vertex n, on
// the boundary, is its last item's fourth).  The items go to the XCDs by
// slabs of rows: the blocks b with b mod 8 == k take the k-th eighth of the
// y range, plane after plane, so the plane below an item was read by the
// same XCD shortly before and its L2 still holds it (a slab plane of a
// 512^3 grid is 64 x 513 vertices; a whole plane would not fit).  Item i of
// XCD k: c = i mod T, then the slab's row, then the plane.
__host__ __device__ constexpr bool items4_fit(int D, int n) { return D == 3 && n % 4 == 0 && n >= 4 && n <= 4096; }

__device__ inline bool items4_at(int n, uint32_t i, uint32_t k, uint32_t &x0, uint32_t &y, uint32_t &z)
{
    const uint32_t nv = (uint32_t)n + 1u, T = (uint32_t)n >> 2;
    const uint32_t base = nv >> 3, rem = nv & 7u;
    const uint32_t rows = base + (k < rem ? 1u : 0u), y0 = k * base + (k < rem ? k : rem);
    if (i >= T * rows * nv) return false;
    const uint32_t t = i / T;
    x0 = 1u + 4u * (i - t * T);
    z = t / rows;
    y = y0 + (t - z * rows);
    return true;
}

// blocks of 256 threads for one item per thread (a multiple of 8)
static inline unsigned items4_blocks(int n)
{
    const int64_t nv = n + 1, rows_max = nv / 8 + (nv % 8 != 0);
    return (unsigned)(8 * (((int64_t)(n / 4) * rows_max * nv + 255) / 256));
}

template <typename T> __device__ inline void ldv4(const T *p, T *o) { __builtin_memcpy(o, p, 4 * sizeof(T)); }
template <typename T> __device__ inline void ldv2(const T *p, T *o) { __builtin_memcpy(o, p, 2 * sizeof(T)); }
template <typename T> __device__ inline void stv4(T *p, const T *o) { __builtin_memcpy(p, o, 4 * sizeof(T)); }

template <int D> struct Grid {
    int n;      // cells per axis
    int64_t nv; // vertices per axis
    int64_t NV;
    __host__ __device__ Grid(int n_) : n(n_), nv(n_ + 1), NV(1)
    {
        for (int m = 0; m < D; ++m) NV *= nv;
    }
    // 32-bit unsigned division whenever the grid allows it (64-bit integer
    // division is a long software sequence on the GPU)
    __device__ inline void coords(int64_t v, int *x) const
    {
        if (NV <= 0xffffffffLL) {
            const uint32_t vv = (uint32_t)v, m = (uint32_t)nv, t = vv / m;
            x[0] = (int)(vv - t * m);
            if (D == 2) x[1] = (int)t;
            else { const uint32_t t2 = t / m; x[1] = (int)(t - t2 * m); x[2] = (int)t2; }
            return;
        }
        x[0] = (int)(v % nv);
        int64_t t = v / nv;
        if (D == 2) { x[1] = (int)t; }
        else { x[1] = (int)(t % nv); x[2] = (int)(t / nv); }
    }
    __device__ inline bool interior(const int *x) const
    {
        for (int m = 0; m < D; ++m)
            if (x[m] == 0 || x[m] == n) return false;
        return true;
    }
    __device__ inline int64_t vid(const int *x) const
    {
        return D == 2 ? x[0] + nv * x[1] : x[0] + nv * (x[1] + nv * (int64_t)x[2]);
    }
};

// ------------------------------------------------------ compressed store
// Tiles of 64 consecutive vertices.  Tier 0: nothing stored.  Tier t > 0:
// [64 scale bytes][slot 0: 64 entries][slot 1] ... entries of 1/2/4 bytes.
__host__ __device__ inline int tier_bytes(int t) { return t == 1 ? 1 : t == 2 ? 2 : t == 3 ? 4 : 0; }
__host__ __device__ inline uint32_t tile_units(int t, int H)
{
    return t == 0 ? 0u : (uint32_t)((64 + 64 * H * tier_bytes(t)) / 64);
}

__device__ inline float e4m3_to_float(uint32_t b)
{
    uint32_t s = (b & 0x80u) << 24, e = (b >> 3) & 15u, m = b & 7u;
    float v = e ? __uint_as_float(((e + 120u) << 23) | (m << 20)) : (float)m * 0.001953125f;
    return __uint_as_float(__float_as_uint(v) | s);
}

__device__ inline float e8m0_to_float(uint32_t e8)
{
    return e8 ? __uint_as_float(e8 << 23) : __uint_as_float(0x00400000u);
}

struct StoreView {
    const uint8_t *tier;
    const uint32_t *off;
    const uint8_t *payload;
    const float *eps_c;
    int n;
    int64_t NV;
    // decoded delta of slot j of vertex v (FP32; exact for every tier)
    __device__ inline float delta(int64_t v, int j, int H) const
    {
        int64_t t = v >> 6;
        int tt = tier[t];
        if (tt == 0) return 0.0f;
        const uint8_t *base = payload + (size_t)off[t] * 64;
        int l = (int)(v & 63);
        float sc = e8m0_to_float(base[l]);
        const uint8_t *slot = base + 64 + (size_t)j * 64 * tier_bytes(tt);
        if (tt == 2) {
            uint16_t hb = ((const uint16_t *)slot)[l];
            return (float)__builtin_bit_cast(_Float16, hb) * sc;
        }
        if (tt == 1) return e4m3_to_float(slot[l]) * sc;
        return ((const float *)slot)[l];
    }
};

// unit-eps Q1 coupling of two vertices differing in `nz` axes
__host__ __device__ inline double kref_unit(int D, int nz)
{
    if (D == 2) return nz == 1 ? -1.0 / 6.0 : -1.0 / 3.0;
    return nz == 1 ? 0.0 : -1.0 / 12.0;
}

// centre samples of the 2^d cells around vertex x (index B: the cell x - B),
// loaded once per vertex; coupling(j) is the centre-sample base coupling of
// slot j (FP64, fixed order: cells holding v and v+o in descending B, i.e.
// ascending index, then * k(o), then * h^{d-2})
template <int D> struct BaseCells {
    double e[1 << D];
    bool ok[1 << D];
    int n;
    __device__ inline void load(const float *eps_c, int n_, const int *x)
    {
        n = n_;
#pragma unroll
        for (int B = 0; B < (1 << D); ++B) {
            bool in = true;
            int64_t c = 0, stride = 1;
            for (int m = 0; m < D; ++m) {
                const int cm = x[m] - ((B >> m) & 1);
                if (cm < 0 || cm >= n) in = false;
                c += (int64_t)cm * stride;
                stride *= n;
            }
            ok[B] = in;
            e[B] = in ? (double)eps_c[c] : 0.0;
        }
    }
    __device__ inline double coupling(int j, double *ref) const
    {
#pragma clang fp contract(off)
        const int o[3] = {half_off(D, j, 0), half_off(D, j, 1), D == 3 ? half_off(D, j, 2) : 0};
        const int nz = (o[0] != 0) + (o[1] != 0) + (o[2] != 0);
        double sum = 0.0, sall = 0.0;
#pragma unroll
        for (int B = (1 << D) - 1; B >= 0; --B) {
            bool shared = true;
            for (int m = 0; m < D; ++m) {
                const int wm = ((B >> m) & 1) + o[m];
                if (wm < 0 || wm > 1) shared = false;
            }
            if (!ok[B]) continue;
            sall = sall + e[B];
            if (shared) sum = sum + e[B];
        }
        const double hp = (D == 2) ? 1.0 : 1.0 / (double)n;
        if (ref) *ref = sall * hp;
        return (sum * kref_unit(D, nz)) * hp;
    }
};

template <int D>
__device__ inline double base_coupling64(const float *eps_c, int n, const int *x, int j, double *ref)
{
    BaseCells<D> bc;
    bc.load(eps_c, n, x);
    return bc.coupling(j, ref);
}

// ------------------------------------------------------- host objects
struct OpSet {           // operators of every level (one version)
    double *S64[MGD_MAXLEV] = {};  // half stencils (FP64 form)
    float *S32[MGD_MAXLEV] = {};   // half stencils (mixed: coarse levels and decoded level 0)
    void *W[MGD_MAXLEV] = {};      // BoxMG weights [2^d][NV_l] (double / float)
    // compressed finest store (mixed)
    uint8_t *tier = nullptr;
    uint32_t *toff = nullptr;
    uint8_t *payload = nullptr;
    float *eps_c = nullptr;
    uint32_t *units_total = nullptr;  // device scalar: payload size in 64-byte units
    int64_t ntile = 0, payload_cap_units = 0;
    // 3D: the diagonal of every level's operator in the order of the
    // zero-start sweep (minus the sum over half slots of own + mirrored
    // coupling), per vertex; bit l of dz_ok says level l's is current.  Every
    // writer of a level's couplings clears dz_ok; the first zero-start sweep
    // after that recomputes it (one pass over the couplings per operator)
    void *Dz[MGD_MAXLEV] = {};
    mutable uint32_t dz_ok = 0;
    // 3D mixed, n % 4 == 0: per item of four finest-level vertices, 1 when
    // all its coupling sources lie in tier-0 tiles (k_item_mask); current
    // while bit kImaskOk of dz_ok is set, so every writer of the finest
    // operator invalidates it together with the diagonals
    uint8_t *imask = nullptr;
    // 3D BoxMG: per 64-vertex tile of level l, 1 where every structurally
    // nonzero weight of W[l] equals the d-linear one (the hierarchical
    // surplus P - P_geo of Sec. 5.5 is zero there), so the transfers take the
    // d-linear value instead of reading the tile's weights
    uint8_t *wgeo[MGD_MAXLEV] = {};
    double *chol = nullptr;  // dense Cholesky factor of the coarsest interior matrix
    double *cinv = nullptr;  // its inverse, for coarse grids of at most kCinvMax unknowns
};
constexpr int64_t kCinvMax = 128;
constexpr uint32_t kImaskOk = 1u << 31;  // above every level bit (MGD_MAXLEV < 31)

struct mgd_hier {
    mgd_ctx *ctx = nullptr;
    int dim = 2, n = 0, precision = MGD_FP64, transfer = MGD_GEOMETRIC, coarsest = 2;
    int store_path = MGD_STORE_AUTO;  // MGD_MIXED: source of the finest operator in the fused 2D kernels
    int nlev = 0, H = 4;
    int nl[MGD_MAXLEV] = {};
    int64_t NV[MGD_MAXLEV] = {};
    int64_t m_coarse = 0;
    OpSet ops;
    // cycle vectors (double for FP64, float for mixed)
    void *u[MGD_MAXLEV] = {}, *f[MGD_MAXLEV] = {}, *r[MGD_MAXLEV] = {}, *t[MGD_MAXLEV] = {};
    // scratch for compression
    float *delta = nullptr;
    uint8_t *vtier = nullptr;
    // reduction scratch and device scalars owned by this hierarchy
    double *partial = nullptr;    // block partial sums / coarse-solve work
    int64_t partial_cap = 0;
    double *scal = nullptr;       // [64] device scalars
    double *host_scal = nullptr;  // pinned [64]
    double *partial2 = nullptr;   // second partial list (matrix-vector product of CG), partial_cap
    const double *p1 = nullptr;   // CG dot partials (z.r then z.(r - r_old)), p1_n each
    int64_t p1_n = 0, p2_n = 0;
    double *host_part = nullptr;      // pinned: squared norms of the last two residual checks
    double *host_part_dev = nullptr;  // its device address
    size_t vec_bytes() const { return precision == MGD_FP64 ? 8 : 4; }
};

// ------------------------------------------------------- launch helpers
static inline unsigned grid_for(int64_t n, int block) { return (unsigned)((n + block - 1) / block); }

// host-side allocation helpers (return MGD_ENOMEM through ctx on failure)
int dev_alloc(mgd_ctx *ctx, void **p, size_t bytes);
extern thread_local size_t g_dev_alloc_bytes;
void dev_free(void *p);

// kernels / launchers implemented in the .hip files
int launch_assemble(mgd_ctx *ctx, int dim, int n, int s, const int64_t *cells, int64_t count,
                    const mgd_eps *eps, int mode, void *K_out, const void *K_old, int k_by_cell,
                    double C, double *rel_out, uint8_t *done_out, const int64_t *count_dev,
                    hipStream_t st, int keep_old = 0);
// the paper's p3-byte format of element-matrix surpluses (paper.hip)
int launch_p3_encode(mgd_ctx *ctx, int dim, const double *K, const double *K1, int64_t count, double tau,
                     uint8_t *p3_out, uint8_t *bytes_out, hipStream_t st);
// finest-level items of the default 3D sweep and its tier-0 ones (cycle.hip)
int item_mask_count(mgd_hier *h, int64_t *items, int64_t *tier0, hipStream_t st);
int launch_compact_open(mgd_ctx *ctx, const uint8_t *done, const int64_t *cells_in, const int64_t *count_dev,
                        int64_t count_bound, int32_t *block_tmp, int64_t *cells_out, int64_t *count_out,
                        hipStream_t st);
int launch_gather(mgd_ctx *ctx, int dim, int n, const void *K, int k_mode, void *S, int s_mode,
                  hipStream_t st);
int launch_centre_eps(mgd_ctx *ctx, int dim, int n, const mgd_eps *eps, float *eps_c, hipStream_t st);
int opset_alloc(mgd_hier *h, OpSet &o);
void opset_free(OpSet &o);
// surplus and tier selection of a level-0 store: delta [H][NV] and vtier [NV]
// are working buffers (the hierarchy's, or the caller's scratch)
int compress_into(mgd_hier *h, OpSet &o, const float *S32, const float *eps_c,
                  const mgd_tier_policy *pol, float *delta, uint8_t *vtier, hipStream_t st);
// the hierarchy's compression buffers, allocated on first use
int hier_compress_buffers(mgd_hier *h);
// per-device static scratch (noalloc.hip): set at context creation
int scratch_init(mgd_ctx *ctx);
int coarsen_ops(mgd_hier *h, OpSet &o, hipStream_t st);
// geometric hierarchy of a provisional operator: coarse levels rediscretised
// from child-averaged cell values (finest: eps_c0), d-linear weights;
// scratch: (n/2)^d + (n/4)^d floats
int coarsen_geometric(mgd_hier *h, OpSet &o, const float *eps_c0, float *scratch, hipStream_t st);
int decode_level_f64(mgd_hier *h, const OpSet &o, int level, double *out, hipStream_t st);
int weights_f64(mgd_hier *h, const OpSet &o, int level, double *out, hipStream_t st);
int cycle_smooth(mgd_hier *h, const OpSet &o, int level, void *u, const void *f, void *tmp,
                 int sweeps, double omega, bool zero_guess, hipStream_t st);
int cycle_residual(mgd_hier *h, const OpSet &o, int level, const void *u, const void *f, void *r,
                   hipStream_t st);
int cycle_restrict(mgd_hier *h, const OpSet &o, int level, const void *r, void *fc, hipStream_t st);
int cycle_prolong(mgd_hier *h, const OpSet &o, int level, const void *ec, void *u, hipStream_t st);
// CG scalars: s[7] restart flag (beta = 0), s[zr_old] / s[zr_new] the
// alternating slots of z.r; p1: partials of z.r and z.(r - r_old), n1 each
struct CgScalars {
    double *s;
    const double *p1;
    int64_t n1;
    int zr_old, zr_new;
};
constexpr int kHostParts = 1024;
// residual checks: the squared norm of check k lands in the device scalar
// s[kChkSlot + (k & 1)] and in the pinned host slot host_part[k & 1]; slot 2
// (s[kChkSlot + 2], host_part[2]) takes the true residual that confirms a
// CG convergence
constexpr int kChkSlot = 24;
// s[kRRuSlot]: the carried iterate's squared residual at an operator change
// (kRRuSlot + 1: scratch); s[kZeroSlot]: 1 when that change restarted from
// the zero start
constexpr int kRRuSlot = 28, kZeroSlot = 30;
int check_sum(mgd_hier *h, int nparts, int slot, hipStream_t st);
// after an operator change (the carried iterate's outer residual partials in
// h->partial): keep the iterate or take the zero start (interior zeroed),
// whichever has the smaller residual; uz, rz: scratch vectors; the chosen
// start's squared residual to check slot `slot`
int restart_pick(mgd_hier *h, const OpSet &o, int nparts, int slot, const double *f, double *u, double *r,
                 double *uz, double *rz, hipStream_t st);
int pcg_dots(mgd_hier *h, const void *z, const double *r, const double *rold, hipStream_t st);
int pcg_matvec(mgd_hier *h, const OpSet &o, const void *z, const double *pold, double *pnew, double *Ap,
               const CgScalars &c, hipStream_t st);
// gate_slot >= 0: a cycle queued before check gate_slot was read; it leaves
// x and r unchanged when that check's squared norm is <= thr (converged)
int pcg_update(mgd_hier *h, double *x, const double *p, double *r, double *rold, const double *Ap,
               const CgScalars &c, int gate_slot, double thr, int *nparts, hipStream_t st);
int compress_partials(mgd_hier *h, const double *partial, int64_t cnt, int nvec, double *out, hipStream_t st);
int lev2_pmv(mgd_hier *h, const OpSet &o, const void *z, const double *pold, double *pnew, double *Ap,
             const CgScalars &c, hipStream_t st);

// CG dot products z.r and z.(r - r_old) fused into the last kernel of a
// V-cycle whose result is z; s: the CG scalars (beta is formed there too)
struct Lev2Dots {
    const double *r, *rold;
    double *s;
};
// V(nu1,nu2) correction cycle on u.  With `result`, the cycle's result may be
// left in another level buffer, whose address is returned there; without it
// the result is always in u.  With `dots`, *dots_done tells whether the dot
// products were formed inside the cycle.
int vcycle_ops(mgd_hier *h, const OpSet &o, void *u, const void *f, double omega, int nu1, int nu2,
               bool zero_guess, hipStream_t st, const Lev2Dots *dots = nullptr, void **result = nullptr,
               bool *dots_done = nullptr);
bool lev2_ok(const mgd_hier *h, int l, int nu1, int nu2);
// one additive adaFAC-x correction *result = B rhs (adafac.hip)
int adafac_ops(mgd_hier *h, const OpSet &o, const void *rhs, double omega, int variant, void **result,
               hipStream_t st);
int lev2_pre(mgd_hier *h, const OpSet &o, int l, const void *u, const void *f, void *u_out, void *r_out,
             double omega, hipStream_t st);
int lev2_prer(mgd_hier *h, const OpSet &o, int l, const void *u, const void *f, void *u_out, void *fc, double omega,
              hipStream_t st);
int lev2_post(mgd_hier *h, const OpSet &o, int l, const void *u, const void *ec, const void *f, void *u_out,
              double omega, const Lev2Dots *dots, hipStream_t st);
int outer_residual(mgd_hier *h, const OpSet &o, const double *u, const double *f, double *r, int *nparts,
                   hipStream_t st);
int hier_alloc_levels(mgd_hier *h);
void hier_free(mgd_hier *h);
