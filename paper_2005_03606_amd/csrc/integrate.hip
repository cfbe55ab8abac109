// Element integration on gfx950 (paper Sec. 4.2, eq. mg:weak-form-of-assembly;
// adaptive criterion Sec. 5.2): eps is held constant on each of the s^d equal
// sub-cells of a cell and the gradient products are integrated exactly, so
//     K_c = sum_q eps(x_q) G_q,
//     G_q[a][b] = h^{d-2} sum_k (sigma_a sigma_b / s)_k prod_{m != k} M_{q_m}(a_m, b_m),
// M_q(a,b) the integral of psi_a psi_b over [q/s, (q+1)/s] (psi_0 = 1 - xi,
// psi_1 = xi).  Two device paths:
//   FP64: VALU, sum-factorised along x-lines, G lanes per cell;
//   mixed: eps split into bf16 hi + lo, contracted on MFMA (16x16x32 bf16)
//          against the integer-scaled G table split exactly into bf16 terms,
//          FP32 accumulation; the [cells x s^d] x [s^d x pairs] contraction.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>

#include "common.h"
#include <algorithm>

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float floatx4;

// ------------------------------------------------------------ eps on device
struct EpsDev {
    int kind, dim, count;
    double p0, p1;
    const double *data;
};

// eps at x; geometric membership decisions in FP64 for every path,
// transcendental laws in T (float for the mixed path).  Balls and boxes are
// taken from `rows` / `count`: the block's candidate list (same row layout,
// same order as the descriptor) or the descriptor's own data.
template <int D, typename T, int EK>
__device__ inline T eps_eval_k(const EpsDev &e, const double *x, const double *rows, int count)
{
    // EK >= 0: the field kind known at compile time, the other cases dropped
    switch (EK >= 0 ? EK : e.kind) {
    case MGD_EPS_CONST:
        return (T)e.p0;
    case MGD_EPS_SINE: {
        T p = (T)1;
        for (int m = 0; m < D; ++m) p *= sin((T)(2.0 * M_PI) * (T)x[m]);
        return (T)1 + (T)e.p0 * p;
    }
    case MGD_EPS_THETA: {
        T p = (T)1, th = (T)e.p0;
        for (int m = 0; m < D; ++m) p *= exp(-th * (T)x[m]) * cos((T)M_PI * th * (T)x[m]);
        return (T)1 + ((T)0.3 / (T)D) * p;
    }
    case MGD_EPS_BALLS: {
#pragma clang fp contract(off)
        for (int b = 0; b < count; ++b) {
            const double *row = rows + (size_t)b * (D + 1);
            double r2 = 0.0;
            for (int m = 0; m < D; ++m) {
                double dx = x[m] - row[m];
                r2 = r2 + dx * dx;
            }
            if (r2 <= row[D] * row[D]) return (T)e.p1;
        }
        return (T)e.p0;
    }
    case MGD_EPS_LATTICE: {
        int L = e.count, base[3];
        T t[3];
        for (int m = 0; m < D; ++m) {
            double y = x[m] * L;
            int i = (int)floor(y);
            i = i < 0 ? 0 : (i > L - 1 ? L - 1 : i);
            base[m] = i;
            t[m] = (T)(y - i);
        }
        T g = (T)0;
        for (int a = 0; a < (1 << D); ++a) {
            T w = (T)1;
            int64_t idx = 0, stride = 1;
            for (int m = 0; m < D; ++m) {
                int bit = (a >> m) & 1;
                w *= bit ? t[m] : (T)1 - t[m];
                idx += (int64_t)(base[m] + bit) * stride;
                stride *= (L + 1);
            }
            g += w * (T)e.data[idx];
        }
        return exp((T)e.p0 * g);
    }
    case MGD_EPS_BOXES: {
        double v = e.p0;
        for (int b = 0; b < count; ++b) {
            const double *row = rows + (size_t)b * (2 * D + 1);
            bool in = true;
            for (int m = 0; m < D; ++m) in = in && x[m] >= row[m] && x[m] < row[D + m];
            if (in) v = row[2 * D];
        }
        return (T)v;
    }
    }
    return (T)NAN;
}

template <int D, typename T>
__device__ inline T eps_eval(const EpsDev &e, const double *x, const double *rows, int count)
{
    return eps_eval_k<D, T, -1>(e, x, rows, count);
}

// Lattice fields: when every sample point of a cell lies in one lattice cell
// (the lattice resolution divides the grid's), the cell's 2^d corner values
// are loaded once and each sample only interpolates; the arithmetic is
// eps_eval's, in the same order, so the values are identical.
template <int D, typename T> struct EpsCell {
    bool ok = false;
    int base[3] = {0, 0, 0};
    T corner[1 << D];
};

template <int D, typename T>
__device__ inline void eps_cell_prepare(const EpsDev &e, int n, bool valid, const int *ci, EpsCell<D, T> &c)
{
    c.ok = false;
    if (e.kind != MGD_EPS_LATTICE || !valid) return;
    const int64_t L = e.count;
    bool one = true;
    for (int m = 0; m < D; ++m) {
        const int64_t lo = (int64_t)ci[m] * L, hi = (int64_t)(ci[m] + 1) * L;
        const int64_t b = lo / n, top = (hi + n - 1) / n - 1;  // floor of every interior point
        one = one && b == top && b <= L - 1;
        c.base[m] = (int)b;
    }
    if (!one) return;
    c.ok = true;
    for (int a = 0; a < (1 << D); ++a) {
        int64_t idx = 0, stride = 1;
        for (int m = 0; m < D; ++m) {
            idx += (int64_t)(c.base[m] + ((a >> m) & 1)) * stride;
            stride *= (L + 1);
        }
        c.corner[a] = (T)e.data[idx];
    }
}

template <int D, typename T, int EK = -1>
__device__ inline T eps_eval_cell(const EpsDev &e, const EpsCell<D, T> &c, const double *x, const double *rows,
                                  int count)
{
    if (!c.ok) return eps_eval_k<D, T, EK>(e, x, rows, count);
    const int L = e.count;
    T t[3];
    for (int m = 0; m < D; ++m) t[m] = (T)(x[m] * L - c.base[m]);
    T g = (T)0;
#pragma unroll
    for (int a = 0; a < (1 << D); ++a) {
        T w = (T)1;
#pragma unroll
        for (int m = 0; m < D; ++m) w *= ((a >> m) & 1) ? t[m] : (T)1 - t[m];
        g += w * c.corner[a];
    }
    return exp((T)e.p0 * g);
}

// ------------------------------------------------------ candidate culling
// A workgroup evaluates eps only inside the bounding box of its cells; balls
// and boxes that cannot reach the box are dropped once per workgroup.  The
// kept rows are copied to LDS in descriptor order (boxes paint in order).
#define MGD_MAX_CAND 192
struct CandLDS {
    double rows[MGD_MAX_CAND * 7];
    int lo[3], hi[3];
    int count, overflow;
    int wave_cnt[16];
};

// Each thread brings the box [lo, hi] of the cells it stands for (valid
// false: none); the box is reduced across the wave first, so the LDS sees
// one update per wave.
template <int D>
__device__ inline void build_candidates(const EpsDev &e, int n, bool valid, const int *clo, const int *chi,
                                        CandLDS &L, const double **rows, int *count)
{
    *rows = e.data;
    *count = e.count;
    if (e.kind != MGD_EPS_BALLS && e.kind != MGD_EPS_BOXES) return;  // uniform branch
    int tid = threadIdx.x;
    if (tid == 0) {
        for (int m = 0; m < 3; ++m) { L.lo[m] = 0x7fffffff; L.hi[m] = -1; }
        L.count = 0;
        L.overflow = 0;
    }
    __syncthreads();
    for (int m = 0; m < D; ++m) {
        int lo = valid ? clo[m] : 0x7fffffff, hi = valid ? chi[m] : -1;
        for (int off = 32; off > 0; off >>= 1) {
            lo = min(lo, __shfl_xor(lo, off));
            hi = max(hi, __shfl_xor(hi, off));
        }
        if ((tid & 63) == 0) {
            atomicMin(&L.lo[m], lo);
            atomicMax(&L.hi[m], hi);
        }
    }
    __syncthreads();
    if (L.hi[0] < 0) return;  // no valid cell in this workgroup
    double blo[3], bhi[3];
    for (int m = 0; m < D; ++m) {
        blo[m] = (double)L.lo[m] / n;
        bhi[m] = (double)(L.hi[m] + 1) / n;
    }
    const int stride = e.kind == MGD_EPS_BALLS ? D + 1 : 2 * D + 1;
    const int lane = tid & 63, wave = tid >> 6, nw = (blockDim.x + 63) >> 6;
    for (int base = 0; base < e.count; base += blockDim.x) {
        int b = base + tid;
        bool keep = false;
        if (b < e.count) {
            const double *row = e.data + (size_t)b * stride;
            if (e.kind == MGD_EPS_BALLS) {
                double d2 = 0.0;
                for (int m = 0; m < D; ++m) {
                    double c = row[m], q = c < blo[m] ? blo[m] : (c > bhi[m] ? bhi[m] : c);
                    d2 += (c - q) * (c - q);
                }
                keep = d2 <= row[D] * row[D] * (1.0 + 1e-12) + 1e-300;
            } else {
                keep = true;
                for (int m = 0; m < D; ++m) keep = keep && row[m] < bhi[m] && row[D + m] > blo[m];
            }
        }
        unsigned long long mask = __ballot(keep);
        if (lane == 0) L.wave_cnt[wave] = __popcll(mask);
        __syncthreads();
        int before = 0, total = 0;
        for (int w = 0; w < nw; ++w) {
            if (w < wave) before += L.wave_cnt[w];
            total += L.wave_cnt[w];
        }
        int pos = L.count + before + __popcll(mask & ((1ull << lane) - 1ull));
        if (keep && pos < MGD_MAX_CAND) {
            const double *row = e.data + (size_t)b * stride;
            for (int k = 0; k < stride; ++k) L.rows[pos * stride + k] = row[k];
        }
        __syncthreads();
        if (tid == 0) {
            L.count += total;
            if (L.count > MGD_MAX_CAND) L.overflow = 1;
        }
        __syncthreads();
    }
    if (!L.overflow) {
        *rows = L.rows;
        *count = L.count;
    }
}

// The same list for the cells of one wavefront (scattered cells: the open
// cells of a ladder rung), built by the wave alone into its own LDS rows
// (capacity cap; on overflow the full list stays in use).
constexpr int kWaveCand = 64;
template <int D>
__device__ inline void build_candidates_wave(const EpsDev &e, int n, bool valid, const int *c, double *wrows,
                                             const double **rows, int *count)
{
    *rows = e.data;
    *count = e.count;
    if (e.kind != MGD_EPS_BALLS && e.kind != MGD_EPS_BOXES) return;  // uniform branch
    const int lane = threadIdx.x & 63;
    int lo[3] = {0, 0, 0}, hi[3] = {-1, -1, -1};
    for (int m = 0; m < D; ++m) {
        int l = valid ? c[m] : 0x7fffffff, h = valid ? c[m] : -1;
        for (int off = 32; off > 0; off >>= 1) {
            l = min(l, __shfl_xor(l, off));
            h = max(h, __shfl_xor(h, off));
        }
        lo[m] = l;
        hi[m] = h;
    }
    if (hi[0] < 0) return;  // no valid cell in this wave
    double blo[3], bhi[3];
    for (int m = 0; m < D; ++m) {
        blo[m] = (double)lo[m] / n;
        bhi[m] = (double)(hi[m] + 1) / n;
    }
    const int stride = e.kind == MGD_EPS_BALLS ? D + 1 : 2 * D + 1;
    int cnt = 0;
    for (int base = 0; base < e.count; base += 64) {
        const int b = base + lane;
        bool keep = false;
        if (b < e.count) {
            const double *row = e.data + (size_t)b * stride;
            if (e.kind == MGD_EPS_BALLS) {
                double d2 = 0.0;
                for (int m = 0; m < D; ++m) {
                    double cc = row[m], q = cc < blo[m] ? blo[m] : (cc > bhi[m] ? bhi[m] : cc);
                    d2 += (cc - q) * (cc - q);
                }
                keep = d2 <= row[D] * row[D] * (1.0 + 1e-12) + 1e-300;
            } else {
                keep = true;
                for (int m = 0; m < D; ++m) keep = keep && row[m] < bhi[m] && row[D + m] > blo[m];
            }
        }
        const unsigned long long mask = __ballot(keep);
        const int pos = cnt + __popcll(mask & ((1ull << lane) - 1ull));
        if (keep && pos < kWaveCand) {
            const double *row = e.data + (size_t)b * stride;
            for (int k = 0; k < stride; ++k) wrows[pos * stride + k] = row[k];
        }
        cnt += __popcll(mask);
    }
    // the wave's LDS rows are written before any lane reads them
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (cnt <= kWaveCand) {
        *rows = wrows;
        *count = cnt;
    }
}

// ------------------------------------------------------ shared argument pack
struct AsmArgs {
    int n, s;
    int64_t count;
    const int64_t *count_dev;  // if set, overrides count (device-side active count)
    const int64_t *cells;      // null: cell = i
    EpsDev eps;
    const double *samples;     // MGD_EPS_SAMPLES: [count][s^d]
    void *K_out;
    const void *K_old;
    int k_by_cell;             // K_out / K_old rows indexed by cell id (in-place ladder)
    double C;
    double *rel_out;
    uint8_t *done_out;
    int keep_old;              // rel < C: leave the row with K_old (K_out == K_old, in place)
};

__device__ inline int64_t asm_count(const AsmArgs &a) { return a.count_dev ? *a.count_dev : a.count; }

template <int D> __device__ inline void cell_coords(int64_t c, int n, int *ci)
{
    if (c <= 0xffffffffLL) {  // 32-bit division (the 64-bit one is a long software sequence)
        const uint32_t cc = (uint32_t)c, m = (uint32_t)n, t = cc / m;
        ci[0] = (int)(cc - t * m);
        if (D == 2) ci[1] = (int)t;
        else { const uint32_t t2 = t / m; ci[1] = (int)(t - t2 * m); ci[2] = (int)t2; }
        return;
    }
    ci[0] = (int)(c % n);
    int64_t t = c / n;
    if (D == 2) ci[1] = (int)t;
    else { ci[1] = (int)(t % n); ci[2] = (int)(t / n); }
}

__device__ inline double sample_coord(int ci, int q, int s, int n)
{
    // s is a power of two: (q + 1/2) / s is the exact product with 1 / s,
    // which the compiler hoists out of the sample loops
    return ((double)ci + ((double)q + 0.5) * (1.0 / (double)s)) / (double)n;
}

// ---- boxes on a cell's sample lattice.  sample_coord is monotone in the
// sample index (each step rounds a monotone function), so the samples of a
// cell that pass a box's test on axis m (x >= lower face, x < upper face)
// form an index range [lo, hi), found once per cell by bisection with that
// same test.  A box whose range is empty on some axis holds none of the
// cell's samples; the others keep the descriptor's order, and painting a
// sample compares small integers: the same box wins as in eps_eval, so eps
// is the same value.
constexpr int kCellBoxes = 8;
template <typename T> struct CellBoxes {
    int count;                 // boxes kept; -1: more than kCellBoxes reach the cell
    T val[kCellBoxes];         // eps inside the box, rounded as eps_eval rounds it
    // XMASK: lo_y | hi_y << 5 | lo_z << 10 | hi_z << 15 | x mask of the lane's
    // 8 samples << 20; else lo_x | hi_x << 5 | lo_y << 10 | hi_y << 15 |
    // lo_z << 20 | hi_z << 25
    uint32_t rng[kCellBoxes];
};

// smallest q in [0, s] whose sample coordinate is >= t
__device__ inline int first_sample_at_least(int ci, int s, int n, double t)
{
    int lo = 0, hi = s;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (sample_coord(ci, mid, s, n) >= t) hi = mid;
        else lo = mid + 1;
    }
    return lo;
}

// the boxes of `rows` that hold samples of cell ci (s <= 16); with XMASK the
// lane's 8 samples have x indices (qx0 + e) mod s
template <int D, typename T, bool XMASK>
__device__ inline void cell_boxes(const int *ci, int s, int n, int qx0, const double *rows, int count,
                                  CellBoxes<T> &cb)
{
    double first[3], last[3];
    for (int m = 0; m < D; ++m) {
        first[m] = sample_coord(ci[m], 0, s, n);
        last[m] = sample_coord(ci[m], s - 1, s, n);
    }
    cb.count = 0;
    for (int b = 0; b < count; ++b) {
        const double *row = rows + (size_t)b * (2 * D + 1);
        bool reach = true;
        for (int m = 0; m < D; ++m) reach = reach && row[D + m] > first[m] && row[m] <= last[m];
        if (!reach) continue;
        int lo[3] = {0, 0, 0}, hi[3] = {1, 1, 1};
        bool empty = false;
        for (int m = 0; m < D; ++m) {
            lo[m] = first_sample_at_least(ci[m], s, n, row[m]);
            hi[m] = first_sample_at_least(ci[m], s, n, row[D + m]);
            empty = empty || lo[m] >= hi[m];
        }
        if (empty) continue;
        if (cb.count == kCellBoxes) {
            cb.count = -1;
            return;
        }
        uint32_t r;
        if (XMASK) {
            uint32_t xm = 0;
            for (int e = 0; e < 8; ++e) {
                const int qx = (qx0 + e) & (s - 1);
                if (qx >= lo[0] && qx < hi[0]) xm |= 1u << e;
            }
            r = (uint32_t)lo[1] | (uint32_t)hi[1] << 5 | (uint32_t)lo[2] << 10 | (uint32_t)hi[2] << 15 | xm << 20;
        } else {
            r = (uint32_t)lo[0] | (uint32_t)hi[0] << 5 | (uint32_t)lo[1] << 10 | (uint32_t)hi[1] << 15 |
                (uint32_t)lo[2] << 20 | (uint32_t)hi[2] << 25;
        }
        const T v = (T)row[2 * D];
#pragma unroll
        for (int k = 0; k < kCellBoxes; ++k)
            if (k == cb.count) {
                cb.val[k] = v;
                cb.rng[k] = r;
            }
        ++cb.count;
    }
}

// ---- boxes at small s (2 and 4 samples per axis, FP64 kernel): the boxes
// of the candidate list that can hold one of the cell's samples (upper face
// above its first sample and lower face at most its last one, per axis), at
// most kCellCand in descriptor order; each sample then takes eps_eval's test
// against those alone, so the same box wins.  count -1: more reach the cell,
// and the whole list is tested.  (In the MFMA kernel the registers it takes
// cost a wave per SIMD at s = 4, more than it saves.)
constexpr int kCellCand = 4;
// instantiation code for box fields below s = 8: box evaluation only (no
// other field kind's code or registers); in the FP64 kernel with the
// per-cell candidates below
constexpr int kBoxesSmall = 64;
struct CellCand {
    int count;
    int idx[kCellCand];
};

template <int D>
__device__ inline void cell_candidates(const int *ci, int s, int n, const double *rows, int count, CellCand &cc)
{
    double first[3], last[3];
    for (int m = 0; m < D; ++m) {
        first[m] = sample_coord(ci[m], 0, s, n);
        last[m] = sample_coord(ci[m], s - 1, s, n);
    }
    cc.count = 0;
    for (int b = 0; b < count; ++b) {
        const double *row = rows + (size_t)b * (2 * D + 1);
        bool reach = true;
        for (int m = 0; m < D; ++m) reach = reach && row[D + m] > first[m] && row[m] <= last[m];
        if (!reach) continue;
        if (cc.count == kCellCand) {
            cc.count = -1;
            return;
        }
#pragma unroll
        for (int k = 0; k < kCellCand; ++k)
            if (k == cc.count) cc.idx[k] = b;
        ++cc.count;
    }
}

// eps_eval's box case over the prefiltered rows
template <int D, typename T>
__device__ inline T eps_boxes_cand(const EpsDev &e, const double *x, const double *rows, const CellCand &cc)
{
    double v = e.p0;
#pragma unroll
    for (int k = 0; k < kCellCand; ++k) {
        if (k >= cc.count) break;
        const double *row = rows + (size_t)cc.idx[k] * (2 * D + 1);
        bool in = true;
        for (int m = 0; m < D; ++m) in = in && x[m] >= row[m] && x[m] < row[D + m];
        if (in) v = row[2 * D];
    }
    return (T)v;
}

// M_q(a,b) over the q-th of s sub-intervals: index 0 = (0,0), 1 = (0,1), 2 = (1,1)
__device__ inline void moments64(int s, int q, double *M)
{
    double S3 = (double)s * s * s;
    int qb = s - 1 - q;
    M[2] = (3.0 * q * q + 3.0 * q + 1.0) / (3.0 * S3);
    M[0] = (3.0 * qb * qb + 3.0 * qb + 1.0) / (3.0 * S3);
    M[1] = (6.0 * q * (s - q) + 3.0 * (s - 2.0 * q) - 2.0) / (6.0 * S3);
}

__device__ inline int mtype(int a, int b) { return a + b; }  // 0: 00, 1: 01/10, 2: 11

// adaptive criterion: max-norm of the change over the full 2^d x 2^d matrices
template <int D, typename T>
__device__ inline double ladder_rel(const T *Knew, const T *Kold)
{
    constexpr int nl = 1 << D, U = n_pairs(D);
    double dnew[nl], dold[nl];
    for (int a = 0; a < nl; ++a) dnew[a] = dold[a] = 0.0;
    double mdiff = 0.0, mold = 0.0;
    for (int a = 0; a < nl; ++a)
        for (int b = a + 1; b < nl; ++b) {
            int p = pair_index(D, a, b);
            double kn = (double)Knew[p], ko = (double)Kold[p];
            dnew[a] -= kn; dnew[b] -= kn;
            dold[a] -= ko; dold[b] -= ko;
            mdiff = fmax(mdiff, fabs(kn - ko));
            mold = fmax(mold, fabs(ko));
        }
    for (int a = 0; a < nl; ++a) {
        mdiff = fmax(mdiff, fabs(dnew[a] - dold[a]));
        mold = fmax(mold, fabs(dold[a]));
    }
    (void)U;
    return mdiff / mold;
}

template <int D, typename T>
__device__ inline void store_and_check(const AsmArgs &a, int64_t i, int64_t cell, const T *K)
{
    constexpr int U = n_pairs(D);
    int64_t row = a.k_by_cell ? cell : i;
    if (a.K_old) {
        int64_t orow = a.k_by_cell ? cell : i;
        const T *Ko = (const T *)a.K_old + orow * U;
        T old[U];
        for (int p = 0; p < U; ++p) old[p] = Ko[p];
        double rel = ladder_rel<D, T>(K, old);
        if (a.rel_out) a.rel_out[i] = rel;
        if (a.done_out) a.done_out[i] = rel < a.C ? 1 : 0;
        if (a.keep_old && rel < a.C) return;
    }
    T *Ko = (T *)a.K_out + row * U;
    for (int p = 0; p < U; ++p) Ko[p] = K[p];
}

// ------------------------------------------------------------ FP64 (VALU)
// G lanes cooperate on one cell; lane g takes x-lines g, g+G, ...  The
// element matrix is computed in FP64 and stored as TO (double, or float for
// the mixed form's short rungs).  One tile of 256 / G cells per block for a
// count known on the host; for a device-side count (the ladder's open
// cells, bounded on the host by every cell) a capped grid strides over the
// tiles up to the count, so the bound costs nothing.  (The tile is written
// inline: as a called function its accumulators leave the registers.)
template <int D, int G, bool STRIDE, typename TO, int EK> __global__ __launch_bounds__(256) void k_integrate64(AsmArgs a)
{
    __shared__ CandLDS cand;
    constexpr int EKF = EK == kBoxesSmall ? MGD_EPS_BOXES : EK;  // the field kind evaluated
    const int64_t cnt = asm_count(a);
    for (int64_t blk = blockIdx.x;; blk += gridDim.x) {
        if (blk * (int64_t)blockDim.x / G >= cnt) return;  // uniform, before any barrier
        int64_t gid = blk * blockDim.x + threadIdx.x;
        int64_t i = gid / G;
        int g = (int)(gid % G);
        bool valid = i < cnt;
        int s = a.s, n = a.n;
        int64_t cell = valid ? (a.cells ? a.cells[i] : i) : 0;
        int ci[3] = {0, 0, 0};
        cell_coords<D>(cell, n, ci);
        const double *rows;
        int nrows;
        build_candidates<D>(a.eps, n, valid, ci, ci, cand, &rows, &nrows);
        EpsCell<D, double> ecell;
        if (EKF < 0 || EKF == MGD_EPS_LATTICE) eps_cell_prepare<D, double>(a.eps, n, valid, ci, ecell);
        // boxes from s = 8 on: painted from the cell's index ranges unless a
        // lane's cell in the wave is reached by more than kCellBoxes boxes
        CellBoxes<double> cbx;
        cbx.count = 0;
        bool fastbox = false;
        int kmax = 0;
        if (EK == MGD_EPS_BOXES && s >= 8) {
            if (valid) cell_boxes<D, double, false>(ci, s, n, 0, rows, nrows, cbx);
            int c = cbx.count, over = cbx.count < 0 ? 1 : 0;
            for (int off = 32; off > 0; off >>= 1) {
                c = max(c, __shfl_xor(c, off));
                over = max(over, __shfl_xor(over, off));
            }
            fastbox = over == 0;
            kmax = c;
        }
        // the generic instantiation at s = 2 and 4 on a box field
        CellCand cand4;
        cand4.count = -1;
        const bool boxcand = (EK < 0 || EK == kBoxesSmall) && a.eps.kind == MGD_EPS_BOXES && s >= 2 && s <= 4;
        if (boxcand && valid) cell_candidates<D>(ci, s, n, rows, nrows, cand4);
        int nlines = (D == 2) ? s : s * s;
        int64_t nq = (int64_t)nlines * s;
        // accumulators: T1[ty][tz] = sum eps My Mz, T2[tx][tz] = sum eps Mx Mz,
        // T3[tx][ty] = sum eps Mx My (2D: T1[ty], T2[tx])
        double T1[9], T2[9], T3[9];
#pragma unroll
        for (int k = 0; k < 9; ++k) T1[k] = T2[k] = T3[k] = 0.0;
        if (valid) {
            for (int line = g; line < nlines; line += G) {
                int qy = line % s, qz = line / s;
                double My[3], Mz[3] = {1.0, 1.0, 1.0};
                moments64(s, qy, My);
                if (D == 3) moments64(s, qz, Mz);
                double L0 = 0.0, L[3] = {0.0, 0.0, 0.0};
                double x[3];
                x[1] = sample_coord(ci[1], qy, s, n);
                if (D == 3) x[2] = sample_coord(ci[2], qz, s, n);
                // the kept boxes whose y and z ranges hold this line
                uint32_t yzm = 0;
                if (EK == MGD_EPS_BOXES && fastbox) {
#pragma unroll
                    for (int k = 0; k < kCellBoxes; ++k) {
                        if (k >= kmax) break;
                        const uint32_t r = cbx.rng[k];
                        if (k < cbx.count && (uint32_t)qy >= (r >> 10 & 31u) && (uint32_t)qy < (r >> 15 & 31u) &&
                            (uint32_t)qz >= (r >> 20 & 31u) && (uint32_t)qz < (r >> 25 & 31u))
                            yzm |= 1u << k;
                    }
                }
                // a lattice cell inside one lattice cell: along the x-line
                // p0 g = ga + t_x gb (FP64), one exp per sample
                const bool latl = EK == MGD_EPS_LATTICE && ecell.ok;
                double ga = 0.0, gb = 0.0;
                if (latl) {
                    const double t1 = x[1] * a.eps.count - ecell.base[1];
                    const double t2 = D == 3 ? x[2] * a.eps.count - ecell.base[2] : 0.0;
                    double f0 = 0.0, f1 = 0.0;
#pragma unroll
                    for (int c = 0; c < (1 << (D - 1)); ++c) {
                        const double w = ((c & 1) ? t1 : 1.0 - t1) * (D == 3 ? ((c & 2) ? t2 : 1.0 - t2) : 1.0);
                        f0 += w * ecell.corner[2 * c];
                        f1 += w * ecell.corner[2 * c + 1];
                    }
                    ga = a.eps.p0 * f0;
                    gb = a.eps.p0 * (f1 - f0);
                }
                for (int qx = 0; qx < s; ++qx) {
                    double e;
                    if ((EKF >= 0 ? EKF : a.eps.kind) == MGD_EPS_SAMPLES) {
                        int64_t q = qx + (int64_t)s * line;
                        e = a.samples[i * nq + q];
                    } else if (latl) {
                        e = exp(ga + (sample_coord(ci[0], qx, s, n) * a.eps.count - ecell.base[0]) * gb);
                    } else if (EK == MGD_EPS_BOXES && fastbox) {
                        e = a.eps.p0;
#pragma unroll
                        for (int k = 0; k < kCellBoxes; ++k) {
                            if (k >= kmax) break;
                            const uint32_t r = cbx.rng[k];
                            if ((yzm >> k & 1u) && (uint32_t)qx >= (r & 31u) && (uint32_t)qx < (r >> 5 & 31u))
                                e = cbx.val[k];
                        }
                    } else {
                        x[0] = sample_coord(ci[0], qx, s, n);
                        e = boxcand && cand4.count >= 0 ? eps_boxes_cand<D, double>(a.eps, x, rows, cand4)
                                                        : eps_eval_cell<D, double, EKF>(a.eps, ecell, x, rows, nrows);
                    }
                    double Mx[3];
                    moments64(s, qx, Mx);
                    L0 += e;
#pragma unroll
                    for (int t = 0; t < 3; ++t) L[t] += e * Mx[t];
                }
                if (D == 2) {
#pragma unroll
                    for (int t = 0; t < 3; ++t) { T1[t] += L0 * My[t]; T2[t] += L[t]; }
                } else {
#pragma unroll
                    for (int ty = 0; ty < 3; ++ty)
#pragma unroll
                        for (int tz = 0; tz < 3; ++tz) T1[ty * 3 + tz] += L0 * My[ty] * Mz[tz];
#pragma unroll
                    for (int tx = 0; tx < 3; ++tx)
#pragma unroll
                        for (int tz = 0; tz < 3; ++tz) T2[tx * 3 + tz] += L[tx] * Mz[tz];
#pragma unroll
                    for (int tx = 0; tx < 3; ++tx)
#pragma unroll
                        for (int ty = 0; ty < 3; ++ty) T3[tx * 3 + ty] += L[tx] * My[ty];
                }
            }
        }
        // reduce over the G lanes of the cell (fixed butterfly order)
#pragma unroll
        for (int off = G / 2; off > 0; off >>= 1)
#pragma unroll
            for (int k = 0; k < 9; ++k) {
                T1[k] += __shfl_xor(T1[k], off, 64);
                T2[k] += __shfl_xor(T2[k], off, 64);
                T3[k] += __shfl_xor(T3[k], off, 64);
            }
        if (valid && g == 0) {
            constexpr int nl = 1 << D, U = n_pairs(D);
            double K[U];
            double inv_s = 1.0 / s, hp = (D == 2) ? 1.0 : 1.0 / n;
#pragma unroll
            for (int aa = 0; aa < nl; ++aa)
#pragma unroll
                for (int bb = aa + 1; bb < nl; ++bb) {
                    int ax = aa & 1, bx = bb & 1, ay = (aa >> 1) & 1, by = (bb >> 1) & 1;
                    double sx = ax == bx ? inv_s : -inv_s, sy = ay == by ? inv_s : -inv_s;
                    double v;
                    if (D == 2) {
                        v = sx * T1[mtype(ay, by)] + sy * T2[mtype(ax, bx)];
                    } else {
                        int az = (aa >> 2) & 1, bz = (bb >> 2) & 1;
                        double sz = az == bz ? inv_s : -inv_s;
                        int tx = mtype(ax, bx), ty = mtype(ay, by), tz = mtype(az, bz);
                        v = hp * (sx * T1[ty * 3 + tz] + sy * T2[tx * 3 + tz] + sz * T3[tx * 3 + ty]);
                    }
                    K[pair_index(D, aa, bb)] = v;
                }
            if constexpr (sizeof(TO) == 8) {
                store_and_check<D, double>(a, i, cell, K);
            } else {
                TO Kt[U];
#pragma unroll
                for (int p = 0; p < U; ++p) Kt[p] = (TO)K[p];
                store_and_check<D, TO>(a, i, cell, Kt);
            }
        }
        if (!STRIDE) return;
        __syncthreads();  // the candidate list is rebuilt for the next tile
    }
}

// ------------------------------------------------------------ mixed (MFMA)
// bf16 bits of f, rounded to nearest even by the hardware conversion
__device__ inline uint16_t bf16_rne_hw(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }
__device__ inline float bf16_value(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

union BF8 {
    bf16x8 v;
    uint16_t u[8];
};

// A wave handles TPW groups of 16 cells; lane l owns cell row l & 15 and
// samples 8 (l >> 4) .. +7 of every 32-sample chunk (the A-operand layout of
// v_mfma_f32_16x16x32_bf16); the B operand (G terms) is pre-laid out per
// lane.  The block's 64 TPW consecutive list entries share one candidate
// list, so small s (one chunk per cell) takes TPW = 4.
template <int D, int NT, int NTERM, int TPW, bool WL, int EK>
__device__ __forceinline__ void integrate_mfma_tile(const AsmArgs &a, const uint4 *Gtab, int nchunks, float inv_den,
                                                    int64_t blk, int64_t cnt, float (*sm)[16][NT * 16 + 1],
                                                    float (*ko)[16][n_pairs(D) + 1], CandLDS &cand,
                                                    double (*wrows)[kWaveCand * 7])
{
    constexpr int EKF = EK == kBoxesSmall ? MGD_EPS_BOXES : EK;  // the field kind evaluated
    int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    int row = lane & 15, kg = lane >> 4;
    const int64_t blk0 = blk * (64 * TPW);
    int s = a.s, n = a.n;
    // candidate box: thread t stands for entries blk0 + t + 256 j of the
    // block's 64 TPW
    int clo[3] = {0x7fffffff, 0x7fffffff, 0x7fffffff}, chi[3] = {-1, -1, -1};
    bool any = false;
    for (int j = 0; j * 256 < 64 * TPW; ++j) {
        const int t = (int)threadIdx.x + 256 * j;
        int64_t i = blk0 + t;
        if (t < 64 * TPW && i < cnt) {
            int cj[3] = {0, 0, 0};
            cell_coords<D>(a.cells ? a.cells[i] : i, n, cj);
            for (int m = 0; m < D; ++m) {
                clo[m] = min(clo[m], cj[m]);
                chi[m] = max(chi[m], cj[m]);
            }
            any = true;
        }
    }
    const double *rows = a.eps.data;
    int nrows = a.eps.count;
    // contiguous cells share one list per block; scattered ones (WL) take
    // one per wave below
    if (!WL) build_candidates<D>(a.eps, n, any, clo, chi, cand, &rows, &nrows);
    int64_t nq = 1;
    for (int m = 0; m < D; ++m) nq *= s;
    for (int j = 0; j < TPW; ++j) {
        const int64_t tile = blk0 + (int64_t)(j * 4 + wave) * 16;
        const int64_t i = tile + row;
        const bool valid = i < cnt;
        const int64_t cell = valid ? (a.cells ? a.cells[i] : i) : 0;
        int ci[3] = {0, 0, 0};
        cell_coords<D>(cell, n, ci);
        if (WL) build_candidates_wave<D>(a.eps, n, valid, ci, wrows[wave], &rows, &nrows);
        EpsCell<D, float> ecell;
        if (EKF < 0 || EKF == MGD_EPS_LATTICE) eps_cell_prepare<D, float>(a.eps, n, valid, ci, ecell);
        // boxes from s = 8 on (below, preparing a cell's ranges costs about
        // what the per-sample test does): the wave paints from the ranges
        // unless a lane's cell is reached by more than kCellBoxes boxes
        CellBoxes<float> cbx;
        cbx.count = 0;
        bool fastbox = false;
        int kmax = 0;
        uint32_t yzm = 0;
        const float bg = (float)a.eps.p0;
        if (EK == MGD_EPS_BOXES && s >= 8) {
            if (valid) cell_boxes<D, float, true>(ci, s, n, kg * 8, rows, nrows, cbx);
            int c = cbx.count, over = cbx.count < 0 ? 1 : 0;
            for (int off = 32; off > 0; off >>= 1) {
                c = max(c, __shfl_xor(c, off));
                over = max(over, __shfl_xor(over, off));
            }
            fastbox = over == 0;
            kmax = c;
        }
        // sample q = ch 32 + kg 8 + e has x-index q mod s = (kg 8 + e) mod s
        // for every chunk (s divides 32): the lane's eight x coordinates are
        // computed once; y and z only when q / s changes
        const int ls = 31 - __clz(s);
        double xq[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) xq[e] = sample_coord(ci[0], (kg * 8 + e) & (s - 1), s, n);
        int qr_last = -1;
        double xy = 0.0, xz = 0.0;
        // a lattice field on a cell inside one lattice cell: eps = exp(p0 g)
        // with g trilinear in the corner values, so along the lane's x-line
        // (y and z fixed) p0 g log2(e) = ga + t_x gb, and a sample costs one
        // FMA and one exp2; ga and gb change with y and z only
        const int kind = EKF >= 0 ? EKF : a.eps.kind;
        const bool lat = kind == MGD_EPS_LATTICE && ecell.ok;
        const float kexp = (float)(a.eps.p0 * 1.4426950408889634);
        float txl[8], ga = 0.0f, gb = 0.0f;
        if (lat) {
#pragma unroll
            for (int e = 0; e < 8; ++e) txl[e] = (float)(xq[e] * a.eps.count - ecell.base[0]);
        }
        floatx4 acc[NT];
        for (int t = 0; t < NT; ++t) acc[t] = floatx4{0.f, 0.f, 0.f, 0.f};
        int nch = tile < cnt ? nchunks : 0;  // idle waves still reach the barriers
        for (int ch = 0; ch < nch; ++ch) {
            BF8 ahi, alo;
            const int q0 = ch * 32 + kg * 8;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int q = q0 + e;
                float ev = 0.0f;
                if (valid && q < nq) {
                    if (kind == MGD_EPS_SAMPLES) {
                        ev = (float)a.samples[i * nq + q];
                    } else if (EK == MGD_EPS_BOXES && fastbox) {
                        const int qr = q >> ls;
                        if (qr != qr_last) {
                            // the kept boxes whose y and z ranges hold this sample row
                            const uint32_t qy = (uint32_t)(qr & (s - 1)), qz = D == 3 ? (uint32_t)(qr >> ls) : 0u;
                            yzm = 0;
#pragma unroll
                            for (int k = 0; k < kCellBoxes; ++k) {
                                if (k >= kmax) break;
                                const uint32_t r = cbx.rng[k];
                                if (k < cbx.count && qy >= (r & 31u) && qy < (r >> 5 & 31u) && qz >= (r >> 10 & 31u) &&
                                    qz < (r >> 15 & 31u))
                                    yzm |= 1u << k;
                            }
                            qr_last = qr;
                        }
                        float v = bg;
#pragma unroll
                        for (int k = 0; k < kCellBoxes; ++k) {
                            if (k >= kmax) break;
                            if ((yzm >> k & 1u) && (cbx.rng[k] >> (20 + e) & 1u)) v = cbx.val[k];
                        }
                        ev = v;
                    } else {
                        const int qr = q >> ls;
                        if (qr != qr_last) {
                            xy = sample_coord(ci[1], qr & (s - 1), s, n);
                            if (D == 3) xz = sample_coord(ci[2], qr >> ls, s, n);
                            qr_last = qr;
                            if (lat) {
                                const float t1 = (float)(xy * a.eps.count - ecell.base[1]);
                                const float t2 = D == 3 ? (float)(xz * a.eps.count - ecell.base[2]) : 0.0f;
                                float f0 = 0.0f, f1 = 0.0f;  // faces x = 0 and x = 1
#pragma unroll
                                for (int c = 0; c < (1 << (D - 1)); ++c) {
                                    const float w = ((c & 1) ? t1 : 1.0f - t1) *
                                                    (D == 3 ? ((c & 2) ? t2 : 1.0f - t2) : 1.0f);
                                    f0 += w * ecell.corner[2 * c];
                                    f1 += w * ecell.corner[2 * c + 1];
                                }
                                ga = kexp * f0;
                                gb = kexp * (f1 - f0);
                            }
                        }
                        if (lat) {
                            // |p0 g| stays far inside the normal range of exp2
                            ev = __builtin_amdgcn_exp2f(ga + txl[e] * gb);
                        } else {
                            const double x[3] = {xq[e], xy, xz};
                            ev = eps_eval_cell<D, float, EKF>(a.eps, ecell, x, rows, nrows);
                        }
                    }
                }
                uint16_t h = bf16_rne_hw(ev);
                ahi.u[e] = h;
                alo.u[e] = bf16_rne_hw(ev - bf16_value(h));
            }
            for (int t = 0; t < NT; ++t) {
                const uint4 *gp = Gtab + ((size_t)(ch * NT + t) * NTERM) * 64 + lane;
                BF8 g0, g1;
                *(uint4 *)&g0 = gp[0];
                *(uint4 *)&g1 = gp[64];
                acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi.v, g0.v, acc[t], 0, 0, 0);
                acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi.v, g1.v, acc[t], 0, 0, 0);
                acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(alo.v, g0.v, acc[t], 0, 0, 0);
                if (NTERM == 3) {
                    BF8 g2;
                    *(uint4 *)&g2 = gp[128];
                    acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi.v, g2.v, acc[t], 0, 0, 0);
                }
            }
        }
        // C layout: lane holds column lane & 15, rows 4 (lane >> 4) + r
        if (j > 0) __syncthreads();  // the previous group's rows are read
        for (int t = 0; t < NT; ++t)
            for (int r = 0; r < 4; ++r) sm[wave][4 * kg + r][t * 16 + (lane & 15)] = acc[t][r] * inv_den;
        __syncthreads();
        constexpr int U = n_pairs(D);
        if (!a.k_by_cell || !a.cells) {
            // the group's 16 rows are contiguous in K_old and K_out: all 64
            // lanes move them in contiguous pieces through LDS
            const int nrow = tile < cnt ? (int)min((int64_t)16, cnt - tile) : 0;
            if (a.K_old) {
                const float *Ko = (const float *)a.K_old + tile * U;
                for (int e = lane; e < nrow * U; e += 64) ko[wave][e / U][e % U] = Ko[e];
                __syncthreads();
                if (lane < 16 && valid) {
                    float K[U], old[U];
                    for (int p = 0; p < U; ++p) { K[p] = sm[wave][lane][p]; old[p] = ko[wave][lane][p]; }
                    const double rel = ladder_rel<D, float>(K, old);
                    if (a.rel_out) a.rel_out[i] = rel;
                    if (a.done_out) a.done_out[i] = rel < a.C ? 1 : 0;
                }
            }
            float *Kout = (float *)a.K_out + tile * U;
            for (int e = lane; e < nrow * U; e += 64) Kout[e] = sm[wave][e / U][e % U];
        } else if (lane < 16 && valid) {
            float K[U];
            for (int p = 0; p < U; ++p) K[p] = sm[wave][lane][p];
            store_and_check<D, float>(a, i, cell, K);
        }
    }
}

template <int D, int NT, int NTERM, int TPW, bool STRIDE, int EK>
__global__ __launch_bounds__(256) void k_integrate_mfma(AsmArgs a, const uint4 *Gtab, int nchunks,
                                                        float inv_den)
{
    __shared__ float sm[4][16][NT * 16 + 1];
    __shared__ float ko[4][16][n_pairs(D) + 1];
    __shared__ CandLDS cand;
    __shared__ double wrows[STRIDE ? 4 : 1][kWaveCand * 7];
    const int64_t cnt = asm_count(a);
    if (!STRIDE) {
        if ((int64_t)blockIdx.x * (64 * TPW) < cnt)
            integrate_mfma_tile<D, NT, NTERM, TPW, false, EK>(a, Gtab, nchunks, inv_den, blockIdx.x, cnt, sm, ko, cand,
                                                              wrows);
        return;
    }
    for (int64_t blk = blockIdx.x; blk * (64 * TPW) < cnt; blk += gridDim.x) {
        integrate_mfma_tile<D, NT, NTERM, TPW, true, EK>(a, Gtab, nchunks, inv_den, blk, cnt, sm, ko, cand, wrows);
        __syncthreads();  // the candidate list and the row buffer are reused by the next tile
    }
}

// ------------------------------------------------------------ G tables
// Exact integer-scaled sub-cell matrices: 2D G = G_int / (6 s^4),
// 3D G = h G_int / (36 s^7); G_int split into bf16 terms exactly.
static inline uint16_t host_bf16_rne(float f)
{
    uint32_t b;
    memcpy(&b, &f, 4);
    return (uint16_t)((b + 0x7FFFu + ((b >> 16) & 1u)) >> 16);
}
static inline float host_bf16_val(uint16_t h)
{
    uint32_t b = (uint32_t)h << 16;
    float f;
    memcpy(&f, &b, 4);
    return f;
}

struct GTable {
    int dim = 0, s = 0, nterm = 0, nchunks = 0, nt = 0;
    uint4 *dev = nullptr;
};
static GTable g_tables[2][5];  // [dim-2][log2 s]
static int g_tables_device = -1;

static int build_gtable(mgd_ctx *ctx, int D, int s, GTable &T)
{
    int nl = 1 << D, U = n_pairs(D);
    int64_t nq = 1;
    for (int m = 0; m < D; ++m) nq *= s;
    // integer moments m_t(q) = 6 s^3 M_t(q)
    auto mint = [&](int q, int t) -> int64_t {
        int64_t qb = s - 1 - q;
        if (t == 2) return 2 * (3LL * q * q + 3LL * q + 1);
        if (t == 0) return 2 * (3 * qb * qb + 3 * qb + 1);
        return 6LL * q * (s - q) + 3LL * (s - 2 * q) - 2;
    };
    std::vector<int64_t> Gint((size_t)nq * U);
    int64_t gmax = 0;
    for (int64_t q = 0; q < nq; ++q) {
        int qq[3] = {(int)(q % s), (int)((q / s) % s), (int)(q / ((int64_t)s * s))};
        for (int a = 0; a < nl; ++a)
            for (int b = a + 1; b < nl; ++b) {
                int64_t sum = 0;
                for (int k = 0; k < D; ++k) {
                    int64_t term = (((a >> k) & 1) == ((b >> k) & 1)) ? 1 : -1;
                    for (int m = 0; m < D; ++m)
                        if (m != k) term *= mint(qq[m], ((a >> m) & 1) + ((b >> m) & 1));
                    sum += term;
                }
                Gint[(size_t)q * U + pair_index(D, a, b)] = sum;
                gmax = sum > gmax ? sum : (-sum > gmax ? -sum : gmax);
            }
    }
    if (gmax >= (1LL << 24))
        return mgd_fail(ctx, MGD_EINVAL, "G table entries exceed 24 bits (d=%d s=%d)", D, s);
    // number of exact bf16 terms
    int nterm = 2;
    for (size_t k = 0; k < Gint.size(); ++k) {
        float g = (float)Gint[k];
        uint16_t h0 = host_bf16_rne(g);
        float r1 = g - host_bf16_val(h0);
        uint16_t h1 = host_bf16_rne(r1);
        float r2 = r1 - host_bf16_val(h1);
        if (r2 != 0.0f) {
            uint16_t h2 = host_bf16_rne(r2);
            if (r2 - host_bf16_val(h2) != 0.0f)
                return mgd_fail(ctx, MGD_EINVAL, "G table not exact in 3 bf16 terms");
            nterm = 3;
        }
    }
    int NT = (U + 15) / 16;
    int nchunks = (int)((nq + 31) / 32);
    size_t nvec = (size_t)nchunks * NT * nterm * 64;
    std::vector<uint16_t> host(nvec * 8, 0);
    for (int ch = 0; ch < nchunks; ++ch)
        for (int t = 0; t < NT; ++t)
            for (int lane = 0; lane < 64; ++lane) {
                int col = t * 16 + (lane & 15);
                for (int e = 0; e < 8; ++e) {
                    int64_t q = (int64_t)ch * 32 + (lane >> 4) * 8 + e;
                    float g = (col < U && q < nq) ? (float)Gint[(size_t)q * U + col] : 0.0f;
                    uint16_t terms[3];
                    terms[0] = host_bf16_rne(g);
                    float r1 = g - host_bf16_val(terms[0]);
                    terms[1] = host_bf16_rne(r1);
                    terms[2] = host_bf16_rne(r1 - host_bf16_val(terms[1]));
                    for (int k = 0; k < nterm; ++k) {
                        size_t vec = ((size_t)(ch * NT + t) * nterm + k) * 64 + lane;
                        host[vec * 8 + e] = terms[k];
                    }
                }
            }
    void *p = nullptr;
    int rc = dev_alloc(ctx, &p, nvec * 16);
    if (rc) return rc;
    HIPCHK(ctx, hipMemcpy(p, host.data(), nvec * 16, hipMemcpyHostToDevice));
    T.dim = D; T.s = s; T.nterm = nterm; T.nchunks = nchunks; T.nt = NT;
    T.dev = (uint4 *)p;
    return MGD_OK;
}

static int get_gtable(mgd_ctx *ctx, int D, int s, GTable **out)
{
    int ls = 0;
    while ((1 << ls) < s) ++ls;
    if (g_tables_device != ctx->device) {
        for (auto &row : g_tables)
            for (auto &t : row) t = GTable();
        g_tables_device = ctx->device;
    }
    GTable &T = g_tables[D - 2][ls];
    if (!T.dev) {
        int rc = build_gtable(ctx, D, s, T);
        if (rc) return rc;
    }
    *out = &T;
    return MGD_OK;
}

// ------------------------------------------------------------ launchers
int launch_assemble(mgd_ctx *ctx, int dim, int n, int s, const int64_t *cells, int64_t count,
                    const mgd_eps *eps, int mode, void *K_out, const void *K_old, int k_by_cell,
                    double C, double *rel_out, uint8_t *done_out, const int64_t *count_dev,
                    hipStream_t st, int keep_old)
{
    if (count <= 0) return MGD_OK;
    AsmArgs a;
    a.keep_old = keep_old;
    a.n = n; a.s = s; a.count = count; a.count_dev = count_dev; a.cells = cells;
    a.eps.kind = eps->kind; a.eps.dim = eps->dim; a.eps.count = eps->count;
    a.eps.p0 = eps->p0; a.eps.p1 = eps->p1; a.eps.data = eps->data;
    a.samples = eps->kind == MGD_EPS_SAMPLES ? eps->data : nullptr;
    a.K_out = K_out; a.K_old = K_old;
    a.k_by_cell = k_by_cell; a.C = C; a.rel_out = rel_out; a.done_out = done_out;
    // block-stride kernels: a capped grid covers any count (the ladder's
    // counts live on the device; `count` is only the host's bound)
    constexpr unsigned kAsmMaxBlocks = 4096;
    // the mixed form's rungs with s <= 2 (at most 2^d samples per cell) are
    // too short a contraction for the matrix cores: FP64 on the vector
    // units, rounded to FP32
    if (mode == MGD_FP64 || s <= 2) {
        // lanes per cell: the per-cell tail (element matrix, criterion,
        // stores) runs on one lane of the G.  In 3D (28 pairs per cell) the
        // tail dominates short rungs, so fewer lanes per cell (more sample
        // lines per lane) spread it over more cells per wave; in 2D (6 pairs)
        // the later rungs' few open cells need the lanes for parallelism
        int lines = dim == 2 ? s : s * s;
        int G = dim == 3 ? (lines >= 256 ? 16 : lines >= 16 ? 4 : 1) : (lines >= 16 ? 16 : lines >= 4 ? 4 : 1);
        const bool stride = count_dev != nullptr;
        unsigned grid = grid_for(count * G, 256);
        if (stride) grid = std::min<unsigned>(grid, kAsmMaxBlocks);
#define L64K(DD, GG, TO, EK)                                                                                   \
    do {                                                                                                       \
        if (stride) hipLaunchKernelGGL((k_integrate64<DD, GG, true, TO, EK>), dim3(grid), dim3(256), 0, st, a); \
        else hipLaunchKernelGGL((k_integrate64<DD, GG, false, TO, EK>), dim3(grid), dim3(256), 0, st, a);       \
    } while (0)
        // lattice, ball and box fields: instantiations without the other kinds'
        // code (boxes from s = 8 on, where painting from index ranges pays for
        // the registers it takes)
#define L64T(DD, GG, TO)                                                                 \
    do {                                                                                 \
        if (a.eps.kind == MGD_EPS_LATTICE) L64K(DD, GG, TO, MGD_EPS_LATTICE);           \
        else if (a.eps.kind == MGD_EPS_BALLS) L64K(DD, GG, TO, MGD_EPS_BALLS);          \
        else if (a.eps.kind == MGD_EPS_BOXES && s >= 8) L64K(DD, GG, TO, MGD_EPS_BOXES); \
        else if (a.eps.kind == MGD_EPS_BOXES) L64K(DD, GG, TO, kBoxesSmall);            \
        else L64K(DD, GG, TO, -1);                                                       \
    } while (0)
#define L64(DD, GG)                                  \
    do {                                             \
        if (mode == MGD_FP64) L64T(DD, GG, double);  \
        else L64T(DD, GG, float);                    \
    } while (0)
        if (dim == 2) { if (G == 16) L64(2, 16); else if (G == 4) L64(2, 4); else L64(2, 1); }
        else { if (G == 16) L64(3, 16); else if (G == 4) L64(3, 4); else L64(3, 1); }
#undef L64
#undef L64T
#undef L64K
    } else {
        GTable *T = nullptr;
        int rc = get_gtable(ctx, dim, s, &T);
        if (rc) return rc;
        double inv_den = dim == 2 ? 1.0 / (6.0 * pow((double)s, 4)) : (1.0 / n) / (36.0 * pow((double)s, 7));
        // one chunk per cell: four 16-cell groups per wave share the block's candidates
        const bool small = T->nchunks == 1;
        const bool stride = count_dev != nullptr;
        unsigned grid = grid_for(count, small ? 256 : 64);
        if (stride) grid = std::min<unsigned>(grid, kAsmMaxBlocks);
#define LMK(DD, NT, NTERM, TPW, EK)                                                                              \
    do {                                                                                                         \
        if (stride)                                                                                              \
            hipLaunchKernelGGL((k_integrate_mfma<DD, NT, NTERM, TPW, true, EK>), dim3(grid), dim3(256), 0, st,   \
                               a, T->dev, T->nchunks, (float)inv_den);                                           \
        else                                                                                                     \
            hipLaunchKernelGGL((k_integrate_mfma<DD, NT, NTERM, TPW, false, EK>), dim3(grid), dim3(256), 0, st,  \
                               a, T->dev, T->nchunks, (float)inv_den);                                           \
    } while (0)
        // lattice, ball and box fields get instantiations without the other
        // kinds' code (the unrolled sample loop then fits the instruction
        // cache; boxes paint from per-cell index ranges, from s = 8 on)
#define LM(DD, NT, NTERM, TPW)                                                                  \
    do {                                                                                        \
        if (a.eps.kind == MGD_EPS_LATTICE) LMK(DD, NT, NTERM, TPW, MGD_EPS_LATTICE);           \
        else if (a.eps.kind == MGD_EPS_BALLS) LMK(DD, NT, NTERM, TPW, MGD_EPS_BALLS);          \
        else if (a.eps.kind == MGD_EPS_BOXES && s >= 8) LMK(DD, NT, NTERM, TPW, MGD_EPS_BOXES); \
        else if (a.eps.kind == MGD_EPS_BOXES) LMK(DD, NT, NTERM, TPW, kBoxesSmall);            \
        else LMK(DD, NT, NTERM, TPW, -1);                                                       \
    } while (0)
        if (dim == 2) {
            if (T->nterm == 2) { if (small) LM(2, 1, 2, 4); else LM(2, 1, 2, 1); }
            else { if (small) LM(2, 1, 3, 4); else LM(2, 1, 3, 1); }
        } else {
            if (T->nterm == 2) { if (small) LM(3, 2, 2, 4); else LM(3, 2, 2, 1); }
            else { if (small) LM(3, 2, 3, 4); else LM(3, 2, 3, 1); }
        }
#undef LM
#undef LMK
    }
    HIPCHK(ctx, hipGetLastError());
    return MGD_OK;
}

// centre samples eps(x_c) as FP32 (the base of the hierarchical surplus)
template <int D> __global__ void k_centre_eps(EpsDev e, int n, int64_t ncell, float *out)
{
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool valid = c < ncell;
    int ci[3] = {0, 0, 0};
    cell_coords<D>(valid ? c : 0, n, ci);
    __shared__ CandLDS cand;
    const double *rows;
    int nrows;
    build_candidates<D>(e, n, valid, ci, ci, cand, &rows, &nrows);
    if (!valid) return;
    double x[3];
    for (int m = 0; m < D; ++m) x[m] = sample_coord(ci[m], 0, 1, n);
    out[c] = eps_eval<D, float>(e, x, rows, nrows);
}

int launch_centre_eps(mgd_ctx *ctx, int dim, int n, const mgd_eps *eps, float *eps_c, hipStream_t st)
{
    EpsDev e{eps->kind, eps->dim, eps->count, eps->p0, eps->p1, eps->data};
    int64_t nc = 1;
    for (int m = 0; m < dim; ++m) nc *= n;
    if (dim == 2) hipLaunchKernelGGL(k_centre_eps<2>, dim3(grid_for(nc, 256)), dim3(256), 0, st, e, n, nc, eps_c);
    else hipLaunchKernelGGL(k_centre_eps<3>, dim3(grid_for(nc, 256)), dim3(256), 0, st, e, n, nc, eps_c);
    HIPCHK(ctx, hipGetLastError());
    return MGD_OK;
}

// ------------------------------------------------------------ stencil gather
// coupling of vertex v to v+o: sum over the cells holding both, ascending
template <int D, typename TK, typename TS>
__global__ void k_gather(const TK *K, int n, TS *S)
{
    Grid<D> g(n);
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= g.NV) return;
    int x[3] = {0, 0, 0};
    g.coords(v, x);
    constexpr int H = n_half(D), U = n_pairs(D);
    for (int j = 0; j < H; ++j) {
        int o[3] = {half_off(D, j, 0), half_off(D, j, 1), D == 3 ? half_off(D, j, 2) : 0};
        TK acc = 0;
        bool first = true;
        for (int B = (1 << D) - 1; B >= 0; --B) {
            bool ok = true;
            int lv = 0, lw = 0;
            int64_t c = 0, stride = 1;
            for (int m = 0; m < D; ++m) {
                int bm = (B >> m) & 1, cm = x[m] - bm, wm = bm + o[m];
                if (cm < 0 || cm >= n || wm < 0 || wm > 1) ok = false;
                lv |= bm << m;
                lw |= wm << m;
                c += (int64_t)cm * stride;
                stride *= n;
            }
            if (!ok) continue;
            TK k = K[c * U + pair_index(D, lv, lw)];
            acc = first ? k : acc + k;
            first = false;
        }
        S[(int64_t)j * g.NV + v] = (TS)acc;
    }
}

// 3D gather staged through LDS.  A block owns the vertices
// [x0, x0 + 64) x [y0, y0 + TY) and marches over the vertex planes
// [z0, z0 + kGatherZ).  A coupling of vertex v is a pair (a, b), a < b, of
// local vertices of a cell with v at corner a; pairs with a on the cell's low
// z face (pair indices 0..21) come from cell layer z, those with a on its high
// z face (22..27) from layer z - 1.  Each step loads cell layer z whole, in
// 16-byte pieces along contiguous cell rows, and keeps its high-face pairs
// for the next plane, so every element matrix is read once per march.  The
// sums run over the same cells in the same order as k_gather.
constexpr int kGatherZ = 16;
template <typename TK, typename TS, int TY>
__global__ __launch_bounds__(64 * TY) void k_gather3(const TK *K, int n, TS *S)
{
    constexpr int U = 28, LO = 22, HI = U - LO, CX = 65, CY = TY + 1;
    constexpr int RL = 23, RH = 7;  // odd row strides: conflict-free lanes
    constexpr int VW = 16 / sizeof(TK), NQ = U / VW, NT = 64 * TY;
    __shared__ TK lo[CY][CX][RL];
    __shared__ TK hi[2][CY][CX][RH];
    const int tid = threadIdx.x, tx = tid & 63, ty = tid >> 6;
    const int x0 = blockIdx.x * 64, y0 = blockIdx.y * TY, z0 = blockIdx.z * kGatherZ;
    const int64_t nv = n + 1, NV = nv * nv * nv;
    // every thread issues all its loads of a layer before any LDS store
    constexpr int NI = (CY * CX * NQ + NT - 1) / NT;
    using V16 = typename std::conditional<VW == 4, float4, double2>::type;
    auto load_layer = [&](int cz, int hb) {
        if (cz < 0 || cz >= n) return;
        V16 w[NI];
        bool ok[NI];
#pragma unroll
        for (int it = 0; it < NI; ++it) {
            const int e = tid + it * NT;
            const int r = e / (CX * NQ), k = e - r * (CX * NQ), i = k / NQ, q = k - i * NQ;
            const int cy = y0 - 1 + r, cx = x0 - 1 + i;
            ok[it] = e < CY * CX * NQ && cy >= 0 && cy < n && cx >= 0 && cx < n;
            if (ok[it]) w[it] = *reinterpret_cast<const V16 *>(K + (cx + (int64_t)n * (cy + (int64_t)n * cz)) * U + q * VW);
        }
#pragma unroll
        for (int it = 0; it < NI; ++it) {
            if (!ok[it]) continue;
            const int e = tid + it * NT;
            const int r = e / (CX * NQ), k = e - r * (CX * NQ), i = k / NQ, q = k - i * NQ;
            const TK *wv = reinterpret_cast<const TK *>(&w[it]);
#pragma unroll
            for (int t = 0; t < VW; ++t) {
                const int pi = q * VW + t;
                if (pi < LO) lo[r][i][pi] = wv[t];
                else hi[hb][r][i][pi - LO] = wv[t];
            }
        }
    };
    load_layer(z0 - 1, (z0 - 1) & 1);
    const int zend = min(z0 + kGatherZ, n + 1);
    const int x = x0 + tx, y = y0 + ty;
    for (int z = z0; z < zend; ++z) {
        __syncthreads();  // the previous plane has read lo and hi[z & 1]
        load_layer(z, z & 1);
        __syncthreads();
        if (x > n || y > n) continue;
        const int xv[3] = {x, y, z};
        const int64_t v = x + nv * (y + nv * (int64_t)z);
#pragma unroll
        for (int j = 0; j < 13; ++j) {
            const int o[3] = {half_off(3, j, 0), half_off(3, j, 1), half_off(3, j, 2)};
            TK acc = 0;
            bool first = true;
#pragma unroll
            for (int B = 7; B >= 0; --B) {
                bool ok = true;
                int lw = 0;
#pragma unroll
                for (int m = 0; m < 3; ++m) {
                    const int bm = (B >> m) & 1, cm = xv[m] - bm, wm = bm + o[m];
                    if (cm < 0 || cm >= n || wm < 0 || wm > 1) ok = false;
                    lw |= wm << m;
                }
                if (!ok) continue;
                const int pi = pair_index(3, B, lw), r = ty + 1 - ((B >> 1) & 1), i = tx + 1 - (B & 1);
                const TK k = (B & 4) ? hi[(z - 1) & 1][r][i][pi - LO] : lo[r][i][pi];
                acc = first ? k : acc + k;
                first = false;
            }
            S[(int64_t)j * NV + v] = (TS)acc;
        }
    }
}

int launch_gather(mgd_ctx *ctx, int dim, int n, const void *K, int k_mode, void *S, int s_mode,
                  hipStream_t st)
{
    int64_t NV = 1;
    for (int m = 0; m < dim; ++m) NV *= (n + 1);
    dim3 gr(grid_for(NV, 256)), bl(256);
#define LG(DD, TK, TS) hipLaunchKernelGGL((k_gather<DD, TK, TS>), gr, bl, 0, st, (const TK *)K, n, (TS *)S)
#define LG3(TK, TS, TY)                                                                                \
    hipLaunchKernelGGL((k_gather3<TK, TS, TY>), dim3((n + 64) / 64, (n + TY) / TY, (n + kGatherZ) / kGatherZ), \
                       dim3(64 * TY), 0, st, (const TK *)K, n, (TS *)S)
    if (dim == 2) {
        if (k_mode == MGD_FP64) { if (s_mode == MGD_FP64) LG(2, double, double); else LG(2, double, float); }
        else { if (s_mode == MGD_FP64) LG(2, float, double); else LG(2, float, float); }
    } else if ((uintptr_t)K % 16 != 0) {
        // the staged kernel reads 16-byte pieces
        if (k_mode == MGD_FP64) { if (s_mode == MGD_FP64) LG(3, double, double); else LG(3, double, float); }
        else { if (s_mode == MGD_FP64) LG(3, float, double); else LG(3, float, float); }
    } else {
        if (k_mode == MGD_FP64) { if (s_mode == MGD_FP64) LG3(double, double, 2); else LG3(double, float, 2); }
        else { if (s_mode == MGD_FP64) LG3(float, double, 4); else LG3(float, float, 4); }
    }
#undef LG
#undef LG3
    HIPCHK(ctx, hipGetLastError());
    return MGD_OK;
}

// ------------------------------------------------------------ compaction
// stable compaction of the entries with flag == 0 (cells still climbing):
// out_cells[k] = cells[i], with a device-side count
__global__ void k_count_open(const uint8_t *done, const int64_t *count_dev, int64_t count, int32_t *block_cnt)
{
    __shared__ int32_t red[256];
    int64_t cnt = count_dev ? *count_dev : count;
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    red[threadIdx.x] = (i < cnt && !done[i]) ? 1 : 0;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) block_cnt[blockIdx.x] = red[0];
}

__global__ void k_scan_blocks(int32_t *block_cnt, int64_t nblocks, int64_t *total)
{
    // single block: exclusive scan in place, chunked
    __shared__ int64_t carry;
    __shared__ int32_t buf[1024];
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int64_t base = 0; base < nblocks; base += 1024) {
        int64_t i = base + threadIdx.x;
        int32_t v = i < nblocks ? block_cnt[i] : 0;
        buf[threadIdx.x] = v;
        __syncthreads();
        for (int o = 1; o < 1024; o <<= 1) {
            int32_t t = threadIdx.x >= o ? buf[threadIdx.x - o] : 0;
            __syncthreads();
            buf[threadIdx.x] += t;
            __syncthreads();
        }
        if (i < nblocks) block_cnt[i] = (int32_t)(carry + buf[threadIdx.x] - v);
        __syncthreads();
        if (threadIdx.x == 1023) carry += buf[1023];
        __syncthreads();
    }
    if (threadIdx.x == 0) *total = carry;
}

__global__ void k_scatter_open(const uint8_t *done, const int64_t *cells_in, const int64_t *count_dev,
                               int64_t count, const int32_t *block_off, int64_t *cells_out)
{
    __shared__ int32_t buf[256];
    int64_t cnt = count_dev ? *count_dev : count;
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    int32_t f = (i < cnt && !done[i]) ? 1 : 0;
    buf[threadIdx.x] = f;
    __syncthreads();
    for (int o = 1; o < 256; o <<= 1) {
        int32_t t = threadIdx.x >= o ? buf[threadIdx.x - o] : 0;
        __syncthreads();
        buf[threadIdx.x] += t;
        __syncthreads();
    }
    if (f) cells_out[block_off[blockIdx.x] + buf[threadIdx.x] - 1] = cells_in ? cells_in[i] : i;
}

int launch_compact_open(mgd_ctx *ctx, const uint8_t *done, const int64_t *cells_in, const int64_t *count_dev,
                        int64_t count_bound, int32_t *block_tmp, int64_t *cells_out, int64_t *count_out,
                        hipStream_t st)
{
    if (count_bound <= 0) {
        HIPCHK(ctx, hipMemsetAsync(count_out, 0, sizeof(int64_t), st));
        return MGD_OK;
    }
    int64_t nb = (count_bound + 255) / 256;
    hipLaunchKernelGGL(k_count_open, dim3(nb), dim3(256), 0, st, done, count_dev, count_bound, block_tmp);
    hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(1024), 0, st, block_tmp, nb, count_out);
    hipLaunchKernelGGL(k_scatter_open, dim3(nb), dim3(256), 0, st, done, cells_in, count_dev, count_bound,
                       block_tmp, cells_out);
    HIPCHK(ctx, hipGetLastError());
    return MGD_OK;
}

// ------------------------------------------------------------ misc
int mgd_fail(mgd_ctx *ctx, int code, const char *fmt, ...)
{
    if (ctx) {
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(ctx->err, sizeof(ctx->err), fmt, ap);
        va_end(ap);
    }
    return code;
}

// bytes handed out by dev_alloc on this host thread (footprint accounting)
thread_local size_t g_dev_alloc_bytes = 0;

int dev_alloc(mgd_ctx *ctx, void **p, size_t bytes)
{
    *p = nullptr;
    if (bytes == 0) bytes = 16;
    g_dev_alloc_bytes += bytes;
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        return mgd_fail(ctx, MGD_ENOMEM, "hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
    }
    return MGD_OK;
}

void dev_free(void *p)
{
    if (p) (void)hipFree(p);
}
