// Multigrid cycle kernels (paper Sec. 4 and 4.1): damped Jacobi
// u <- u + omega D^{-1} (f - A u), residual, restriction R = P^T,
// prolongation, on any operator view: FP64 / FP32 half stencils or the
// compressed surplus store decoded on the fly; plus the FP64 outer residual
// and the vector kernels of the outer iteration, with deterministic
// (fixed-order) reductions.
#include <algorithm>
#include <vector>

#include "common.h"

// ------------------------------------------------------------ operator views
template <typename T> struct OpHalf {
    const T *S;
    int64_t NV;
    __device__ inline T c(int64_t v, int j, const int *) const { return S[(int64_t)j * NV + v]; }
};


// ------------------------------------------------------------ reductions
template <int BS> __device__ inline double block_sum(double v, double *red)
{
    red[threadIdx.x] = v;
    __syncthreads();
    for (int o = BS / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    double r = red[0];
    __syncthreads();
    return r;
}

// (A u)_v and the diagonal D_v = -sum of the couplings of v (interior v)
template <int D, class Op, typename T>
__device__ inline void apply_row(const Op &A, const Grid<D> &g, int64_t v, const int *x, const T *u, T &Au, T &Dv)
{
    constexpr int H = n_half(D);
    T acc = (T)0, dsum = (T)0;
    for (int j = 0; j < H; ++j) {
        int64_t lin = half_lin(D, j, g.nv);
        T a = A.c(v, j, x);
        acc += a * u[v + lin];
        dsum += a;
        int y[3] = {x[0] - half_off(D, j, 0), x[1] - half_off(D, j, 1), D == 3 ? x[2] - half_off(D, j, 2) : 0};
        T b = A.c(v - lin, j, y);
        acc += b * u[v - lin];
        dsum += b;
    }
    Dv = -dsum;
    Au = Dv * u[v] + acc;
}

// MODE 0: Jacobi sweep out = u + omega (f - A u) / D; MODE 1: residual out = f - A u;
// ZERO: u treated as 0 (first sweep from a zero start).
template <int D, class Op, typename T, int MODE, bool ZERO>
__global__ __launch_bounds__(256) void k_sweep(Op A, int n, const T *u, const T *f, T *out, T omega, double *partial)
{
    constexpr int mode = MODE;
    constexpr bool zero_guess = ZERO;
    __shared__ double red[256];
    Grid<D> g(n);
    int64_t v = block_index<D>() * blockDim.x + threadIdx.x;
    double rr = 0.0;
    if (v < g.NV) {
        int x[3] = {0, 0, 0};
        g.coords(v, x);
        if (!g.interior(x)) {
            out[v] = (T)0;
        } else {
            T Au, Dv;
            if (zero_guess) {
                constexpr int H = n_half(D);
                T dsum = (T)0;
                for (int j = 0; j < H; ++j) {
                    int64_t lin = half_lin(D, j, g.nv);
                    int y[3] = {x[0] - half_off(D, j, 0), x[1] - half_off(D, j, 1), D == 3 ? x[2] - half_off(D, j, 2) : 0};
                    dsum += A.c(v, j, x) + A.c(v - lin, j, y);
                }
                Dv = -dsum;
                Au = (T)0;
            } else {
                apply_row<D, Op, T>(A, g, v, x, u, Au, Dv);
            }
            T r = f[v] - Au;
            rr = (double)r * (double)r;
            if (mode == 0) out[v] = (zero_guess ? (T)0 : u[v]) + omega * r / Dv;
            else out[v] = r;
        }
    }
    if (partial) {
        double s = block_sum<256>(rr, red);
        if (threadIdx.x == 0) partial[blockIdx.x] = s;
    }
}

// ---- 3D sweep and residual in items of four vertices (n % 4 == 0).  Per
// half slot one 4-wide load brings the item's own couplings and one its
// mirrored ones (those of v - o), and the nine iterate rows it touches come
// as 6-value segments: a vertex costs about a third of the memory
// instructions of k_sweep, whose instruction count, not HBM, set its pace at
// 512^3.  Each vertex takes the same terms in the same order as k_sweep, so
// the results are the same bits.
template <typename T, int MODE, bool ZERO>
__global__ __launch_bounds__(256) void k_sweep3x4(const T *__restrict__ S, int n, const T *__restrict__ u,
                                                  const T *__restrict__ f, T *__restrict__ out, T omega)
{
    uint32_t x0, y, z;
    if (!items4_at(n, (blockIdx.x >> 3) * 256u + threadIdx.x, blockIdx.x & 7u, x0, y, z)) return;
    const size_t nv = (size_t)n + 1, NV = nv * nv * nv;
    const size_t v = x0 + nv * (y + nv * z);
    if (x0 == 1) out[v - 1] = (T)0;
    T o[4] = {(T)0, (T)0, (T)0, (T)0};
    if (y != 0 && z != 0 && y != (uint32_t)n && z != (uint32_t)n) {
        T U[9][6];
        if (!ZERO) {
            // x0 + 4 lies past the row's end on its last item (the last row
            // of the array has nothing after it); vertex n, the one that
            // would use it, is a boundary vertex.  In FP32 that item reads
            // its pair one place lower and zeroes the missing value, so no
            // load sits behind a branch and all of them issue together (80
            // -> 64 VGPRs); the FP64 kernel keeps the branch: with the same
            // change its 3D solves took 5-7 % longer
            const bool last = x0 + 3 >= (uint32_t)n;
#pragma unroll
            for (int r = 0; r < 9; ++r) {
                const T *p = u + v - 1 + (ptrdiff_t)(r % 3 - 1) * (ptrdiff_t)nv + (ptrdiff_t)(r / 3 - 1) * (ptrdiff_t)(nv * nv);
                ldv4(p, U[r]);
                if constexpr (sizeof(T) == 4) {
                    T t[2];
                    ldv2(p + (last ? 3 : 4), t);
                    U[r][4] = last ? t[1] : t[0];
                    U[r][5] = last ? (T)0 : t[1];
                } else if (!last) {
                    ldv2(p + 4, U[r] + 4);
                } else {
                    U[r][4] = p[4];
                    U[r][5] = (T)0;
                }
            }
        }
        T acc[4] = {(T)0, (T)0, (T)0, (T)0}, dsum[4] = {(T)0, (T)0, (T)0, (T)0};
#pragma unroll
        for (int j = 0; j < 13; ++j) {
            const int ox = half_off(3, j, 0), oy = half_off(3, j, 1), oz = half_off(3, j, 2);
            const ptrdiff_t lin = ox + (ptrdiff_t)oy * (ptrdiff_t)nv + (ptrdiff_t)oz * (ptrdiff_t)(nv * nv);
            const T *Sj = S + (size_t)j * NV;
            T A[4], B[4];
            ldv4(Sj + v, A);
            ldv4(Sj + v - lin, B);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                if (ZERO) {
                    dsum[i] += A[i] + B[i];
                } else {
                    acc[i] += A[i] * U[(oy + 1) + 3 * (oz + 1)][1 + ox + i];
                    dsum[i] += A[i];
                    acc[i] += B[i] * U[(1 - oy) + 3 * (1 - oz)][1 - ox + i];
                    dsum[i] += B[i];
                }
            }
        }
        T F[4];
        ldv4(f + v, F);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const T Dv = -dsum[i];
            const T Au = ZERO ? (T)0 : Dv * U[4][1 + i] + acc[i];
            const T r = F[i] - Au;
            o[i] = MODE == 1 ? r : (ZERO ? (T)0 : U[4][1 + i]) + omega * r / Dv;
        }
        if (x0 + 3 == (uint32_t)n) o[3] = (T)0;
    }
    stv4(out + v, o);
}

// ---- 3D mixed finest level in items of four, the default path.  The FP32
// decode streams 52 bytes of couplings per vertex, yet in a tier-0 tile (no
// stored surplus, Sec. 5.5) every coupling is the centre-sample base alone:
// a function of the 2 x 2 x 2 cells around the vertex, whose samples cost
// 4 bytes per cell.  k_item_mask marks with 1 each item (natural order
// c + T (y + nv z), x0 = 1 + 4c) whose coupling sources all lie in tier-0
// tiles: its own couplings (tiles of v and v + 3) and the mirrored ones of
// every half slot j (tiles of v - o_j and v - o_j + 3).  Boundary rows get 0.
__global__ __launch_bounds__(256) void k_item_mask(const uint8_t *__restrict__ tier, int n, uint8_t *__restrict__ im)
{
    const int64_t nv = (int64_t)n + 1, T = n >> 2;
    const int64_t id = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (id >= T * nv * nv) return;
    const int64_t t = id / T, c = id - t * T, y = t % nv, z = t / nv;
    bool all = false;
    if (y != 0 && z != 0 && y != n && z != n) {
        const int64_t v = 1 + 4 * c + nv * (y + nv * z);
        auto base = [&](int64_t w) { return tier[w >> 6] == 0 && tier[(w + 3) >> 6] == 0; };
        all = base(v);
        for (int j = 0; j < 13; ++j) all = all && base(v - half_lin(3, j, nv));
    }
    im[id] = all ? 1 : 0;
}

// Centre-sample coupling (surplus 0) between vertex x0 + i of an item and
// its neighbour at a face or body diagonal offset o, from the item's cells
// e[cz][cy][cx] = eps_c(x0 - 1 + cx, y - 1 + cy, z - 1 + cz): the samples of
// the cells holding both vertices (descending B, as the decode sums them),
// times k(o), times h, rounded once to FP32 -- the decode's value, up to the
// sign of a zero (the decode adds the zero surplus, turning -0 into +0),
// which no sum below can see: every accumulator starts at +0, and a sum of
// FP32 values that starts at +0 never becomes -0, so adding +0 or -0 leaves
// it unchanged.
__device__ inline float base_item(const float (&e)[2][2][5], int i, int o0, int o1, int o2, double hp)
{
#pragma clang fp contract(off)
    double sum = 0.0;
#pragma unroll
    for (int B = 7; B >= 0; --B) {
        const int b0 = B & 1, b1 = (B >> 1) & 1, b2 = B >> 2;
        if ((unsigned)(b0 + o0) <= 1u && (unsigned)(b1 + o1) <= 1u && (unsigned)(b2 + o2) <= 1u)
            sum = sum + (double)e[1 - b2][1 - b1][i + 1 - b0];
    }
    return (float)((sum * (-1.0 / 12.0)) * hp);
}

// k_sweep3x4<float, MODE, false> on the mixed finest level, with the
// couplings of a tier-0 item re-evaluated from eps_c (its 5 x 2 x 2 cells, 20
// floats instead of 104 couplings) and those of every other item read from
// the decode S.  Each vertex takes the same values in the same order as in
// k_sweep3x4 (vertex by vertex instead of slot by slot: the four vertices'
// sums are independent), so the results are the same bits (for finite
// iterates: the skipped zero couplings would turn an infinite u into NaN).
template <int MODE>
__global__ __launch_bounds__(256) void k_sweep3x4h(const float *__restrict__ S, const uint8_t *__restrict__ im,
                                                   const float *__restrict__ eps_c, int n, double hp,
                                                   const float *__restrict__ u, const float *__restrict__ f,
                                                   float *__restrict__ out, float omega)
{
    uint32_t x0, y, z;
    if (!items4_at(n, (blockIdx.x >> 3) * 256u + threadIdx.x, blockIdx.x & 7u, x0, y, z)) return;
    const size_t nv = (size_t)n + 1, NV = nv * nv * nv;
    const size_t v = x0 + nv * (y + nv * z);
    if (x0 == 1) out[v - 1] = 0.0f;
    float o[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    if (y != 0 && z != 0 && y != (uint32_t)n && z != (uint32_t)n) {
        const bool tier0 = im[(x0 >> 2) + (size_t)(n >> 2) * (y + nv * z)] != 0;
        // every load below the flag is issued without a branch, so that one
        // wait covers the iterate, the load and (for a tier-0 item) the
        // samples: on the item that ends a row (vertex x0 + 3 = n, a boundary
        // vertex) the two values past x0 + 2 are read one place lower, where
        // they stay inside the row, and the one that does not exist is zeroed
        const bool last = x0 + 3 >= (uint32_t)n;
        float U[9][6];
#pragma unroll
        for (int r = 0; r < 9; ++r) {
            const float *p = u + v - 1 + (ptrdiff_t)(r % 3 - 1) * (ptrdiff_t)nv + (ptrdiff_t)(r / 3 - 1) * (ptrdiff_t)(nv * nv);
            ldv4(p, U[r]);
            float t[2];
            ldv2(p + (last ? 3 : 4), t);
            U[r][4] = last ? t[1] : t[0];
            U[r][5] = last ? 0.0f : t[1];
        }
        float F[4];
        ldv4(f + v, F);
        // the item's cell samples are loaded for every item, beside the
        // iterate: a tier-0 item then waits for one round of loads, and the
        // 20 floats of another item are mostly cache hits of its neighbours.
        // The empty asm uses them here, so that the compiler cannot move the
        // loads into the tier-0 branch behind the wait for the flag.
        float e[2][2][5];
#pragma unroll
        for (int cz = 0; cz < 2; ++cz)
#pragma unroll
            for (int cy = 0; cy < 2; ++cy) {
                const float *row = eps_c + (x0 - 1) + (size_t)n * ((y - 1 + cy) + (size_t)n * (z - 1 + cz));
                ldv4(row, e[cz][cy]);
                // cell x0 + 3 exists unless vertex x0 + 3 = n
                const float e4 = row[last ? 3 : 4];
                e[cz][cy][4] = last ? 0.0f : e4;
                asm volatile("" ::"v"(e[cz][cy][0]), "v"(e[cz][cy][1]), "v"(e[cz][cy][2]), "v"(e[cz][cy][3]),
                             "v"(e[cz][cy][4]));
            }
        float acc[4] = {0.0f, 0.0f, 0.0f, 0.0f}, dsum[4] = {0.0f, 0.0f, 0.0f, 0.0f};
        if (tier0) {
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 13; ++j) {
                    const int ox = half_off(3, j, 0), oy = half_off(3, j, 1), oz = half_off(3, j, 2);
                    // couplings along one axis are k = 0 times the samples:
                    // zeros, which leave both sums unchanged for a finite
                    // iterate (see base_item)
                    if ((ox != 0) + (oy != 0) + (oz != 0) == 1) continue;
                    const float a = base_item(e, i, ox, oy, oz, hp), b = base_item(e, i, -ox, -oy, -oz, hp);
                    acc[i] += a * U[(oy + 1) + 3 * (oz + 1)][1 + ox + i];
                    dsum[i] += a;
                    acc[i] += b * U[(1 - oy) + 3 * (1 - oz)][1 - ox + i];
                    dsum[i] += b;
                }
        } else {
#pragma unroll
            for (int j = 0; j < 13; ++j) {
                const int ox = half_off(3, j, 0), oy = half_off(3, j, 1), oz = half_off(3, j, 2);
                const ptrdiff_t lin = ox + (ptrdiff_t)oy * (ptrdiff_t)nv + (ptrdiff_t)oz * (ptrdiff_t)(nv * nv);
                const float *Sj = S + (size_t)j * NV;
                float A[4], B[4];
                ldv4(Sj + v, A);
                ldv4(Sj + v - lin, B);
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    acc[i] += A[i] * U[(oy + 1) + 3 * (oz + 1)][1 + ox + i];
                    dsum[i] += A[i];
                    acc[i] += B[i] * U[(1 - oy) + 3 * (1 - oz)][1 - ox + i];
                    dsum[i] += B[i];
                }
            }
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const float Dv = -dsum[i];
            const float Au = Dv * U[4][1 + i] + acc[i];
            const float r = F[i] - Au;
            o[i] = MODE == 1 ? r : U[4][1 + i] + omega * r / Dv;
        }
        if (x0 + 3 == (uint32_t)n) o[3] = 0.0f;
    }
    stv4(out + v, o);
}

// ---- 3D sweep and residual on the compressed finest store (mixed form).
// A vertex's 26 couplings all lie in the 2 x 2 x 2 cells around it: the
// centre-sample base of the coupling to v + o sums the samples of the cells
// holding both (at most two with a nonzero unit coupling, so the order of
// the sum does not matter), times k(o) h; the surplus of an upper slot sits
// in v's tile, that of a lower slot in the tile of v - o.  Each coupling is
// base + surplus in FP64, rounded once to FP32: the values of the store's
// FP32 decode, applied in the same order as apply_row, so the results agree
// bit for bit with the sweep that reads the decode.  Cells of a tier-0 tile
// thus cost their centre samples only (4 bytes per cell instead of 52 per
// vertex): the operator is re-evaluated from eps_c on the fly.
__device__ inline void store3_couplings(const StoreView &sv, const Grid<3> &g, int64_t v, const int *x,
                                        float *own, float *low)
{
#pragma clang fp contract(off)
    const int n = g.n;
    double e[8];
    bool ok[8];
#pragma unroll
    for (int B = 0; B < 8; ++B) {
        const int c0 = x[0] - (B & 1), c1 = x[1] - ((B >> 1) & 1), c2 = x[2] - (B >> 2);
        ok[B] = c0 >= 0 && c0 < n && c1 >= 0 && c1 < n && c2 >= 0 && c2 < n;
        e[B] = ok[B] ? (double)sv.eps_c[(int64_t)c0 + (int64_t)n * (c1 + (int64_t)n * c2)] : 0.0;
    }
    const double hp = 1.0 / (double)n;
#pragma unroll
    for (int j = 0; j < 13; ++j) {
        const int o0 = half_off(3, j, 0), o1 = half_off(3, j, 1), o2 = half_off(3, j, 2);
        const int nz = (o0 != 0) + (o1 != 0) + (o2 != 0);
        // cells holding v and v + o (own) / v and v - o (low)
        double so = 0.0, sl = 0.0;
#pragma unroll
        for (int B = 7; B >= 0; --B) {
            const int b0 = B & 1, b1 = (B >> 1) & 1, b2 = B >> 2;
            const bool sh_o = (unsigned)(b0 + o0) <= 1u && (unsigned)(b1 + o1) <= 1u && (unsigned)(b2 + o2) <= 1u;
            const bool sh_l = (unsigned)(b0 - o0) <= 1u && (unsigned)(b1 - o1) <= 1u && (unsigned)(b2 - o2) <= 1u;
            if (ok[B] && sh_o) so = so + e[B];
            if (ok[B] && sh_l) sl = sl + e[B];
        }
        const double k = kref_unit(3, nz);
        const int64_t lin = half_lin(3, j, g.nv);
        own[j] = (float)((so * k) * hp + (double)sv.delta(v, j, 13));
        low[j] = (float)((sl * k) * hp + (double)sv.delta(v - lin, j, 13));
    }
}

// MODE 0: Jacobi sweep, MODE 1: residual (as k_sweep<3, ..., float>)
template <int MODE, bool ZERO>
__global__ __launch_bounds__(256) void k_sweep3_store(StoreView sv, int n, const float *u, const float *f, float *out,
                                                     float omega)
{
    Grid<3> g(n);
    int64_t v = block_index<3>() * blockDim.x + threadIdx.x;
    if (v >= g.NV) return;
    int x[3];
    g.coords(v, x);
    if (!g.interior(x)) {
        out[v] = 0.0f;
        return;
    }
    float own[13], low[13];
    store3_couplings(sv, g, v, x, own, low);
    float Au, Dv;
    if (ZERO) {
        float dsum = 0.0f;
#pragma unroll
        for (int j = 0; j < 13; ++j) dsum += own[j] + low[j];
        Dv = -dsum;
        Au = 0.0f;
    } else {
        float acc = 0.0f, dsum = 0.0f;
#pragma unroll
        for (int j = 0; j < 13; ++j) {
            const int64_t lin = half_lin(3, j, g.nv);
            acc += own[j] * u[v + lin];
            dsum += own[j];
            acc += low[j] * u[v - lin];
            dsum += low[j];
        }
        Dv = -dsum;
        Au = Dv * u[v] + acc;
    }
    const float r = f[v] - Au;
    if (MODE == 0) out[v] = (ZERO ? 0.0f : u[v]) + omega * r / Dv;
    else out[v] = r;
}

__device__ inline double pw1c(int d) { return d == 0 ? 1.0 : (d == 1 || d == -1) ? 0.5 : 0.0; }

template <int D, typename T, typename TW>
__device__ inline T wt(const TW *W, int64_t NV, int64_t v, const int *x, const int *X)
{
    int B = 0;
    for (int m = 0; m < D; ++m) {
        int b = X[m] - (x[m] >> 1);
        if (b < 0 || b > 1) return (T)0;
        B |= b << m;
    }
    if (W) return (T)W[(int64_t)B * NV + v];
    double p = 1.0;
    for (int m = 0; m < D; ++m) p *= pw1c(x[m] - 2 * X[m]);
    return (T)p;
}


// u[v] += sum_B P[v][corner B] e[corner B] (interior fine v)
template <int D, typename T>
__global__ void k_prolong(const T *W, int nf, const T *ec, T *u)
{
    Grid<D> gf(nf), gc(nf / 2);
    int64_t v = block_index<D>() * blockDim.x + threadIdx.x;
    if (v >= gf.NV) return;
    int x[3] = {0, 0, 0};
    gf.coords(v, x);
    if (!gf.interior(x)) return;
    T s = (T)0;
    // along an axis where x is even only the corner x / 2 carries weight: the
    // other corners' weights are structural zeros and are not read
    int evenmask = 0;
    for (int m = 0; m < D; ++m) evenmask |= ((x[m] & 1) ^ 1) << m;
    for (int B = 0; B < (1 << D); ++B) {
        if (B & evenmask) continue;
        int X[3] = {0, 0, 0};
        bool ok = true;
        for (int m = 0; m < D; ++m) {
            X[m] = (x[m] >> 1) + ((B >> m) & 1);
            if (X[m] > gc.n) ok = false;
        }
        if (!ok) continue;
        T w = wt<D, T, T>(W, gf.NV, v, x, X);
        if (w != (T)0) s += w * ec[gc.vid(X)];
    }
    u[v] += s;
}

// 2D restriction with the 9 fine vertices 2X + d unrolled (as k_restrict3);
// fc[X] = sum_v P[v][X] r[v] on interior X, 0 on the boundary
template <typename T, bool GEO>
__global__ __launch_bounds__(256) void k_restrict2(const T *W, int nf, const T *r, T *fc)
{
    const int nc = nf / 2;
    const int64_t nvc = nc + 1, NVc = nvc * nvc, nvf = nf + 1, NVf = nvf * nvf;
    const int64_t V = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (V >= NVc) return;
    const int X0 = (int)(V % nvc), X1 = (int)(V / nvc);
    if (X0 == 0 || X0 == nc || X1 == 0 || X1 == nc) {
        fc[V] = (T)0;
        return;
    }
    const int64_t c0 = 2 * (int64_t)X0 + nvf * 2 * (int64_t)X1;
    T s = (T)0;
#pragma unroll
    for (int sv = 0; sv < 9; ++sv) {
        const int d0 = sv % 3 - 1, d1 = sv / 3 - 1;
        const int B = (d0 < 0 ? 1 : 0) | (d1 < 0 ? 2 : 0);
        const int64_t v = c0 + d0 + nvf * d1;
        T w;
        if (GEO) w = (T)((d0 ? 0.5 : 1.0) * (d1 ? 0.5 : 1.0));
        else w = W[(int64_t)B * NVf + v];
        s += w * r[v];
    }
    fc[V] = s;
}

// 3D restriction with the 27 fine vertices 2X + d unrolled: the corner of X
// in the box of 2X + d is B_m = 1 where d_m = -1, else 0, fixed at compile
// time; the terms of R = P^T in the order of the fine offsets (x fastest)
template <typename T, bool GEO>
__global__ __launch_bounds__(256) void k_restrict3(const T *W, const uint8_t *wgeo, int nf, const T *r, T *fc)
{
    const int nc = nf / 2;
    const int64_t nvc = nc + 1, NVc = nvc * nvc * nvc, nvf = nf + 1, NVf = nvf * nvf * nvf;
    const int64_t V = block_index<3>() * blockDim.x + threadIdx.x;
    if (V >= NVc) return;
    const int X0 = (int)(V % nvc), X1 = (int)((V / nvc) % nvc), X2 = (int)(V / (nvc * nvc));
    if (X0 == 0 || X0 == nc || X1 == 0 || X1 == nc || X2 == 0 || X2 == nc) {
        fc[V] = (T)0;
        return;
    }
    const int64_t c0 = 2 * (int64_t)X0 + nvf * (2 * (int64_t)X1 + nvf * 2 * (int64_t)X2);
    T s = (T)0;
#pragma unroll
    for (int sv = 0; sv < 27; ++sv) {
        const int d0 = sv % 3 - 1, d1 = sv / 3 % 3 - 1, d2 = sv / 9 - 1;
        const int B = (d0 < 0 ? 1 : 0) | (d1 < 0 ? 2 : 0) | (d2 < 0 ? 4 : 0);
        const int64_t v = c0 + d0 + nvf * (d1 + nvf * d2);
        T w;
        if (GEO || (wgeo && wgeo[v >> 6])) w = (T)((d0 ? 0.5 : 1.0) * (d1 ? 0.5 : 1.0) * (d2 ? 0.5 : 1.0));
        else w = W[(int64_t)B * NVf + v];
        s += w * r[v];
    }
    fc[V] = s;
}

// 3D prolongation by coarse vertex: the thread of X updates the fine
// vertices 2X + b, b in {0,1}^3.  Child b takes the corners X + B with B a
// subset of b (along an even axis only the corner X_m carries weight), in
// ascending B as k_prolong, so the same bits; the 8 corner values are loaded
// once for the 8 children.
template <typename T, bool GEO>
__global__ __launch_bounds__(256) void k_prolong3(const T *W, const uint8_t *wgeo, int nf, const T *ec, T *u)
{
    const int nc = nf / 2;
    const int64_t nvc = nc + 1, NVc = nvc * nvc * nvc, nvf = nf + 1, NVf = nvf * nvf * nvf;
    const int64_t V = block_index<3>() * blockDim.x + threadIdx.x;
    if (V >= NVc) return;
    const int X0 = (int)(V % nvc), X1 = (int)((V / nvc) % nvc), X2 = (int)(V / (nvc * nvc));
    T e[8];
#pragma unroll
    for (int B = 0; B < 8; ++B) {
        const int Y0 = X0 + (B & 1), Y1 = X1 + ((B >> 1) & 1), Y2 = X2 + (B >> 2);
        e[B] = (Y0 <= nc && Y1 <= nc && Y2 <= nc) ? ec[Y0 + nvc * (Y1 + nvc * (int64_t)Y2)] : (T)0;
    }
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        const int x0 = 2 * X0 + (b & 1), x1 = 2 * X1 + ((b >> 1) & 1), x2 = 2 * X2 + (b >> 2);
        if (x0 < 1 || x0 > nf - 1 || x1 < 1 || x1 > nf - 1 || x2 < 1 || x2 > nf - 1) continue;
        const int64_t v = x0 + nvf * (x1 + nvf * (int64_t)x2);
        const bool geo = GEO || (wgeo && wgeo[v >> 6]);
        T acc = (T)0;
#pragma unroll
        for (int B = 0; B < 8; ++B) {
            if (B & ~b) continue;  // compile time after unrolling
            T w;
            if (geo) w = (T)((b & 1 ? 0.5 : 1.0) * ((b >> 1) & 1 ? 0.5 : 1.0) * ((b >> 2) & 1 ? 0.5 : 1.0));
            else w = W[(int64_t)B * NVf + v];
            if (w != (T)0) acc += w * e[B];
        }
        u[v] += acc;
    }
}

template <typename T> __global__ void k_fill(T *a, int64_t n, T val)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = val;
}

// ------------------------------------------------------------ reductions across blocks
// Kernels that produce a global sum leave one partial per block; kernels
// that need the sum add those partials themselves, every block in the same
// fixed order (so the result is deterministic and identical in all blocks);
// the residual norm's partials go straight to pinned host memory and the host
// adds them.  Reducing kernels therefore run at most kRedBlocks persistent
// blocks, which keeps the partial lists short; the generic product p -> A p
// of the outer iteration runs up to kPmvBlocks.
constexpr int kRedBlocks = 512;
constexpr int kPmvBlocks = 4096;
static inline unsigned red_grid(int64_t items) { return (unsigned)std::min<int64_t>(grid_for(items, 256), kRedBlocks); }

__device__ inline double sum_partials(const double *p, int64_t cnt, double *red)
{
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < cnt; i += 256) s += p[i];
    return block_sum<256>(s, red);
}

// ------------------------------------------------------------ staged 2D store kernels
// Finest level of the compressed store, 2D: a 64 x 4 block of vertices
// stages in LDS the centre samples of cells [x0-2, x0+64] x [y0-2, y0+3], the
// decoded couplings (centre-sample base + surplus) of vertices
// [x0-1, x0+64] x [y0-1, y0+3] and the iterate on [x0-1, x0+64] x [y0-1, y0+4];
// each vertex then reads its 4 own and 4 low-side neighbour couplings and
// its 9 iterate values from LDS.  TC: coupling / arithmetic type.
enum { ST_SWEEP = 0, ST_SWEEP0 = 1, ST_RESID = 2, ST_OUTER = 3, ST_PMATVEC = 4 };

template <typename TC> struct StageArgs {
    StoreView sv;
    int n, ntx, nt;    // cells per axis; tiles along x and in all
    const void *u;     // iterate (SWEEP/RESID: float; OUTER: double) / z (PMATVEC: float)
    const void *f;     // rhs (float / double)
    void *out;         // float / double
    const double *pold;
    double *pnew;
    double *s;         // CG scalars: [7] restart flag, zr slots
    const double *p1;  // PMATVEC: partials of z.r and z.(r - r_old), n1 each
    int64_t n1;
    int zr_old, zr_new;
    double *partial;   // one partial per block (OUTER: r.r, PMATVEC: p.Ap)
    float *rf;         // OUTER: FP32 copy of the residual (rhs of the FP32 cycle)
    float omega;
};

template <typename TC, int KIND>
__global__ __launch_bounds__(256) void k_stage2(StageArgs<TC> a)
{
#pragma clang fp contract(off)
    constexpr int BX = 64, BY = 4;
    __shared__ float s_eps[BY + 2][BX + 3];
    __shared__ TC s_c[4][BY + 1][BX + 2];
    __shared__ TC s_u[BY + 2][BX + 2];
    __shared__ double red[256];
    const int n = a.n, nv = n + 1;
    const int tid = threadIdx.x;
    double beta = 0.0, part = 0.0;
    if (KIND == ST_PMATVEC) {
        // Polak-Ribiere coefficient from the dot partials (every block sums them in the same order)
        const double zr = sum_partials(a.p1, a.n1, red), zdr = sum_partials(a.p1 + a.n1, a.n1, red);
        beta = a.s[7] != 0.0 ? 0.0 : zdr / a.s[a.zr_old];
        if (blockIdx.x == 0 && tid == 0) a.s[a.zr_new] = zr;
    }
    for (int tile = blockIdx.x; tile < a.nt; tile += gridDim.x) {
    const int x0 = (tile % a.ntx) * BX, y0 = (tile / a.ntx) * BY;
    // centre samples of cells x in [x0-2, x0+64], y in [y0-2, y0+3]
    for (int k = tid; k < (BY + 2) * (BX + 3); k += 256) {
        int cx = x0 - 2 + k % (BX + 3), cy = y0 - 2 + k / (BX + 3);
        s_eps[k / (BX + 3)][k % (BX + 3)] = (cx >= 0 && cx < n && cy >= 0 && cy < n) ? a.sv.eps_c[(int64_t)cy * n + cx] : 0.0f;
    }
    // iterate with a one-vertex halo
    for (int k = tid; k < (BY + 2) * (BX + 2); k += 256) {
        int vx = x0 - 1 + k % (BX + 2), vy = y0 - 1 + k / (BX + 2);
        TC val = (TC)0;
        if (KIND != ST_SWEEP0 && vx >= 0 && vx < nv && vy >= 0 && vy < nv) {
            int64_t v = (int64_t)vy * nv + vx;
            if (KIND == ST_PMATVEC) val = (TC)((double)((const float *)a.u)[v] + beta * a.pold[v]);
            else if (KIND == ST_OUTER) val = (TC)((const double *)a.u)[v];
            else val = (TC)((const float *)a.u)[v];
        }
        s_u[k / (BX + 2)][k % (BX + 2)] = val;
    }
    __syncthreads();
    // decoded couplings of vertices x in [x0-1, x0+64], y in [y0-1, y0+3]
    for (int k = tid; k < (BY + 1) * (BX + 2); k += 256) {
        int lx = k % (BX + 2), ly = k / (BX + 2);
        int vx = x0 - 1 + lx, vy = y0 - 1 + ly;
        TC c[4] = {(TC)0, (TC)0, (TC)0, (TC)0};
        if (vx >= 0 && vx < nv && vy >= 0 && vy < nv) {
            int64_t v = (int64_t)vy * nv + vx;
            // cells around (vx, vy): e(cx, cy) at s_eps[cy - y0 + 2][cx - x0 + 2]
            // base + surplus in FP64, rounded once to FP32 (the store's decode, bit for bit)
            const double e10 = s_eps[ly][lx + 1];                                 // (vx, vy-1)
            const double e01 = s_eps[ly + 1][lx], e11 = s_eps[ly + 1][lx + 1];  // (vx-1, vy), (vx, vy)
            const double k6 = -1.0 / 6.0, k3 = -1.0 / 3.0;
            const double base[4] = {(e10 + e11) * k6, e01 * k3, (e01 + e11) * k6, e11 * k3};
            int64_t t = v >> 6;
            int tt = a.sv.tier[t];
            if (tt == 0) {
                for (int j = 0; j < 4; ++j) c[j] = (TC)(float)base[j];  // rounded as the decoded operator
            } else {
                const uint8_t *bp = a.sv.payload + (size_t)a.sv.off[t] * 64;
                int l = (int)(v & 63);
                float sc = e8m0_to_float(bp[l]);
                for (int j = 0; j < 4; ++j) {
                    float d;
                    if (tt == 2) d = (float)__builtin_bit_cast(_Float16, ((const uint16_t *)(bp + 64 + j * 128))[l]) * sc;
                    else if (tt == 1) d = e4m3_to_float(bp[64 + j * 64 + l]) * sc;
                    else d = ((const float *)(bp + 64 + j * 256))[l];
                    c[j] = (TC)(float)(base[j] + (double)d);
                }
            }
        }
        for (int j = 0; j < 4; ++j) s_c[j][ly][lx] = c[j];
    }
    __syncthreads();
    const int tx = tid & 63, ty = tid >> 6;
    const int vx = x0 + tx, vy = y0 + ty;
    if (vx < nv && vy < nv) {
        int64_t v = (int64_t)vy * nv + vx;
        const int cx = tx + 1, cy = ty + 1;  // this vertex in s_c / s_u coordinates
        bool inner = vx > 0 && vx < n && vy > 0 && vy < n;
        // own upper couplings: (1,0), (-1,1), (0,1), (1,1); low-side ones from
        // the neighbours' slots: (-1,0) slot 0 of (x-1,y), (1,-1) slot 1 of
        // (x+1,y-1), (0,-1) slot 2 of (x,y-1), (-1,-1) slot 3 of (x-1,y-1)
        TC a0 = s_c[0][cy][cx], a1 = s_c[1][cy][cx], a2 = s_c[2][cy][cx], a3 = s_c[3][cy][cx];
        TC b0 = s_c[0][cy][cx - 1], b1 = s_c[1][cy - 1][cx + 1], b2 = s_c[2][cy - 1][cx], b3 = s_c[3][cy - 1][cx - 1];
        TC dsum = ((a0 + a1) + (a2 + a3)) + ((b0 + b1) + (b2 + b3));
        TC Dv = -dsum;
        TC uc = s_u[cy][cx];
        TC acc = a0 * s_u[cy][cx + 1] + a1 * s_u[cy + 1][cx - 1] + a2 * s_u[cy + 1][cx] + a3 * s_u[cy + 1][cx + 1] +
                 b0 * s_u[cy][cx - 1] + b1 * s_u[cy - 1][cx + 1] + b2 * s_u[cy - 1][cx] + b3 * s_u[cy - 1][cx - 1];
        TC Au = Dv * uc + acc;
        if (KIND == ST_SWEEP || KIND == ST_SWEEP0) {
            const float *f = (const float *)a.f;
            float *o = (float *)a.out;
            o[v] = inner ? (float)(uc + (TC)a.omega * ((TC)f[v] - Au) / Dv) : 0.0f;
        } else if (KIND == ST_RESID) {
            ((float *)a.out)[v] = inner ? (float)((TC)((const float *)a.f)[v] - Au) : 0.0f;
        } else if (KIND == ST_OUTER) {
            double r = inner ? (double)((TC)((const double *)a.f)[v] - Au) : 0.0;
            ((double *)a.out)[v] = r;
            if (a.rf) a.rf[v] = (float)r;
            part += r * r;
        } else {  // PMATVEC
            a.pnew[v] = (double)uc;
            double ap = inner ? (double)Au : 0.0;
            ((double *)a.out)[v] = ap;
            part += (double)uc * ap;
        }
    }
    __syncthreads();  // the next tile overwrites the staged data
    }
    if (KIND == ST_OUTER || KIND == ST_PMATVEC) {
        double sum = block_sum<256>(part, red);
        if (tid == 0) a.partial[blockIdx.x] = sum;
    }
}

// 64 x 4 tiles; the reducing modes run persistent blocks (at most kRedBlocks)
static inline void stage2_tiles(int n, int &ntx, int &nt)
{
    ntx = (n + 1 + 63) / 64;
    nt = ntx * ((n + 1 + 3) / 4);
}

// ------------------------------------------------------------ dispatch
int store_set_base(mgd_hier *h, OpSet &o, const float *eps_c, hipStream_t st);
StoreView store_view(const mgd_hier *h, const OpSet &o);

// the 3D mixed finest level decodes the compressed store per vertex only when
// asked to (MGD_STORE_DECODE): the per-vertex decode re-evaluates 26
// couplings in FP64 for every vertex of every pass and looks up the tiles of
// its mirrored couplings one by one.  MGD_STORE_COPY reads the FP32 decode;
// by default (MGD_STORE_AUTO) the sweeps and residuals re-evaluate only
// items whose sources are all tier 0, sharing the work across the item
// (k_sweep3x4h).  Same values, same results bit for bit
static bool store3_decode(const mgd_hier *h)
{
    if (h->dim != 3 || h->precision != MGD_MIXED) return false;
    return h->store_path == MGD_STORE_DECODE;
}

// the tier-0 item mask of the finest level, rebuilt after every change of
// the operator (one pass over the tile tiers)
static void ensure_imask(mgd_hier *h, const OpSet &o, hipStream_t st)
{
    if (o.dz_ok & kImaskOk) return;
    const int n = h->n;
    const int64_t items = (int64_t)(n / 4) * (n + 1) * (n + 1);
    hipLaunchKernelGGL(k_item_mask, dim3(grid_for(items, 256)), dim3(256), 0, st, o.tier, n, o.imask);
    o.dz_ok |= kImaskOk;
}

// items of the finest level and those the default 3D sweep re-evaluates
// from the centre samples (synchronous; 0 and 0 where that path is absent)
int item_mask_count(mgd_hier *h, int64_t *items, int64_t *tier0, hipStream_t st)
{
    *items = 0;
    *tier0 = 0;
    if (h->dim != 3 || h->precision != MGD_MIXED || !h->ops.imask) return MGD_OK;
    const int n = h->n;
    const int64_t cnt = (int64_t)(n / 4) * (n + 1) * (n + 1);
    ensure_imask(h, h->ops, st);
    HIPCHK(h->ctx, hipGetLastError());
    std::vector<uint8_t> m((size_t)cnt);
    HIPCHK(h->ctx, hipStreamSynchronize(st));
    HIPCHK(h->ctx, hipMemcpy(m.data(), h->ops.imask, (size_t)cnt, hipMemcpyDeviceToHost));
    int64_t c = 0;
    for (uint8_t b : m) c += b != 0;
    *items = cnt;
    *tier0 = c;
    return MGD_OK;
}

template <int D, typename T>
static int sweep_t(mgd_hier *h, const OpSet &o, int level, const T *u, const T *f, T *out, double omega, int mode,
                   bool zero_guess, double *partial, hipStream_t st)
{
    int n = h->nl[level];
    dim3 gr(grid_for(h->NV[level], 256));
    if (D == 2 && h->precision == MGD_MIXED && level == 0) {
        StageArgs<float> sa;
        memset(&sa, 0, sizeof(sa));
        sa.sv = store_view(h, o);
        sa.n = n;
        sa.u = u;
        sa.f = f;
        sa.out = out;
        sa.omega = (float)omega;
        stage2_tiles(n, sa.ntx, sa.nt);
        dim3 g2((unsigned)sa.nt);
        if (mode == 1) hipLaunchKernelGGL((k_stage2<float, ST_RESID>), g2, dim3(256), 0, st, sa);
        else if (zero_guess) hipLaunchKernelGGL((k_stage2<float, ST_SWEEP0>), g2, dim3(256), 0, st, sa);
        else hipLaunchKernelGGL((k_stage2<float, ST_SWEEP>), g2, dim3(256), 0, st, sa);
        HIPCHK(h->ctx, hipGetLastError());
        return MGD_OK;
    }
    if (D == 3 && h->precision == MGD_MIXED && level == 0 && store3_decode(h) && !partial) {
        // the mixed finest level streamed from HBM: decode the store per vertex
        const StoreView sv = store_view(h, o);
        const float *uf = (const float *)u, *ff = (const float *)f;
        float *of = (float *)out;
        if (mode == 1) hipLaunchKernelGGL((k_sweep3_store<1, false>), gr, dim3(256), 0, st, sv, n, uf, ff, of, (float)omega);
        else if (zero_guess) hipLaunchKernelGGL((k_sweep3_store<0, true>), gr, dim3(256), 0, st, sv, n, uf, ff, of, (float)omega);
        else hipLaunchKernelGGL((k_sweep3_store<0, false>), gr, dim3(256), 0, st, sv, n, uf, ff, of, (float)omega);
        HIPCHK(h->ctx, hipGetLastError());
        return MGD_OK;
    }
    if (D == 3 && h->precision == MGD_MIXED && level == 0 && h->store_path == MGD_STORE_AUTO && o.imask &&
        !zero_guess && !partial) {
        // the default: tier-0 sources re-evaluated from eps_c, the rest read
        // from the FP32 decode
        ensure_imask(h, o, st);
        const dim3 g4(items4_blocks(n));
        const float *uf = (const float *)u, *ff = (const float *)f;
        float *of = (float *)out;
        const double hp = 1.0 / (double)n;
        if (mode == 1)
            hipLaunchKernelGGL((k_sweep3x4h<1>), g4, dim3(256), 0, st, o.S32[0], o.imask, o.eps_c, n, hp, uf, ff, of,
                               (float)omega);
        else
            hipLaunchKernelGGL((k_sweep3x4h<0>), g4, dim3(256), 0, st, o.S32[0], o.imask, o.eps_c, n, hp, uf, ff, of,
                               (float)omega);
        HIPCHK(h->ctx, hipGetLastError());
        return MGD_OK;
    }
    if (items4_fit(D, n) && !partial) {
        const T *S = h->precision == MGD_FP64 ? (const T *)o.S64[level] : (const T *)o.S32[level];
        const dim3 g4(items4_blocks(n));
        if (mode == 1) hipLaunchKernelGGL((k_sweep3x4<T, 1, false>), g4, dim3(256), 0, st, S, n, u, f, out, (T)omega);
        else if (zero_guess) hipLaunchKernelGGL((k_sweep3x4<T, 0, true>), g4, dim3(256), 0, st, S, n, u, f, out, (T)omega);
        else hipLaunchKernelGGL((k_sweep3x4<T, 0, false>), g4, dim3(256), 0, st, S, n, u, f, out, (T)omega);
        HIPCHK(h->ctx, hipGetLastError());
        return MGD_OK;
    }
    auto go = [&](auto A) {
        using OpT = decltype(A);
        if (mode == 1)
            hipLaunchKernelGGL((k_sweep<D, OpT, T, 1, false>), gr, dim3(256), 0, st, A, n, u, f, out, (T)omega, partial);
        else if (zero_guess)
            hipLaunchKernelGGL((k_sweep<D, OpT, T, 0, true>), gr, dim3(256), 0, st, A, n, u, f, out, (T)omega, partial);
        else
            hipLaunchKernelGGL((k_sweep<D, OpT, T, 0, false>), gr, dim3(256), 0, st, A, n, u, f, out, (T)omega, partial);
        return MGD_OK;
    };
    if (h->precision == MGD_FP64) go(OpHalf<double>{o.S64[level], h->NV[level]});
    else go(OpHalf<float>{o.S32[level], h->NV[level]});  // level 0: the store's FP32 decode
    HIPCHK(h->ctx, hipGetLastError());
    return MGD_OK;
}

static int sweep(mgd_hier *h, const OpSet &o, int level, const void *u, const void *f, void *out, double omega,
                 int mode, bool zero_guess, double *partial, hipStream_t st)
{
    if (h->precision == MGD_FP64) {
        if (h->dim == 2) return sweep_t<2, double>(h, o, level, (const double *)u, (const double *)f, (double *)out, omega, mode, zero_guess, partial, st);
        return sweep_t<3, double>(h, o, level, (const double *)u, (const double *)f, (double *)out, omega, mode, zero_guess, partial, st);
    }
    if (h->dim == 2) return sweep_t<2, float>(h, o, level, (const float *)u, (const float *)f, (float *)out, omega, mode, zero_guess, partial, st);
    return sweep_t<3, float>(h, o, level, (const float *)u, (const float *)f, (float *)out, omega, mode, zero_guess, partial, st);
}

// ---- the 3D zero-start sweep from the stored diagonal.  From u = 0 a
// damped-Jacobi sweep is u_1 = omega f / D: only the diagonal of the
// operator enters, so with D kept per level (Dz, computed once per operator
// by k_diag_zero with the zero-start sweep's own sum order) the pass reads
// 8 bytes per vertex instead of the whole stencil.  Same values as the
// stencil kernels' zero-start mode, bit for bit.
template <typename T> __global__ __launch_bounds__(256) void k_diag_zero(const T *__restrict__ S, int n, T *__restrict__ Dz)
{
    Grid<3> g(n);
    const int64_t v = block_index<3>() * blockDim.x + threadIdx.x;
    if (v >= g.NV) return;
    int x[3];
    g.coords(v, x);
    T d = (T)1;
    if (g.interior(x)) {
        T dsum = (T)0;
        for (int j = 0; j < 13; ++j) {
            const int64_t lin = half_lin(3, j, g.nv);
            dsum += S[(int64_t)j * g.NV + v] + S[(int64_t)j * g.NV + v - lin];
        }
        d = -dsum;
    }
    Dz[v] = d;
}

template <typename T>
__global__ __launch_bounds__(256) void k_zero_sweep_d(const T *__restrict__ Dz, int n, const T *__restrict__ f,
                                                     T *__restrict__ out, T omega)
{
    Grid<3> g(n);
    const int64_t v = block_index<3>() * blockDim.x + threadIdx.x;
    if (v >= g.NV) return;
    int x[3];
    g.coords(v, x);
    out[v] = g.interior(x) ? (T)0 + omega * (f[v] - (T)0) / Dz[v] : (T)0;
}

template <typename T>
static int zero_sweep_t(mgd_hier *h, const OpSet &o, int level, const T *f, T *out, double omega, hipStream_t st)
{
    const int n = h->nl[level];
    const dim3 gr(grid_for(h->NV[level], 256));
    T *Dz = (T *)o.Dz[level];
    if (!(o.dz_ok >> level & 1u)) {
        const T *S = h->precision == MGD_FP64 ? (const T *)o.S64[level] : (const T *)o.S32[level];
        hipLaunchKernelGGL((k_diag_zero<T>), gr, dim3(256), 0, st, S, n, Dz);
        HIPCHK(h->ctx, hipGetLastError());
        o.dz_ok |= 1u << level;
    }
    hipLaunchKernelGGL((k_zero_sweep_d<T>), gr, dim3(256), 0, st, Dz, n, f, out, (T)omega);
    HIPCHK(h->ctx, hipGetLastError());
    return MGD_OK;
}

// the 3D zero-start sweep takes the stored diagonal except on the
// store-decoding finest level (whose kernels read the store only)
static bool zero_sweep_by_diag(const mgd_hier *h, const OpSet &o, int level)
{
    return h->dim == 3 && o.Dz[level] && !(h->precision == MGD_MIXED && level == 0 && store3_decode(h));
}

int cycle_smooth(mgd_hier *h, const OpSet &o, int level, void *u, const void *f, void *tmp, int sweeps,
                 double omega, bool zero_guess, hipStream_t st)
{
    // ping-pong u -> tmp -> u; an odd count ends with a copy back
    for (int k = 0; k < sweeps; ++k) {
        const void *src = (k % 2 == 0) ? u : tmp;
        void *dst = (k % 2 == 0) ? tmp : u;
        int rc;
        if (zero_guess && k == 0 && zero_sweep_by_diag(h, o, level))
            rc = h->precision == MGD_FP64
                     ? zero_sweep_t<double>(h, o, level, (const double *)f, (double *)dst, omega, st)
                     : zero_sweep_t<float>(h, o, level, (const float *)f, (float *)dst, omega, st);
        else
            rc = sweep(h, o, level, src, f, dst, omega, 0, zero_guess && k == 0, nullptr, st);
        if (rc) return rc;
    }
    if (sweeps % 2 == 1)
        HIPCHK(h->ctx, hipMemcpyAsync(u, tmp, h->NV[level] * h->vec_bytes(), hipMemcpyDeviceToDevice, st));
    return MGD_OK;
}

int cycle_residual(mgd_hier *h, const OpSet &o, int level, const void *u, const void *f, void *r, hipStream_t st)
{
    return sweep(h, o, level, u, f, r, 0.0, 1, false, nullptr, st);
}

int cycle_restrict(mgd_hier *h, const OpSet &o, int level, const void *r, void *fc, hipStream_t st)
{
    int nf = h->nl[level];
    dim3 gr(grid_for(h->NV[level + 1], 256));
    bool box = h->transfer == MGD_BOXMG;
    if (h->precision == MGD_FP64) {
        const double *W = box ? (const double *)o.W[level] : nullptr;
        if (h->dim == 2 && W) hipLaunchKernelGGL((k_restrict2<double, false>), gr, dim3(256), 0, st, W, nf, (const double *)r, (double *)fc);
        else if (h->dim == 2) hipLaunchKernelGGL((k_restrict2<double, true>), gr, dim3(256), 0, st, W, nf, (const double *)r, (double *)fc);
        else if (W) hipLaunchKernelGGL((k_restrict3<double, false>), gr, dim3(256), 0, st, W, o.wgeo[level], nf, (const double *)r, (double *)fc);
        else hipLaunchKernelGGL((k_restrict3<double, true>), gr, dim3(256), 0, st, W, nullptr, nf, (const double *)r, (double *)fc);
    } else {
        const float *W = box ? (const float *)o.W[level] : nullptr;
        if (h->dim == 2 && W) hipLaunchKernelGGL((k_restrict2<float, false>), gr, dim3(256), 0, st, W, nf, (const float *)r, (float *)fc);
        else if (h->dim == 2) hipLaunchKernelGGL((k_restrict2<float, true>), gr, dim3(256), 0, st, W, nf, (const float *)r, (float *)fc);
        else if (W) hipLaunchKernelGGL((k_restrict3<float, false>), gr, dim3(256), 0, st, W, o.wgeo[level], nf, (const float *)r, (float *)fc);
        else hipLaunchKernelGGL((k_restrict3<float, true>), gr, dim3(256), 0, st, W, nullptr, nf, (const float *)r, (float *)fc);
    }
    HIPCHK(h->ctx, hipGetLastError());
    return MGD_OK;
}

int cycle_prolong(mgd_hier *h, const OpSet &o, int level, const void *ec, void *u, hipStream_t st)
{
    int nf = h->nl[level];
    dim3 gr(grid_for(h->NV[level], 256)), gc3(grid_for(h->NV[level + 1], 256));
    bool box = h->transfer == MGD_BOXMG;
    if (h->precision == MGD_FP64) {
        const double *W = box ? (const double *)o.W[level] : nullptr;
        if (h->dim == 2) hipLaunchKernelGGL((k_prolong<2, double>), gr, dim3(256), 0, st, W, nf, (const double *)ec, (double *)u);
        else if (W) hipLaunchKernelGGL((k_prolong3<double, false>), gc3, dim3(256), 0, st, W, o.wgeo[level], nf, (const double *)ec, (double *)u);
        else hipLaunchKernelGGL((k_prolong3<double, true>), gc3, dim3(256), 0, st, W, nullptr, nf, (const double *)ec, (double *)u);
    } else {
        const float *W = box ? (const float *)o.W[level] : nullptr;
        if (h->dim == 2) hipLaunchKernelGGL((k_prolong<2, float>), gr, dim3(256), 0, st, W, nf, (const float *)ec, (float *)u);
        else if (W) hipLaunchKernelGGL((k_prolong3<float, false>), gc3, dim3(256), 0, st, W, o.wgeo[level], nf, (const float *)ec, (float *)u);
        else hipLaunchKernelGGL((k_prolong3<float, true>), gc3, dim3(256), 0, st, W, nullptr, nf, (const float *)ec, (float *)u);
    }
    HIPCHK(h->ctx, hipGetLastError());
    return MGD_OK;
}

static int fill_zero(mgd_hier *h, void *a, int64_t n, hipStream_t st)
{
    if (h->precision == MGD_FP64) hipLaunchKernelGGL(k_fill<double>, dim3(grid_for(n, 256)), dim3(256), 0, st, (double *)a, n, 0.0);
    else hipLaunchKernelGGL(k_fill<float>, dim3(grid_for(n, 256)), dim3(256), 0, st, (float *)a, n, 0.0f);
    HIPCHK(h->ctx, hipGetLastError());
    return MGD_OK;
}

// ------------------------------------------------------------ coarse tail
// The small levels of the V-cycle, from level `first` (zero initial guess or
// a given u) down to the dense coarsest solve and back up, in one workgroup
// of 1024 threads.  The vectors of every tail level (iterate, right-hand
// side, scratch) live in LDS for the whole tail; stencils and transfer
// weights are read from memory (they stay in L2), each phase issuing all its
// loads before its LDS arithmetic.  Phases are separated by workgroup
// barriers.  The coarsest solve multiplies by the precomputed FP64 inverse
// (small coarse grids) or runs FP64 forward and backward substitution with
// the Cholesky factor.
constexpr int kTailThreads = 1024;
struct TailLevel {
    const void *S, *W;
    int n, NV;
    int off;    // element offset of this level's vectors in LDS: u | f | t
    float rnv;  // 1 / (n + 1)
};
// 2D: global arrays copied into LDS when the tail starts.  Each segment
// starts at a multiple of the block size in the flat item space, so a
// thread's k-th item belongs to segment seg_of[k] for every thread alike.
constexpr int kTailSegs = 2 * MGD_MAXLEV + 2, kTailStageK = 24;
struct TailSeg {
    const void *src;
    int dst, cnt;  // LDS element offset, items
};
struct TailArgs {
    int first, last, nu1, nu2, zero_guess, m, work_off;
    double omega;
    void *u;
    const void *f;
    const double *chol, *cinv;
    TailLevel L[MGD_MAXLEV];
    int nslot;                // 2D staging: item slots per thread in use
    int8_t seg_of[kTailStageK];  // segment of each slot
    int16_t seg_k0[kTailStageK]; // the segment's first slot
    TailSeg seg[kTailSegs];
};

// vertex coordinates by a float reciprocal (exact for the tail's sizes:
// v < 2^13, so the quotient's error is far below the 1/(2 nv) margin)
template <int D> __device__ inline void tail_coords(int v, const TailLevel &lv, int *x)
{
    const int nv = lv.n + 1;
    const int q = (int)(((float)v + 0.5f) * lv.rnv);
    x[0] = v - q * nv;
    if (D == 2) {
        x[1] = q;
    } else {
        const int q2 = (int)(((float)q + 0.5f) * lv.rnv);
        x[1] = q - q2 * nv;
        x[2] = q2;
    }
}
template <int D> __device__ inline bool tail_interior(const int *x, int n)
{
    for (int m = 0; m < D; ++m)
        if (x[m] == 0 || x[m] == n) return false;
    return true;
}

// one stencil pass: MODE 0 damped Jacobi sweep uout = u + omega D^-1 (f - A u)
// (ZERO: from u = 0), MODE 1 residual uout = f - A u.  CK vertices per
// thread have their stencil loads in flight together.
template <int D, typename T, int CK, int MODE>
__device__ void tail_pass(const TailLevel &lv, const T *S, const T *uin, T *uout, const T *f, bool zero, T omega)
{
    constexpr int H = n_half(D);
    const int nv = lv.n + 1, NV = lv.NV;
    const int safe = D == 2 ? 1 + nv : 1 + nv + nv * nv;  // an interior vertex
    int lin[H];
#pragma unroll
    for (int j = 0; j < H; ++j) lin[j] = half_off(D, j, 0) + half_off(D, j, 1) * nv + (D == 3 ? half_off(D, j, 2) * nv * nv : 0);
    for (int v0 = threadIdx.x; v0 < NV; v0 += CK * (int)blockDim.x) {
        T c[CK][2 * H];
        bool in[CK];
#pragma unroll
        for (int q = 0; q < CK; ++q) {
            const int v = v0 + q * (int)blockDim.x;
            int x[3] = {0, 0, 0};
            tail_coords<D>(v < NV ? v : 0, lv, x);
            in[q] = v < NV && tail_interior<D>(x, lv.n);
            const uint32_t vs = (uint32_t)(in[q] ? v : safe);
#pragma unroll
            for (int j = 0; j < H; ++j) {
                c[q][j] = S[(uint32_t)j * (uint32_t)NV + vs];
                c[q][H + j] = S[(uint32_t)j * (uint32_t)NV + vs - (uint32_t)lin[j]];
            }
        }
#pragma unroll
        for (int q = 0; q < CK; ++q) {
            const int v = v0 + q * (int)blockDim.x;
            if (v >= NV) continue;
            T out = (T)0;
            if (in[q]) {
                T acc = (T)0, dsum = (T)0;
#pragma unroll
                for (int j = 0; j < H; ++j) {
                    if (MODE == 1 || !zero) acc += c[q][j] * uin[v + lin[j]] + c[q][H + j] * uin[v - lin[j]];
                    dsum += c[q][j] + c[q][H + j];
                }
                const T Dv = -dsum;
                if (MODE == 1) out = f[v] - (Dv * uin[v] + acc);
                else out = zero ? omega * f[v] / Dv : uin[v] + omega * (f[v] - (Dv * uin[v] + acc)) / Dv;
            }
            uout[v] = out;
        }
    }
    __syncthreads();
}

template <int D, typename T, int MODE>
__device__ inline void tail_pass_any(const TailLevel &lv, const T *S, const T *uin, T *uout, const T *f, bool zero,
                                     T omega)
{
    // several vertices per thread in flight where registers allow (2D), else one
    constexpr int CK = D == 3 ? 1 : sizeof(T) == 8 ? 3 : 5;
    if (CK > 1 && lv.NV > (int)blockDim.x) tail_pass<D, T, CK, MODE>(lv, S, uin, uout, f, zero, omega);
    else tail_pass<D, T, 1, MODE>(lv, S, uin, uout, f, zero, omega);
}

template <int D, typename T>
__device__ void tail_smooth(const TailLevel &lv, const T *S, T *u, const T *f, T *t, int sweeps, bool zero, T omega)
{
    for (int k = 0; k < sweeps; ++k) {
        if (k % 2 == 0) tail_pass_any<D, T, 0>(lv, S, u, t, f, zero && k == 0, omega);
        else tail_pass_any<D, T, 0>(lv, S, t, u, f, false, omega);
    }
    if (sweeps % 2 == 1) {
        for (int v = threadIdx.x; v < lv.NV; v += (int)blockDim.x) u[v] = t[v];
        __syncthreads();
    }
    if (sweeps == 0 && zero) {
        for (int v = threadIdx.x; v < lv.NV; v += (int)blockDim.x) u[v] = (T)0;
        __syncthreads();
    }
}

// fc = P^T r on the interior coarse vertices, uc = 0
template <int D, typename T>
__device__ void tail_restrict(const TailLevel &lv, const TailLevel &lc, const T *W, const T *r, T *fc, T *uc)
{
    constexpr int ns = D == 2 ? 9 : 27;
    const int nv = lv.n + 1, NV = lv.NV;
    for (int V = threadIdx.x; V < lc.NV; V += (int)blockDim.x) {
        int X[3] = {0, 0, 0};
        tail_coords<D>(V, lc, X);
        uc[V] = (T)0;
        if (!tail_interior<D>(X, lc.n)) {
            fc[V] = (T)0;
            continue;
        }
        T w[ns];
        int vv[ns];
#pragma unroll
        for (int sv = 0; sv < ns; ++sv) {
            int t = sv, B = 0, v = 0, st = 1;
            bool geo_full = true;
            for (int m = 0; m < D; ++m) {
                const int o = t % 3 - 1;
                t /= 3;
                v += (2 * X[m] + o) * st;
                st *= nv;
                B |= (o < 0 ? 1 : 0) << m;  // X - (x >> 1) is 1 exactly when o = -1
                if (o != 0) geo_full = false;
            }
            vv[sv] = v;
            if (W) {
                w[sv] = W[(uint32_t)B * (uint32_t)NV + (uint32_t)v];
            } else {
                double p = 1.0;
                int tt = sv;
                for (int m = 0; m < D; ++m) { p *= (tt % 3 == 1) ? 1.0 : 0.5; tt /= 3; }
                (void)geo_full;
                w[sv] = (T)p;
            }
        }
        T s = (T)0;
#pragma unroll
        for (int sv = 0; sv < ns; ++sv) s += w[sv] * r[vv[sv]];
        fc[V] = s;
    }
    __syncthreads();
}

// u += P ec on the interior fine vertices
template <int D, typename T>
__device__ void tail_prolong(const TailLevel &lv, const TailLevel &lc, const T *W, T *u, const T *ec)
{
    constexpr int nl = 1 << D;
    const int ncv = lc.n + 1;
    for (int v = threadIdx.x; v < lv.NV; v += (int)blockDim.x) {
        int x[3] = {0, 0, 0};
        tail_coords<D>(v, lv, x);
        if (!tail_interior<D>(x, lv.n)) continue;
        T w[nl];
        int ic[nl];
#pragma unroll
        for (int B = 0; B < nl; ++B) {
            bool use = true;
            int c = 0, st = 1;
            double p = 1.0;
            for (int m = 0; m < D; ++m) {
                const int b = (B >> m) & 1;
                if (b && !(x[m] & 1)) use = false;  // only odd axes reach the upper corner
                c += ((x[m] >> 1) + b) * st;
                st *= ncv;
                p *= (x[m] & 1) ? 0.5 : 1.0;
            }
            ic[B] = use ? c : 0;
            w[B] = use ? (W ? W[(uint32_t)B * (uint32_t)lv.NV + (uint32_t)v] : (T)p) : (T)0;
        }
        T s = (T)0;
#pragma unroll
        for (int B = 0; B < nl; ++B)
            if (w[B] != (T)0) s += w[B] * ec[ic[B]];
        u[v] += s;
    }
    __syncthreads();
}

// dense FP64 solve on the interior of the coarsest level: u = A^{-1} f
template <int D, typename T>
__device__ void tail_coarse(const TailArgs &a, const TailLevel &lv, T *u, const T *f, double *work)
{
    const int m = a.m, nin = lv.n - 1, nv = lv.n + 1;
    auto vof = [&](int k) {  // interior index -> vertex
        int v = 0, st = 1, t = k;
        for (int mm = 0; mm < D; ++mm) { v += (1 + t % nin) * st; t /= nin; st *= nv; }
        return v;
    };
    for (int k = threadIdx.x; k < m; k += (int)blockDim.x) work[k] = (double)f[vof(k)];
    for (int v = threadIdx.x; v < lv.NV; v += (int)blockDim.x) u[v] = (T)0;
    __syncthreads();
    if (a.cinv) {
        for (int i = threadIdx.x; i < m; i += (int)blockDim.x) {
            double s = 0.0;
            for (int k = 0; k < m; ++k) s += a.cinv[(int64_t)i * m + k] * work[k];
            u[vof(i)] = (T)s;
        }
        __syncthreads();
        return;
    }
    const double *L = a.chol;
    // forward: L y = b, column by column
    for (int i = 0; i < m; ++i) {
        const double yi = work[i] / L[(int64_t)i * m + i];
        __syncthreads();
        if (threadIdx.x == 0) work[i] = yi;
        for (int k = i + 1 + threadIdx.x; k < m; k += (int)blockDim.x) work[k] -= L[(int64_t)k * m + i] * yi;
        __syncthreads();
    }
    // backward: L^T x = y, row i needs x_k for k > i
    for (int i = m - 1; i >= 0; --i) {
        const double xi = work[i] / L[(int64_t)i * m + i];
        __syncthreads();
        if (threadIdx.x == 0) work[i] = xi;
        for (int k = threadIdx.x; k < i; k += (int)blockDim.x) work[k] -= L[(int64_t)i * m + k] * xi;
        __syncthreads();
    }
    for (int k = threadIdx.x; k < m; k += (int)blockDim.x) u[vof(k)] = (T)work[k];
    __syncthreads();
}

template <int D, typename T> __global__ __launch_bounds__(1024) void k_tail(TailArgs a)
{
    extern __shared__ __align__(16) unsigned char tail_lds[];
    T *base = (T *)tail_lds;
    double *work = (double *)(tail_lds + a.work_off);
    const T omega = (T)a.omega;
    auto U = [&](int l) { return base + a.L[l].off; };
    auto F = [&](int l) { return base + a.L[l].off + a.L[l].NV; };
    auto Tt = [&](int l) { return base + a.L[l].off + 2 * a.L[l].NV; };
    // stencils and weights are read from memory (L2): a phase is bound by its
    // barrier-to-barrier dependency chain, and staging them in LDS as well
    // was measured slower
    auto Sp = [&](int l) { return (const T *)a.L[l].S; };
    auto Wp = [&](int l) { return (const T *)a.L[l].W; };
    {
        const TailLevel &l0 = a.L[a.first];
        const T *fg = (const T *)a.f, *ug = (const T *)a.u;
        T *u0 = U(a.first), *f0 = F(a.first);
        for (int v = threadIdx.x; v < l0.NV; v += (int)blockDim.x) {
            f0[v] = fg[v];
            u0[v] = a.zero_guess ? (T)0 : ug[v];
        }
        __syncthreads();
    }
    for (int l = a.first; l < a.last; ++l) {
        const bool zero = l > a.first || a.zero_guess;
        tail_smooth<D, T>(a.L[l], Sp(l), U(l), F(l), Tt(l), a.nu1, zero, omega);
        tail_pass_any<D, T, 1>(a.L[l], Sp(l), U(l), Tt(l), F(l), false, omega);
        tail_restrict<D, T>(a.L[l], a.L[l + 1], Wp(l), Tt(l), F(l + 1), U(l + 1));
    }
    tail_coarse<D, T>(a, a.L[a.last], U(a.last), F(a.last), work);
    for (int l = a.last - 1; l >= a.first; --l) {
        tail_prolong<D, T>(a.L[l], a.L[l + 1], Wp(l), U(l), U(l + 1));
        tail_smooth<D, T>(a.L[l], Sp(l), U(l), F(l), Tt(l), a.nu2, false, omega);
    }
    {
        T *ug = (T *)a.u;
        const T *u0 = U(a.first);
        for (int v = threadIdx.x; v < a.L[a.first].NV; v += (int)blockDim.x) ug[v] = u0[v];
    }
}

// ---- 2D tail with the operators in LDS.  Every tail level's half stencils
// and transfer weights are copied into LDS once per call (all loads of a
// thread in flight together), with the first level's right-hand side and
// iterate; from then on every phase reads and writes LDS only.  Level
// layout (element offsets from L[l].off): u | f | t | S [4][NV] | W [4][NV].
__device__ inline void t2_coords(int v, const TailLevel &lv, int &x, int &y)
{
    const int nv = lv.n + 1;
    y = (int)(((float)v + 0.5f) * lv.rnv);
    x = v - y * nv;
}

// stencil application at interior vertex v: acc = sum of the 8 couplings
// times the neighbours' iterate, dsum = sum of the 8 couplings
template <typename T>
__device__ inline void t2_apply(const T *S, int NV, int nv, const T *u, int v, T &acc, T &dsum, bool need_acc)
{
    const int lin[4] = {1, nv - 1, nv, nv + 1};
    const T a0 = S[v], a1 = S[NV + v], a2 = S[2 * NV + v], a3 = S[3 * NV + v];
    const T b0 = S[v - lin[0]], b1 = S[NV + v - lin[1]], b2 = S[2 * NV + v - lin[2]], b3 = S[3 * NV + v - lin[3]];
    dsum = ((a0 + a1) + (a2 + a3)) + ((b0 + b1) + (b2 + b3));
    acc = (T)0;
    if (need_acc)
        acc = a0 * u[v + lin[0]] + a1 * u[v + lin[1]] + a2 * u[v + lin[2]] + a3 * u[v + lin[3]] + b0 * u[v - lin[0]] +
              b1 * u[v - lin[1]] + b2 * u[v - lin[2]] + b3 * u[v - lin[3]];
}

// MODE 0: damped Jacobi sweep uout = (1 - omega) u + (omega / D) (f - offdiag u)
// (ZERO: from u = 0); MODE 1: residual uout = f - A u
template <typename T, int MODE>
__device__ void t2_pass(const TailLevel &lv, T *base, const T *uin, T *uout, bool zero, T omega)
{
    const int nv = lv.n + 1, NV = lv.NV;
    const T *f = base + lv.off + NV, *S = base + lv.off + 3 * NV;
    for (int v = threadIdx.x; v < NV; v += kTailThreads) {
        int x, y;
        t2_coords(v, lv, x, y);
        T out = (T)0;
        if (x > 0 && x < lv.n && y > 0 && y < lv.n) {
            T acc, dsum;
            t2_apply(S, NV, nv, uin, v, acc, dsum, MODE == 1 || !zero);
            if (MODE == 1) out = f[v] - (-dsum * uin[v] + acc);
            else if (zero) out = (omega / -dsum) * f[v];
            else out = ((T)1 - omega) * uin[v] + (omega / -dsum) * (f[v] - acc);
        }
        uout[v] = out;
    }
    __syncthreads();
}

template <typename T> __global__ __launch_bounds__(1024) void k_tail2d(TailArgs a)
{
    extern __shared__ __align__(16) unsigned char tail_lds[];
    T *base = (T *)tail_lds;
    double *work = (double *)(tail_lds + a.work_off);
    const T omega = (T)a.omega;
    const int tid = threadIdx.x;
    // ---- staging: slot k of every thread lies in segment seg_of[k] (uniform),
    // all loads issued before the LDS stores
    {
        T val[kTailStageK];
        int dst[kTailStageK];
#pragma unroll
        for (int k = 0; k < kTailStageK; ++k) {
            dst[k] = -1;
            val[k] = (T)0;
            if (k < a.nslot) {
                const TailSeg &sg = a.seg[a.seg_of[k]];
                const int i = tid + (k - a.seg_k0[k]) * kTailThreads;
                if (i < sg.cnt) {
                    val[k] = ((const T *)sg.src)[i];
                    dst[k] = sg.dst + i;
                }
            }
        }
#pragma unroll
        for (int k = 0; k < kTailStageK; ++k)
            if (dst[k] >= 0) base[dst[k]] = val[k];
        if (a.zero_guess) {
            const TailLevel &l0 = a.L[a.first];
            for (int v = tid; v < l0.NV; v += kTailThreads) base[l0.off + v] = (T)0;
        }
        __syncthreads();
    }
    auto U = [&](int l) { return base + a.L[l].off; };
    auto F = [&](int l) { return base + a.L[l].off + a.L[l].NV; };
    auto Tt = [&](int l) { return base + a.L[l].off + 2 * a.L[l].NV; };
    auto Wl = [&](int l) { return a.L[l].W ? base + a.L[l].off + 7 * a.L[l].NV : nullptr; };
    auto smooth = [&](int l, int sweeps, bool zero) {
        for (int k = 0; k < sweeps; ++k) {
            if (k % 2 == 0) t2_pass<T, 0>(a.L[l], base, U(l), Tt(l), zero && k == 0, omega);
            else t2_pass<T, 0>(a.L[l], base, Tt(l), U(l), false, omega);
        }
        if (sweeps % 2 == 1) {
            for (int v = tid; v < a.L[l].NV; v += kTailThreads) U(l)[v] = Tt(l)[v];
            __syncthreads();
        }
        if (sweeps == 0 && zero) {
            for (int v = tid; v < a.L[l].NV; v += kTailThreads) U(l)[v] = (T)0;
            __syncthreads();
        }
    };
    for (int l = a.first; l < a.last; ++l) {
        const TailLevel &lv = a.L[l], &lc = a.L[l + 1];
        smooth(l, a.nu1, l > a.first || a.zero_guess);
        t2_pass<T, 1>(lv, base, U(l), Tt(l), false, omega);
        // fc = P^T r on the interior coarse vertices, uc = 0
        const T *r = Tt(l), *W = Wl(l);
        const int nv = lv.n + 1;
        T *fc = F(l + 1), *uc = U(l + 1);
        for (int V = tid; V < lc.NV; V += kTailThreads) {
            int X, Y;
            t2_coords(V, lc, X, Y);
            T s = (T)0;
            if (X > 0 && X < lc.n && Y > 0 && Y < lc.n) {
#pragma unroll
                for (int sv = 0; sv < 9; ++sv) {
                    const int ox = sv % 3 - 1, oy = sv / 3 - 1;
                    const int B = (ox < 0 ? 1 : 0) | (oy < 0 ? 2 : 0);  // X - (x >> 1) is 1 exactly where o = -1
                    const int v = (2 * Y + oy) * nv + 2 * X + ox;
                    const T w = W ? W[B * lv.NV + v] : (T)((ox ? 0.5 : 1.0) * (oy ? 0.5 : 1.0));
                    s += w * r[v];
                }
            }
            fc[V] = s;
            uc[V] = (T)0;
        }
        __syncthreads();
    }
    tail_coarse<2, T>(a, a.L[a.last], U(a.last), F(a.last), work);
    for (int l = a.last - 1; l >= a.first; --l) {
        // u += P ec on the interior fine vertices
        const TailLevel &lv = a.L[l], &lc = a.L[l + 1];
        const T *W = Wl(l), *ec = U(l + 1);
        T *u = U(l);
        const int ncv = lc.n + 1;
        for (int v = tid; v < lv.NV; v += kTailThreads) {
            int x, y;
            t2_coords(v, lv, x, y);
            if (!(x > 0 && x < lv.n && y > 0 && y < lv.n)) continue;
            T s = (T)0;
#pragma unroll
            for (int B = 0; B < 4; ++B) {
                const int bx = B & 1, by = B >> 1;
                if ((bx && !(x & 1)) || (by && !(y & 1))) continue;  // only odd axes reach the upper corner
                const T w = W ? W[B * lv.NV + v] : (T)(((x & 1) ? 0.5 : 1.0) * ((y & 1) ? 0.5 : 1.0));
                if (w != (T)0) s += w * ec[((y >> 1) + by) * ncv + (x >> 1) + bx];
            }
            u[v] += s;
        }
        __syncthreads();
        smooth(l, a.nu2, false);
    }
    {
        T *ug = (T *)a.u;
        const T *u0 = U(a.first);
        for (int v = tid; v < a.L[a.first].NV; v += kTailThreads) ug[v] = u0[v];
    }
}

// first level handled by the single-workgroup tail: in 2D the levels up to
// 33 x 33 vertices (larger ones run faster as fused multi-block passes), in
// 3D up to 9^3 (17^3 runs as multi-block passes: a single workgroup large
// enough for it waits long for a free CU while assembly runs beside the
// cycles)
static int tail_first(const mgd_hier *h)
{
    const int64_t kTailNV = h->dim == 2 ? 1100 : 800;
    int l = h->nlev - 1;
    while (l > 0 && h->NV[l - 1] <= kTailNV) --l;
    if (h->precision == MGD_MIXED && l == 0) l = h->nlev > 1 ? 1 : 0;  // level 0 is the compressed store
    return l;
}

template <typename T> static void tail2d_launch_t(const TailArgs &a, size_t lds, hipStream_t st)
{
    static bool attr = false;  // once per instantiation: allow more than 64 KB of dynamic LDS
    if (!attr) {
        (void)hipFuncSetAttribute((const void *)k_tail2d<T>, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        attr = true;
    }
    hipLaunchKernelGGL((k_tail2d<T>), dim3(1), dim3(kTailThreads), lds, st, a);
}

template <int D, typename T> static void tail_launch_t(const TailArgs &a, size_t lds, hipStream_t st)
{
    static bool attr = false;  // once per instantiation: allow more than 64 KB of dynamic LDS
    if (!attr) {
        (void)hipFuncSetAttribute((const void *)k_tail<D, T>, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        attr = true;
    }
    // 3D tails hold only small levels: one quarter of the threads, so the
    // workgroup finds room beside a concurrent assembly kernel
    hipLaunchKernelGGL((k_tail<D, T>), dim3(1), dim3(D == 3 ? kTailThreads / 4 : kTailThreads), lds, st, a);
}

static int launch_tail(mgd_hier *h, const OpSet &o, int first, void *u, const void *f, double omega, int nu1, int nu2,
                       bool zero_guess, hipStream_t st)
{
    TailArgs a;
    memset(&a, 0, sizeof(a));
    a.first = first;
    a.last = h->nlev - 1;
    a.nu1 = nu1;
    a.nu2 = nu2;
    a.zero_guess = zero_guess ? 1 : 0;
    a.omega = omega;
    a.u = u;
    a.f = f;
    a.chol = o.chol;
    a.cinv = o.cinv;
    a.m = (int)h->m_coarse;
    const size_t vb = h->vec_bytes(), cap = 160 * 1024;
    if (h->dim == 2) {
        // operators, weights and the first level's vectors staged in LDS
        int64_t off = 0;
        int ns = 0, nslot = 0;
        bool fits = true;
        auto seg = [&](const void *src, int64_t dst, int64_t cnt) {
            const int k = (int)((cnt + kTailThreads - 1) / kTailThreads);
            if (nslot + k > kTailStageK) {
                fits = false;
                return;
            }
            a.seg[ns].src = src;
            a.seg[ns].dst = (int)dst;
            a.seg[ns].cnt = (int)cnt;
            for (int q = 0; q < k; ++q) {
                a.seg_of[nslot + q] = (int8_t)ns;
                a.seg_k0[nslot + q] = (int16_t)nslot;
            }
            nslot += k;
            ns++;
        };
        for (int l = first; l <= a.last && fits; ++l) {
            TailLevel &L = a.L[l];
            const int64_t NV = h->NV[l];
            L.S = h->precision == MGD_FP64 ? (const void *)o.S64[l] : (const void *)o.S32[l];
            L.W = h->transfer == MGD_BOXMG && l < a.last ? o.W[l] : nullptr;
            L.n = h->nl[l];
            L.NV = (int)NV;
            L.off = (int)off;
            L.rnv = 1.0f / (float)(h->nl[l] + 1);
            if ((int64_t)(h->nl[l] + 1) * NV >= ((int64_t)1 << 22) || ns + 4 > kTailSegs) {
                fits = false;
                break;
            }
            seg(L.S, off + 3 * NV, 4 * NV);
            if (L.W) seg(L.W, off + 7 * NV, 4 * NV);
            if (l == first) {
                seg(f, off + NV, NV);
                if (!zero_guess) seg(u, off, NV);
            }
            off += (L.W ? 11 : 7) * NV;
        }
        size_t bytes = ((size_t)off * vb + 15) / 16 * 16;
        a.work_off = (int)bytes;
        bytes += (size_t)(a.m > 0 ? a.m : 1) * 8;
        if (fits && bytes <= cap) {
            a.nslot = nslot;
            if (h->precision == MGD_FP64) tail2d_launch_t<double>(a, bytes, st);
            else tail2d_launch_t<float>(a, bytes, st);
            HIPCHK(h->ctx, hipGetLastError());
            return MGD_OK;
        }
    }
    int64_t off = 0;
    for (int l = first; l <= a.last; ++l) {
        TailLevel &L = a.L[l];
        L.S = h->precision == MGD_FP64 ? (const void *)o.S64[l] : (const void *)o.S32[l];
        L.W = h->transfer == MGD_BOXMG && l < a.last ? o.W[l] : nullptr;
        L.n = h->nl[l];
        L.NV = (int)h->NV[l];
        L.off = (int)off;
        L.rnv = 1.0f / (float)(h->nl[l] + 1);
        if ((int64_t)(h->nl[l] + 1) * h->NV[l] >= ((int64_t)1 << 22))  // float-reciprocal indexing stays exact below
            return mgd_fail(h->ctx, MGD_EINVAL, "coarse level %d too large for the single-workgroup tail", l);
        off += 3 * h->NV[l];
    }
    size_t bytes = ((size_t)off * vb + 15) / 16 * 16;
    a.work_off = (int)bytes;
    bytes += (size_t)(a.m > 0 ? a.m : 1) * 8;
    if (bytes > cap) return mgd_fail(h->ctx, MGD_EINVAL, "coarse levels need %zu bytes of LDS", bytes);
    if (h->precision == MGD_FP64) {
        if (h->dim == 2) tail_launch_t<2, double>(a, bytes, st);
        else tail_launch_t<3, double>(a, bytes, st);
    } else {
        if (h->dim == 2) tail_launch_t<2, float>(a, bytes, st);
        else tail_launch_t<3, float>(a, bytes, st);
    }
    HIPCHK(h->ctx, hipGetLastError());
    return MGD_OK;
}

// multiplicative V(nu1,nu2) correction scheme from level l down; *res: the
// buffer holding the level's result (u, or the level's spare buffer when the
// fused 2D kernels ran from a zero start)
constexpr int64_t kPrerMaxNV = 300000;  // levels up to 513 x 513 vertices

static int vcycle_rec(mgd_hier *h, const OpSet &o, int l, void *u, const void *f, double omega, int nu1, int nu2,
                      bool zero_guess, const Lev2Dots *dots, bool *dots_done, void **res, hipStream_t st)
{
    int rc;
    *res = u;
    if (l == tail_first(h)) return launch_tail(h, o, l, u, f, omega, nu1, nu2, zero_guess, st);
    if (lev2_ok(h, l, nu1, nu2)) {
        // pre half: u (or its spare) <- S^2 u, r <- f - A u; post half into the other buffer
        void *us = zero_guess ? u : h->t[l];
        // small levels restrict inside the pre half (one launch less, the
        // weights stay in cache); large ones run the restriction as its own
        // pass, since the fused form re-reads the halo's transfer weights
        if (h->NV[l] <= kPrerMaxNV) {
            if ((rc = lev2_prer(h, o, l, zero_guess ? nullptr : u, f, us, h->f[l + 1], omega, st))) return rc;
        } else {
            if ((rc = lev2_pre(h, o, l, zero_guess ? nullptr : u, f, us, h->r[l], omega, st))) return rc;
            if ((rc = cycle_restrict(h, o, l, h->r[l], h->f[l + 1], st))) return rc;
        }
        void *ec = nullptr;
        if ((rc = vcycle_rec(h, o, l + 1, h->u[l + 1], h->f[l + 1], omega, nu1, nu2, true, nullptr, nullptr, &ec, st)))
            return rc;
        void *dst = us == u ? h->t[l] : u;
        if ((rc = lev2_post(h, o, l, us, ec, f, dst, omega, dots, st))) return rc;
        if (dots && dots_done) *dots_done = true;
        *res = dst;
        return MGD_OK;
    }
    if (nu1 > 0) {
        if ((rc = cycle_smooth(h, o, l, u, f, h->t[l], nu1, omega, zero_guess, st))) return rc;
    } else if (zero_guess) {
        if ((rc = fill_zero(h, u, h->NV[l], st))) return rc;
    }
    if ((rc = cycle_residual(h, o, l, u, f, h->r[l], st))) return rc;
    if ((rc = cycle_restrict(h, o, l, h->r[l], h->f[l + 1], st))) return rc;
    void *ec = nullptr;
    if ((rc = vcycle_rec(h, o, l + 1, h->u[l + 1], h->f[l + 1], omega, nu1, nu2, true, nullptr, nullptr, &ec, st)))
        return rc;
    if ((rc = cycle_prolong(h, o, l, ec, u, st))) return rc;
    if (nu2 > 0)
        if ((rc = cycle_smooth(h, o, l, u, f, h->t[l], nu2, omega, false, st))) return rc;
    return MGD_OK;
}

int vcycle_ops(mgd_hier *h, const OpSet &o, void *u, const void *f, double omega, int nu1, int nu2, bool zero_guess,
               hipStream_t st, const Lev2Dots *dots, void **result, bool *dots_done)
{
    if (dots_done) *dots_done = false;
    void *res = nullptr;
    int rc = vcycle_rec(h, o, 0, u, f, omega, nu1, nu2, zero_guess, dots, dots_done, &res, st);
    if (rc) return rc;
    if (result) *result = res;
    else if (res != u)
        HIPCHK(h->ctx, hipMemcpyAsync(u, res, h->NV[0] * h->vec_bytes(), hipMemcpyDeviceToDevice, st));
    return MGD_OK;
}

// ------------------------------------------------------------ FP64 outer

template <int D, class Op>
__global__ __launch_bounds__(256) void k_outer_residual(Op A, int n, const double *u, const double *f, double *r,
                                                        double *partial, float *rf)
{
    __shared__ double red[256];
    Grid<D> g(n);
    double rr = 0.0;
    for (int64_t v = block_index<D>() * blockDim.x + threadIdx.x; v < g.NV; v += (int64_t)gridDim.x * blockDim.x) {
        int x[3] = {0, 0, 0};
        g.coords(v, x);
        double rv = 0.0;
        if (g.interior(x)) {
            double Au, Dv;
            apply_row<D, Op, double>(A, g, v, x, u, Au, Dv);
            rv = f[v] - Au;
            rr += rv * rv;
        }
        r[v] = rv;
        if (rf) rf[v] = (float)rv;
    }
    double s = block_sum<256>(rr, red);
    if (threadIdx.x == 0 && partial) partial[blockIdx.x] = s;
}

// fixed-order sum of nvec runs of cnt block partials by one block
__global__ void k_reduce(const double *partial, int64_t cnt, int nvec, double *out)
{
    __shared__ double red[1024];
    for (int k = 0; k < nvec; ++k) {
        double s = 0.0;
        for (int64_t i = threadIdx.x; i < cnt; i += 1024) s += partial[k * cnt + i];
        double t = block_sum<1024>(s, red);
        if (threadIdx.x == 0) out[k] = t;
    }
}

// long partial lists (fused kernels on large grids) are first summed to one
int compress_partials(mgd_hier *h, const double *partial, int64_t cnt, int nvec, double *out, hipStream_t st)
{
    hipLaunchKernelGGL(k_reduce, dim3(1), dim3(1024), 0, st, partial, cnt, nvec, out);
    HIPCHK(h->ctx, hipGetLastError());
    return MGD_OK;
}

template <int D>
static int outer_residual_t(mgd_hier *h, const OpSet &o, const double *u, const double *f, double *r,
                            double *partial, unsigned grid, hipStream_t st)
{
    if (h->precision == MGD_FP64)
        hipLaunchKernelGGL((k_outer_residual<D, OpHalf<double>>), dim3(grid), dim3(256), 0, st,
                           OpHalf<double>{o.S64[0], h->NV[0]}, h->n, u, f, r, partial, (float *)nullptr);
    else
        // the mixed operator is the store's FP32 decode (kept current in S32[0]), applied in FP64
        hipLaunchKernelGGL((k_outer_residual<D, OpHalf<float>>), dim3(grid), dim3(256), 0, st,
                           OpHalf<float>{o.S32[0], h->NV[0]}, h->n, u, f, r, partial, (float *)h->f[0]);
    HIPCHK(h->ctx, hipGetLastError());
    return MGD_OK;
}

// r = f - A u (finest operator as stored, FP64); the partials of ||r||^2 go
// to h->partial (*nparts of them, when asked)
int outer_residual(mgd_hier *h, const OpSet &o, const double *u, const double *f, double *r, int *nparts,
                   hipStream_t st)
{
    double *partial = h->partial;
    if (h->dim == 2 && h->precision == MGD_MIXED) {
        StageArgs<double> sa;
        memset(&sa, 0, sizeof(sa));
        sa.sv = store_view(h, o);
        sa.n = h->n;
        sa.u = u;
        sa.f = f;
        sa.out = r;
        sa.partial = partial;
        sa.rf = (float *)h->f[0];
        stage2_tiles(h->n, sa.ntx, sa.nt);
        const unsigned grid = (unsigned)std::min<int64_t>({(int64_t)sa.nt, (int64_t)kRedBlocks, h->partial_cap});
        hipLaunchKernelGGL((k_stage2<double, ST_OUTER>), dim3(grid), dim3(256), 0, st, sa);
        HIPCHK(h->ctx, hipGetLastError());
        if (nparts) *nparts = (int)grid;
        return MGD_OK;
    }
    // as many blocks as the host-side sum takes (kHostParts): each thread's
    // rows gather 3^d FP64 neighbours, so occupancy hides their latency
    const unsigned grid = (unsigned)std::min<int64_t>({grid_for(h->NV[0], 256), (int64_t)kHostParts, h->partial_cap});
    if (nparts) *nparts = (int)grid;
    return h->dim == 2 ? outer_residual_t<2>(h, o, u, f, r, partial, grid, st)
                       : outer_residual_t<3>(h, o, u, f, r, partial, grid, st);
}

// ------------------------------------------------------------ outer vectors
// convert the FP64 residual to the cycle type (rhs of the correction equation)
template <typename T> __global__ void k_cast(const double *a, int64_t n, T *b)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = (T)a[i];
}

// u += e (e in the cycle type)
template <typename T> __global__ void k_add(double *u, const T *e, int64_t n)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) u[i] += (double)e[i];
}

// partials of z.r and z.(r - r_old): [blocks] then [blocks]
template <typename T>
__global__ __launch_bounds__(256) void k_dots_zr(const T *z, const double *r, const double *rold, int64_t n,
                                                 double *partial)
{
    __shared__ double red[256];
    double a = 0.0, b = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        double zz = (double)z[i];
        a += zz * r[i];
        b += zz * (r[i] - rold[i]);
    }
    double sa = block_sum<256>(a, red), sb = block_sum<256>(b, red);
    if (threadIdx.x == 0) { partial[blockIdx.x] = sa; partial[gridDim.x + blockIdx.x] = sb; }
}

// p_new = z + beta p_old on every vertex; Ap = A p_new on the interior,
// with partials of p_new . Ap; beta from the dot partials
template <int D, class Op, typename TZ>
__global__ __launch_bounds__(256) void k_p_matvec(Op A, int n, const TZ *z, const double *pold, double *pnew,
                                                  double *Ap, CgScalars c, double *partial)
{
    __shared__ double red[256];
    Grid<D> g(n);
    const double zr = sum_partials(c.p1, c.n1, red), zdr = sum_partials(c.p1 + c.n1, c.n1, red);
    const double beta = c.s[7] != 0.0 ? 0.0 : zdr / c.s[c.zr_old];
    if (blockIdx.x == 0 && threadIdx.x == 0) c.s[c.zr_new] = zr;
    double prod = 0.0;
    for (int64_t v = block_index<D>() * blockDim.x + threadIdx.x; v < g.NV; v += (int64_t)gridDim.x * blockDim.x) {
        int x[3] = {0, 0, 0};
        g.coords(v, x);
        double pv = (double)z[v] + beta * pold[v];
        pnew[v] = pv;
        if (g.interior(x)) {
            constexpr int H = n_half(D);
            double acc = 0.0, dsum = 0.0;
            for (int j = 0; j < H; ++j) {
                int64_t lin = half_lin(D, j, g.nv);
                double a = A.c(v, j, x);
                acc += a * ((double)z[v + lin] + beta * pold[v + lin]);
                dsum += a;
                int y[3] = {x[0] - half_off(D, j, 0), x[1] - half_off(D, j, 1), D == 3 ? x[2] - half_off(D, j, 2) : 0};
                double b = A.c(v - lin, j, y);
                acc += b * ((double)z[v - lin] + beta * pold[v - lin]);
                dsum += b;
            }
            double apv = -dsum * pv + acc;
            Ap[v] = apv;
            prod += pv * apv;
        } else {
            Ap[v] = 0.0;
        }
    }
    double sum = block_sum<256>(prod, red);
    if (threadIdx.x == 0) partial[blockIdx.x] = sum;
}

// 3D form of the same step: A p_new = A z + beta A p_old, with A p_old the
// previous step's product (the restart sets beta = 0 and the old product is
// not read), so the 27-point gather reads the FP32 z instead of the FP64
// p_old; the FP64 vectors are read and written at the vertex only
template <int D, class Op, typename TZ>
__global__ __launch_bounds__(256) void k_p_matvec_rec(Op A, int n, const TZ *z, const double *pold, double *pnew,
                                                      double *Ap, CgScalars c, double *partial)
{
    __shared__ double red[256];
    Grid<D> g(n);
    const double zr = sum_partials(c.p1, c.n1, red), zdr = sum_partials(c.p1 + c.n1, c.n1, red);
    const double beta = c.s[7] != 0.0 ? 0.0 : zdr / c.s[c.zr_old];
    if (blockIdx.x == 0 && threadIdx.x == 0) c.s[c.zr_new] = zr;
    double prod = 0.0;
    for (int64_t v = block_index<D>() * blockDim.x + threadIdx.x; v < g.NV; v += (int64_t)gridDim.x * blockDim.x) {
        int x[3] = {0, 0, 0};
        g.coords(v, x);
        const double zv = (double)z[v];
        const double pv = beta != 0.0 ? zv + beta * pold[v] : zv;
        pnew[v] = pv;
        if (g.interior(x)) {
            constexpr int H = n_half(D);
            double acc = 0.0, dsum = 0.0;
            for (int j = 0; j < H; ++j) {
                int64_t lin = half_lin(D, j, g.nv);
                double a = A.c(v, j, x);
                acc += a * (double)z[v + lin];
                dsum += a;
                int y[3] = {x[0] - half_off(D, j, 0), x[1] - half_off(D, j, 1), D == 3 ? x[2] - half_off(D, j, 2) : 0};
                double b = A.c(v - lin, j, y);
                acc += b * (double)z[v - lin];
                dsum += b;
            }
            const double az = -dsum * zv + acc;
            const double apv = beta != 0.0 ? az + beta * Ap[v] : az;
            Ap[v] = apv;
            prod += pv * apv;
        } else {
            Ap[v] = 0.0;
        }
    }
    double sum = block_sum<256>(prod, red);
    if (threadIdx.x == 0) partial[blockIdx.x] = sum;
}

// x += alpha p; r_old = r; r -= alpha Ap (and its FP32 copy); partials of
// r.r to pinned host memory; alpha = zr / p.Ap from the matvec's partials
__global__ __launch_bounds__(256) void k_cg_update(double *x, const double *p, double *r, double *rold,
                                                   const double *Ap, int64_t n, CgScalars c, const double *p2,
                                                   int64_t n2, double *partial, float *rf, const double *gate,
                                                   double thr)
{
    __shared__ double red[256];
    if (blockIdx.x == 0 && threadIdx.x == 0) c.s[7] = 0.0;  // restart consumed
    if (gate && *gate <= thr) {
        // the previous check converged: no update, the check repeats its norm
        if (threadIdx.x == 0) partial[blockIdx.x] = blockIdx.x == 0 ? *gate : 0.0;
        return;
    }
    const double pAp = sum_partials(p2, n2, red);
    const double alpha = c.s[c.zr_new] / pAp;
    double rr = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        x[i] += alpha * p[i];
        double ri = r[i];
        rold[i] = ri;
        ri -= alpha * Ap[i];
        r[i] = ri;
        if (rf) rf[i] = (float)ri;
        rr += ri * ri;
    }
    double sum = block_sum<256>(rr, red);
    if (threadIdx.x == 0) partial[blockIdx.x] = sum;
}

// host helpers used by the solver
int vec_cast_to_cycle(mgd_hier *h, const double *a, void *b, hipStream_t st)
{
    int64_t n = h->NV[0];
    if (h->precision == MGD_FP64) HIPCHK(h->ctx, hipMemcpyAsync(b, a, n * 8, hipMemcpyDeviceToDevice, st));
    else hipLaunchKernelGGL(k_cast<float>, dim3(grid_for(n, 256)), dim3(256), 0, st, a, n, (float *)b);
    HIPCHK(h->ctx, hipGetLastError());
    return MGD_OK;
}

int vec_add_cycle(mgd_hier *h, double *u, const void *e, hipStream_t st)
{
    int64_t n = h->NV[0];
    if (h->precision == MGD_FP64) hipLaunchKernelGGL(k_add<double>, dim3(grid_for(n, 256)), dim3(256), 0, st, u, (const double *)e, n);
    else hipLaunchKernelGGL(k_add<float>, dim3(grid_for(n, 256)), dim3(256), 0, st, u, (const float *)e, n);
    HIPCHK(h->ctx, hipGetLastError());
    return MGD_OK;
}

// partials of z.r and z.(r - r_old) into h->partial (h->p1_n each)
int pcg_dots(mgd_hier *h, const void *z, const double *r, const double *rold, hipStream_t st)
{
    int64_t n = h->NV[0];
    const unsigned grid = red_grid(n);
    if (h->precision == MGD_FP64) hipLaunchKernelGGL(k_dots_zr<double>, dim3(grid), dim3(256), 0, st, (const double *)z, r, rold, n, h->partial);
    else hipLaunchKernelGGL(k_dots_zr<float>, dim3(grid), dim3(256), 0, st, (const float *)z, r, rold, n, h->partial);
    HIPCHK(h->ctx, hipGetLastError());
    h->p1 = h->partial;
    h->p1_n = grid;
    return MGD_OK;
}

// k_p_matvec_rec on the 3D mixed finest store: the couplings decoded per
// vertex as in k_sweep3_store (the same values as the FP32 decode, applied
// in the same order, so the same bits)
template <typename TZ>
__global__ __launch_bounds__(256) void k_p_matvec_rec_store(StoreView sv, int n, const TZ *z, const double *pold,
                                                            double *pnew, double *Ap, CgScalars c, double *partial)
{
    __shared__ double red[256];
    Grid<3> g(n);
    const double zr = sum_partials(c.p1, c.n1, red), zdr = sum_partials(c.p1 + c.n1, c.n1, red);
    const double beta = c.s[7] != 0.0 ? 0.0 : zdr / c.s[c.zr_old];
    if (blockIdx.x == 0 && threadIdx.x == 0) c.s[c.zr_new] = zr;
    double prod = 0.0;
    for (int64_t v = block_index<3>() * blockDim.x + threadIdx.x; v < g.NV; v += (int64_t)gridDim.x * blockDim.x) {
        int x[3] = {0, 0, 0};
        g.coords(v, x);
        const double zv = (double)z[v];
        const double pv = beta != 0.0 ? zv + beta * pold[v] : zv;
        pnew[v] = pv;
        if (g.interior(x)) {
            float own[13], low[13];
            store3_couplings(sv, g, v, x, own, low);
            double acc = 0.0, dsum = 0.0;
#pragma unroll
            for (int j = 0; j < 13; ++j) {
                const int64_t lin = half_lin(3, j, g.nv);
                const double a = own[j];
                acc += a * (double)z[v + lin];
                dsum += a;
                const double b = low[j];
                acc += b * (double)z[v - lin];
                dsum += b;
            }
            const double az = -dsum * zv + acc;
            const double apv = beta != 0.0 ? az + beta * Ap[v] : az;
            Ap[v] = apv;
            prod += pv * apv;
        } else {
            Ap[v] = 0.0;
        }
    }
    double sum = block_sum<256>(prod, red);
    if (threadIdx.x == 0) partial[blockIdx.x] = sum;
}

template <int D, typename TZ>
static int pcg_matvec_t(mgd_hier *h, const OpSet &o, const TZ *z, const double *pold, double *pnew, double *Ap,
                        const CgScalars &c, hipStream_t st)
{
    // more blocks than the other reducing kernels: each thread's rows gather
    // 27 neighbours, and the product needs the occupancy to hide that latency
    const unsigned grid = (unsigned)std::min<int64_t>({grid_for(h->NV[0], 256), (int64_t)kPmvBlocks, h->partial_cap});
    if (D == 3) {
        if (h->precision == MGD_FP64)
            hipLaunchKernelGGL((k_p_matvec_rec<D, OpHalf<double>, TZ>), dim3(grid), dim3(256), 0, st,
                               OpHalf<double>{o.S64[0], h->NV[0]}, h->n, z, pold, pnew, Ap, c, h->partial2);
        else if (store3_decode(h))
            hipLaunchKernelGGL((k_p_matvec_rec_store<TZ>), dim3(grid), dim3(256), 0, st, store_view(h, o), h->n, z,
                               pold, pnew, Ap, c, h->partial2);
        else
            hipLaunchKernelGGL((k_p_matvec_rec<D, OpHalf<float>, TZ>), dim3(grid), dim3(256), 0, st,
                               OpHalf<float>{o.S32[0], h->NV[0]}, h->n, z, pold, pnew, Ap, c, h->partial2);
    } else if (h->precision == MGD_FP64)
        hipLaunchKernelGGL((k_p_matvec<D, OpHalf<double>, TZ>), dim3(grid), dim3(256), 0, st,
                           OpHalf<double>{o.S64[0], h->NV[0]}, h->n, z, pold, pnew, Ap, c, h->partial2);
    else
        hipLaunchKernelGGL((k_p_matvec<D, OpHalf<float>, TZ>), dim3(grid), dim3(256), 0, st,
                           OpHalf<float>{o.S32[0], h->NV[0]}, h->n, z, pold, pnew, Ap, c, h->partial2);
    HIPCHK(h->ctx, hipGetLastError());
    h->p2_n = grid;
    return MGD_OK;
}

// p_new = z + beta p_old, Ap = A p_new, partials of p.Ap into h->partial2
int pcg_matvec(mgd_hier *h, const OpSet &o, const void *z, const double *pold, double *pnew, double *Ap,
               const CgScalars &c, hipStream_t st)
{
    if (h->dim == 2 && h->NV[0] * 4 < ((int64_t)1 << 31)) return lev2_pmv(h, o, z, pold, pnew, Ap, c, st);
    if (h->precision == MGD_FP64)
        return h->dim == 2 ? pcg_matvec_t<2, double>(h, o, (const double *)z, pold, pnew, Ap, c, st)
                           : pcg_matvec_t<3, double>(h, o, (const double *)z, pold, pnew, Ap, c, st);
    return h->dim == 2 ? pcg_matvec_t<2, float>(h, o, (const float *)z, pold, pnew, Ap, c, st)
                       : pcg_matvec_t<3, float>(h, o, (const float *)z, pold, pnew, Ap, c, st);
}

// x += alpha p, r -= alpha Ap; the partials of r.r to the pinned host array
int pcg_update(mgd_hier *h, double *x, const double *p, double *r, double *rold, const double *Ap,
               const CgScalars &c, int gate_slot, double thr, int *nparts, hipStream_t st)
{
    int64_t n = h->NV[0];
    const unsigned grid = (unsigned)std::min<int64_t>({grid_for(n, 256), kHostParts, h->partial_cap});
    float *rf = h->precision == MGD_MIXED ? (float *)h->f[0] : nullptr;
    const double *gate = gate_slot >= 0 ? h->scal + kChkSlot + (gate_slot & 1) : nullptr;
    hipLaunchKernelGGL(k_cg_update, dim3(grid), dim3(256), 0, st, x, p, r, rold, Ap, n, c, (const double *)h->partial2,
                       h->p2_n, h->partial, rf, gate, thr);
    HIPCHK(h->ctx, hipGetLastError());
    *nparts = (int)grid;
    return MGD_OK;
}

// squared norm of a residual check from its partials, summed in one fixed
// order; to the device slot (the next cycle's gate) and the pinned host slot
__global__ __launch_bounds__(1024) void k_check_sum(const double *part, int n, double *dev_slot, double *host_slot)
{
    __shared__ double red[1024];
    red[threadIdx.x] = (int)threadIdx.x < n ? part[threadIdx.x] : 0.0;
    __syncthreads();
    for (int o = 512; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        *dev_slot = red[0];
        *host_slot = red[0];
    }
}

int check_sum(mgd_hier *h, int nparts, int slot, hipStream_t st)
{
    if (nparts < 1 || nparts > 1024 || nparts > h->partial_cap)
        return mgd_fail(h->ctx, MGD_EINVAL, "residual check with %d partials", nparts);
    if (slot < 0 || slot > 2) return mgd_fail(h->ctx, MGD_EINVAL, "residual check slot %d", slot);
    hipLaunchKernelGGL(k_check_sum, dim3(1), dim3(1024), 0, st, (const double *)h->partial, nparts,
                       h->scal + kChkSlot + slot, h->host_part_dev + slot);
    HIPCHK(h->ctx, hipGetLastError());
    return MGD_OK;
}

// ---- start of the iteration after an operator change.  The iterate carried
// over from the previous operator is kept unless its residual on the new
// operator exceeds that of the zero start (interior zeroed, boundary values
// kept); then the iteration restarts from the zero start.  Both squared
// norms are FP64 sums of block partials in fixed order.

// uz = u with the interior zeroed
template <int D> __global__ __launch_bounds__(256) void k_zero_interior(const double *u, int n, double *uz)
{
    Grid<D> g(n);
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= g.NV) return;
    int xc[3] = {0, 0, 0};
    g.coords(v, xc);
    uz[v] = g.interior(xc) ? 0.0 : u[v];
}

// the zero start's squared residual from its partials against the carried
// iterate's (*rr_u): the choice to *flag (1: zero start), the chosen start's
// squared residual to the check slots
__global__ __launch_bounds__(1024) void k_restart_pick(const double *part, int n, const double *rr_u, double *flag,
                                                       double *dev_slot, double *host_slot)
{
    __shared__ double red[1024];
    red[threadIdx.x] = (int)threadIdx.x < n ? part[threadIdx.x] : 0.0;
    __syncthreads();
    for (int o = 512; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const bool zero = *rr_u > red[0];
        *flag = zero ? 1.0 : 0.0;
        const double v = zero ? red[0] : *rr_u;
        *dev_slot = v;
        *host_slot = v;
    }
}

// the chosen start: u, r replaced by the zero start's when *flag is set; the
// FP32 copy of r (FP32 cycles) rewritten from the chosen residual
__global__ __launch_bounds__(256) void k_apply_start(const double *flag, const double *uz, const double *rz, int64_t n,
                                                     double *u, double *r, float *rf)
{
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    double rv = r[v];
    if (*flag != 0.0) {
        u[v] = uz[v];
        rv = rz[v];
        r[v] = rv;
    }
    if (rf) rf[v] = (float)rv;
}

int restart_pick(mgd_hier *h, const OpSet &o, int nparts, int slot, const double *f, double *u, double *r,
                 double *uz, double *rz, hipStream_t st)
{
    if (nparts < 1 || nparts > 1024 || nparts > h->partial_cap)
        return mgd_fail(h->ctx, MGD_EINVAL, "restart check with %d partials", nparts);
    // the carried iterate's squared residual (its partials are in h->partial)
    hipLaunchKernelGGL(k_check_sum, dim3(1), dim3(1024), 0, st, (const double *)h->partial, nparts,
                       h->scal + kRRuSlot, h->scal + kRRuSlot + 1);
    dim3 gv(grid_for(h->NV[0], 256));
    if (h->dim == 2) hipLaunchKernelGGL(k_zero_interior<2>, gv, dim3(256), 0, st, (const double *)u, h->n, uz);
    else hipLaunchKernelGGL(k_zero_interior<3>, gv, dim3(256), 0, st, (const double *)u, h->n, uz);
    HIPCHK(h->ctx, hipGetLastError());
    int nz = 0, rc;
    if ((rc = outer_residual(h, o, uz, f, rz, &nz, st))) return rc;
    if (nz < 1 || nz > 1024) return mgd_fail(h->ctx, MGD_EINVAL, "restart check with %d partials", nz);
    hipLaunchKernelGGL(k_restart_pick, dim3(1), dim3(1024), 0, st, (const double *)h->partial, nz,
                       (const double *)(h->scal + kRRuSlot), h->scal + kZeroSlot, h->scal + kChkSlot + (slot & 1),
                       h->host_part_dev + (slot & 1));
    float *rf = h->precision == MGD_MIXED ? (float *)h->f[0] : nullptr;
    hipLaunchKernelGGL(k_apply_start, gv, dim3(256), 0, st, (const double *)(h->scal + kZeroSlot),
                       (const double *)uz, (const double *)rz, h->NV[0], u, r, rf);
    HIPCHK(h->ctx, hipGetLastError());
    return MGD_OK;
}

int vec_fill_f64(mgd_ctx *ctx, double *a, int64_t n, double v, hipStream_t st)
{
    hipLaunchKernelGGL(k_fill<double>, dim3(grid_for(n, 256)), dim3(256), 0, st, a, n, v);
    HIPCHK(ctx, hipGetLastError());
    return MGD_OK;
}
