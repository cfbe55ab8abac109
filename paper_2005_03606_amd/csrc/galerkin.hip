// Coarse operators (paper Sec. 4): prolongation P (d-linear, or BoxMG's
// operator-dependent interpolation), R = P^T and the Ritz-Galerkin product
// A_{l+1} = P^T A_l P, computed stencil-wise for every coarse vertex; plus the
// dense FP64 Cholesky factor of the coarsest interior matrix.
#include <type_traits>

#include "common.h"

// ----------------------------------------------------- half-stencil rows
template <int D, typename T> struct HalfRow {
    const T *S;
    int64_t NV, nv;
    // coupling A[v][v+o] for a full-stencil index oi != centre
    __device__ inline T at(int64_t v, int oi) const
    {
        constexpr int c = D == 2 ? 4 : 13;
        if (oi > c) return S[(int64_t)(oi - c - 1) * NV + v];
        int mo = (D == 2 ? 8 : 26) - oi;  // index of -o
        int64_t lin = 0, st = 1;
        for (int m = 0; m < D; ++m) {
            int om = oi % 3 - 1;
            oi /= 3;
            lin += om * st;
            st *= nv;
        }
        return S[(int64_t)(mo - c - 1) * NV + v + lin];
    }
};

__device__ inline void off_of(int D, int oi, int *o)
{
    for (int m = 0; m < D; ++m) { o[m] = oi % 3 - 1; oi /= 3; }
}

__device__ inline double pw1(int d) { return d == 0 ? 1.0 : (d == 1 || d == -1) ? 0.5 : 0.0; }

// d-linear weights of fine vertex x toward the corners (x_m >> 1) + B_m
template <int D, typename T> __device__ inline void geo_weights(const int *x, T *w)
{
    for (int B = 0; B < (1 << D); ++B) {
        double p = 1.0;
        for (int m = 0; m < D; ++m) p *= pw1(x[m] - 2 * ((x[m] >> 1) + ((B >> m) & 1)));
        w[B] = (T)p;
    }
}

// BoxMG weights of an interior fine vertex v with odd coordinates: the row of
// v with offsets along even axes summed (collapsed); each odd-axis neighbour
// u contributes its own (final) weights wn(uv, u, wu); divided by the
// collapsed diagonal.  Computed in FP64 whatever the stored type T.
template <int D, typename T, class WN>
__device__ __forceinline__ void boxmg_row(const HalfRow<D, T> &A, const Grid<D> &g, int64_t v, const int *x, WN wn, double *w)
{
    constexpr int nl = 1 << D, ns = D == 2 ? 9 : 27, c = ns / 2;
    double acc[nl], diag = 0.0;
    for (int B = 0; B < nl; ++B) acc[B] = 0.0;
    // diagonal of the row: minus the sum of its couplings
    double dsum = 0.0;
    for (int oi = 0; oi < ns; ++oi)
        if (oi != c) dsum += (double)A.at(v, oi);
    for (int oi = 0; oi < ns; ++oi) {
        int o[3] = {0, 0, 0}, u[3] = {0, 0, 0};
        off_of(D, oi, o);
        double a = oi == c ? -dsum : (double)A.at(v, oi);
        bool self = true;
        for (int m = 0; m < D; ++m) {
            int om = (x[m] & 1) ? o[m] : 0;
            u[m] = x[m] + om;
            if (om) self = false;
        }
        if (self) { diag += a; continue; }
        double wu[nl];
        wn(g.vid(u), u, wu);
        for (int Bu = 0; Bu < nl; ++Bu) {
            if (wu[Bu] == 0.0) continue;
            int B = 0;
            for (int m = 0; m < D; ++m) B |= (((u[m] >> 1) + ((Bu >> m) & 1)) - (x[m] >> 1)) << m;
            acc[B] -= a * wu[Bu];
        }
    }
    for (int B = 0; B < nl; ++B) w[B] = acc[B] / diag;
}

// pass k: fine vertices with k odd coordinates (k = 0 also sets every
// boundary vertex, d-linear weights); pass k reads the weights of pass k - 1
template <int D, typename T>
__device__ __forceinline__ void weights_vertex(const HalfRow<D, T> &A, const Grid<D> &g, int pass, int64_t v, T *W)
{
    int x[3] = {0, 0, 0};
    g.coords(v, x);
    int odd = 0;
    for (int m = 0; m < D; ++m) odd += x[m] & 1;
    bool bnd = !g.interior(x);
    constexpr int nl = 1 << D;
    double w[nl];
    if (pass == 0) {
        if (!(bnd || odd == 0)) return;
        geo_weights<D, double>(x, w);
    } else {
        if (bnd || odd != pass) return;
        boxmg_row<D, T>(A, g, v, x,
                        [&](int64_t uv, const int *, double *wu) {
                            for (int Bu = 0; Bu < nl; ++Bu) wu[Bu] = (double)W[(int64_t)Bu * g.NV + uv];
                        },
                        w);
    }
    for (int B = 0; B < nl; ++B) W[(int64_t)B * g.NV + v] = (T)w[B];
}

template <int D, typename T>
__global__ void k_weights(HalfRow<D, T> A, int n, int pass, T *W)
{
    Grid<D> g(n);
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v < g.NV) weights_vertex<D, T>(A, g, pass, v, W);
}

// 2D in two phases: phase 0 sets the boundary, even-even (d-linear) and
// one-odd vertices (their odd-axis neighbours are even-even, whose weights
// are d-linear); phase 1 the vertices with both coordinates odd, from the
// stored weights of their neighbours
template <typename T, int PHASE>
__device__ __forceinline__ void weights2_vertex(const HalfRow<2, T> &A, const Grid<2> &g, int64_t v, T *W)
{
    int x[3] = {0, 0, 0};
    g.coords(v, x);
    const int odd = (x[0] & 1) + (x[1] & 1);
    const bool in = g.interior(x);
    if ((PHASE == 1) != (in && odd == 2)) return;
    double w[4];
    if (!in || odd == 0) {
        geo_weights<2, double>(x, w);
    } else if (odd == 1) {
        boxmg_row<2, T>(A, g, v, x, [&](int64_t, const int *u, double *wu) { geo_weights<2, double>(u, wu); }, w);
    } else {
        boxmg_row<2, T>(A, g, v, x,
                        [&](int64_t uv, const int *, double *wu) {
                            for (int Bu = 0; Bu < 4; ++Bu) wu[Bu] = (double)W[(int64_t)Bu * g.NV + uv];
                        },
                        w);
    }
    for (int B = 0; B < 4; ++B) W[(int64_t)B * g.NV + v] = (T)w[B];
}

template <typename T, int PHASE>
__global__ __launch_bounds__(256) void k_weights2(HalfRow<2, T> A, int n, T *W)
{
    Grid<2> g(n);
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v < g.NV) weights2_vertex<T, PHASE>(A, g, v, W);
}

// weight of fine vertex x toward coarse vertex X (0 unless X is a corner of x's box)
template <int D, typename T>
__device__ inline T weight_to(const T *W, int64_t NV, int64_t v, const int *x, const int *X)
{
    int B = 0;
    for (int m = 0; m < D; ++m) {
        int b = X[m] - (x[m] >> 1);
        if (b < 0 || b > 1) return (T)0;
        B |= b << m;
    }
    if (W) return W[(int64_t)B * NV + v];
    double p = 1.0;
    for (int m = 0; m < D; ++m) p *= pw1(x[m] - 2 * X[m]);
    return (T)p;
}

// coarse coupling A_c[X][X+O_J] = sum_v sum_{w != v} P_vX A_vw (P_w,X+O - P_v,X+O),
// valid because every row of A sums to zero and P reproduces constants.  The
// 3^d fine vertices v around 2X are taken by separate threads (CPB coarse
// vertices per workgroup) and their partial sums are added in v order.
// Computed in FP64 whatever the stored type T.
template <int D> constexpr int gal_cpb() { return D == 2 ? 32 : 8; }
template <int D> constexpr int gal_threads() { return gal_cpb<D>() * (D == 2 ? 9 : 27); }

// one group of gal_threads() threads (tg: index in the group, -1 for a
// thread of the workgroup outside every group) computes the coarse vertices
// V0 .. V0 + CPB - 1; every thread of the workgroup calls it (one barrier)
// k-th vertex on the boundary of the 3D grid with nc cells per axis: the
// planes z = 0 and z = nc, then per interior plane the rows y = 0 and y = nc
// and the two end vertices of every other row
__device__ inline int64_t bnd_vertex3(int64_t k, int nc)
{
    const int64_t nv = nc + 1, face = nv * nv;
    int x, y, z;
    if (k < 2 * face) {
        z = k < face ? 0 : nc;
        const int64_t r = k < face ? k : k - face;
        x = (int)(r % nv);
        y = (int)(r / nv);
    } else {
        const int64_t kk = k - 2 * face, per = 4 * (int64_t)nc;
        z = 1 + (int)(kk / per);
        const int64_t r = kk % per;
        if (r < 2 * nv) {
            y = r < nv ? 0 : nc;
            x = (int)(r % nv);
        } else {
            const int64_t q = r - 2 * nv;
            y = 1 + (int)(q / 2);
            x = (q & 1) ? nc : 0;
        }
    }
    return x + nv * (y + nv * (int64_t)z);
}
__host__ __device__ inline int64_t bnd_count3(int nc) { return 2 * (int64_t)(nc + 1) * (nc + 1) + (int64_t)(nc - 1) * 4 * nc; }

// BND: the group's vertices are boundary vertices (bnd_vertex3 order)
template <int D, typename T, bool BND = false>
__device__ __forceinline__ void galerkin_group(const HalfRow<D, T> &A, const T *W, int nf, T *Sc, int64_t V0, int tg,
                                      double (*part)[gal_cpb<D>()][n_half(D)])
{
    constexpr int H = n_half(D), ns = D == 2 ? 9 : 27, c = ns / 2, CPB = gal_cpb<D>();
    Grid<D> gf(nf), gc(nf / 2);
    const int cv = tg % CPB, sv = tg / CPB;
    const int64_t cnt = BND ? bnd_count3(gc.n) : gc.NV;
    auto vert = [&](int64_t k) { if constexpr (BND) return bnd_vertex3(k, gc.n); else return k; };
    const int64_t V = V0 + cv < cnt ? vert(V0 + cv) : 0;
    double acc[H];
    for (int j = 0; j < H; ++j) acc[j] = 0.0;
    int X[3] = {0, 0, 0};
    if (tg >= 0 && V0 + cv < cnt) {
        gc.coords(V, X);
        int dv[3] = {0, 0, 0}, x[3] = {0, 0, 0};
        off_of(D, sv, dv);
        bool ok = true;
        for (int m = 0; m < D; ++m) {
            x[m] = 2 * X[m] + dv[m];
            if (x[m] < 0 || x[m] > nf) ok = false;
        }
        const int64_t v = ok ? gf.vid(x) : 0;
        const double pV = ok ? (double)weight_to<D, T>(W, gf.NV, v, x, X) : 0.0;
        if (pV != 0.0) {
            double pvW[H];
            for (int j = 0; j < H; ++j) {
                int XW[3] = {0, 0, 0};
                for (int m = 0; m < D; ++m) XW[m] = X[m] + half_off(D, j, m);
                pvW[j] = (double)weight_to<D, T>(W, gf.NV, v, x, XW);
            }
            for (int oi = 0; oi < ns; ++oi) {
                if (oi == c) continue;
                int o[3] = {0, 0, 0}, y[3] = {0, 0, 0};
                off_of(D, oi, o);
                bool okw = true;
                for (int m = 0; m < D; ++m) {
                    y[m] = x[m] + o[m];
                    if (y[m] < 0 || y[m] > nf) okw = false;
                }
                if (!okw) continue;
                const int64_t w = gf.vid(y);
                const double a = (double)A.at(v, oi);
                if (a == 0.0) continue;
                const double pa = pV * a;
                for (int j = 0; j < H; ++j) {
                    int XW[3] = {0, 0, 0};
                    for (int m = 0; m < D; ++m) XW[m] = X[m] + half_off(D, j, m);
                    acc[j] += pa * ((double)weight_to<D, T>(W, gf.NV, w, y, XW) - pvW[j]);
                }
            }
        }
    }
    if (tg >= 0)
        for (int j = 0; j < H; ++j) part[sv][cv][j] = acc[j];
    __syncthreads();
    for (int t = tg; t >= 0 && t < CPB * H; t += CPB * ns) {
        const int c2 = t / H, j = t % H;
        if (V0 + c2 >= cnt) continue;
        const int64_t V2 = vert(V0 + c2);
        double sum = 0.0;
        for (int k = 0; k < ns; ++k) sum += part[k][c2][j];
        int X2[3] = {0, 0, 0};
        gc.coords(V2, X2);
        // couplings to vertices outside the coarse grid are zero
        bool inside = true;
        for (int m = 0; m < D; ++m) {
            int Y = X2[m] + half_off(D, j, m);
            if (Y < 0 || Y > gc.n) inside = false;
        }
        Sc[(int64_t)j * gc.NV + V2] = inside ? (T)sum : (T)0;
    }
}

template <int D, typename T, bool BND = false>
__global__ __launch_bounds__(gal_threads<D>()) void k_galerkin_p(HalfRow<D, T> A, const T *W, int nf, T *Sc)
{
    __shared__ double part[D == 2 ? 9 : 27][gal_cpb<D>()][n_half(D)];
    galerkin_group<D, T, BND>(A, W, nf, Sc, (int64_t)blockIdx.x * gal_cpb<D>(), (int)threadIdx.x, part);
}

// 3D interior coarse vertices (1 <= X_m <= nc - 1), one thread each, every
// fine vertex v = 2X + dv of the support and every neighbour w = v + o
// unrolled.  With X interior the whole 5^3 fine neighbourhood exists, and
// whether P[v'][X + O] can be nonzero depends only on v' - 2X and O (P is
// supported on the box corners of v' and, along an even axis of v', only on
// the coarse vertex v'_m / 2), so every structurally zero term is dropped at
// compile time: 1707 FP64 terms, 702 coupling and 185 weight loads per
// coarse vertex.  The sums run in galerkin_group's order (per fine vertex
// over its neighbours, then over the fine vertices), so both give the same
// bits.
template <int N, class F> __device__ __forceinline__ void unroll(F &&f)
{
    if constexpr (N > 0) {
        unroll<N - 1>(f);
        f(std::integral_constant<int, N - 1>{});
    }
}
__host__ __device__ constexpr int floor_half(int e) { return (e + 4) / 2 - 2; }
// corner index (bit m set: corner X_m + 1 of v's box) of X + O for v = 2X + e
// when P[v][X + O] can be nonzero, else -1
__host__ __device__ constexpr int p_corner(int e0, int e1, int e2, int O0, int O1, int O2)
{
    const int e[3] = {e0, e1, e2}, O[3] = {O0, O1, O2};
    int B = 0;
    for (int m = 0; m < 3; ++m) {
        const int b = O[m] - floor_half(e[m]);
        if (b < 0 || b > 1 || (e[m] % 2 == 0 && b == 1)) return -1;
        B |= b << m;
    }
    return B;
}
__host__ __device__ constexpr int hoff(int j, int m)
{
    int i = 14 + j;
    for (int k = 0; k < m; ++k) i /= 3;
    return i % 3 - 1;
}

template <typename T, bool GEO>
__global__ __launch_bounds__(256) void k_galerkin3_int(HalfRow<3, T> A, const T *W, int nf, T *Sc)
{
    const int nc = nf / 2, ni = nc - 1;
    const int64_t idx = block_index<3>() * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)ni * ni * ni) return;
    const int X0 = 1 + (int)(idx % ni), X1 = 1 + (int)((idx / ni) % ni), X2 = 1 + (int)(idx / ((int64_t)ni * ni));
    const int64_t nv = A.nv, nv2 = nv * nv, NVf = A.NV;
    const int64_t c0 = 2 * (int64_t)X0 + nv * 2 * X1 + nv2 * 2 * X2;  // fine index of 2X
    auto fidx = [&](int e0, int e1, int e2) { return c0 + e0 + e1 * nv + e2 * nv2; };
    // P[2X + e][X + O], B its corner index (compile-time)
    auto pw = [&](int B, int e0, int e1, int e2, int O0, int O1, int O2) -> double {
        if constexpr (GEO) {
            double p = 1.0;
            const int d[3] = {e0 - 2 * O0, e1 - 2 * O1, e2 - 2 * O2};
            for (int m = 0; m < 3; ++m) p *= d[m] == 0 ? 1.0 : 0.5;
            return p;
        } else {
            return (double)W[(int64_t)B * NVf + fidx(e0, e1, e2)];
        }
    };
    double acc[13];
#pragma unroll
    for (int j = 0; j < 13; ++j) acc[j] = 0.0;
    unroll<27>([&](auto SV) {
        constexpr int sv = decltype(SV)::value;
        constexpr int d0 = sv % 3 - 1, d1 = sv / 3 % 3 - 1, d2 = sv / 9 - 1;
        constexpr int BX = p_corner(d0, d1, d2, 0, 0, 0);
        const double pV = pw(BX, d0, d1, d2, 0, 0, 0);
        if (pV == 0.0) return;
        double pvW[13];
        unroll<13>([&](auto J) {
            constexpr int j = decltype(J)::value;
            constexpr int B = p_corner(d0, d1, d2, hoff(j, 0), hoff(j, 1), hoff(j, 2));
            if constexpr (B >= 0) pvW[j] = pw(B, d0, d1, d2, hoff(j, 0), hoff(j, 1), hoff(j, 2));
            else pvW[j] = 0.0;
        });
        const int64_t v = fidx(d0, d1, d2);
        double t[13];
#pragma unroll
        for (int j = 0; j < 13; ++j) t[j] = 0.0;
        unroll<27>([&](auto OI) {
            constexpr int oi = decltype(OI)::value;
            if constexpr (oi != 13) {
                constexpr int o0 = oi % 3 - 1, o1 = oi / 3 % 3 - 1, o2 = oi / 9 - 1;
                constexpr int e0 = d0 + o0, e1 = d1 + o1, e2 = d2 + o2;
                const double pa = pV * (double)A.at(v, oi);
                unroll<13>([&](auto J) {
                    constexpr int j = decltype(J)::value;
                    constexpr int O0 = hoff(j, 0), O1 = hoff(j, 1), O2 = hoff(j, 2);
                    constexpr int Bw = p_corner(e0, e1, e2, O0, O1, O2);
                    constexpr int Bv = p_corner(d0, d1, d2, O0, O1, O2);
                    if constexpr (Bw >= 0) t[j] += pa * (pw(Bw, e0, e1, e2, O0, O1, O2) - pvW[j]);
                    else if constexpr (Bv >= 0) t[j] += pa * (0.0 - pvW[j]);
                });
            }
        });
#pragma unroll
        for (int j = 0; j < 13; ++j) acc[j] += t[j];
    });
    const int64_t nvc = nc + 1, V = X0 + nvc * (X1 + nvc * (int64_t)X2), NVc = nvc * nvc * nvc;
#pragma unroll
    for (int j = 0; j < 13; ++j) Sc[(int64_t)j * NVc + V] = (T)acc[j];
}

// ------------------------------------------------------------ coarsest solve
// interior index of vertex x on a grid with n cells: sum (x_m - 1) (n-1)^m
template <int D> __device__ inline int64_t interior_index(const int *x, int n)
{
    int64_t k = 0, st = 1;
    for (int m = 0; m < D; ++m) { k += (int64_t)(x[m] - 1) * st; st *= (n - 1); }
    return k;
}

template <int D, typename T>
__global__ void k_dense_assemble(HalfRow<D, T> A, int n, int64_t m, double *M)
{
    Grid<D> g(n);
    for (int64_t i = threadIdx.x; i < m * m; i += blockDim.x) M[i] = 0.0;
    __syncthreads();
    constexpr int ns = D == 2 ? 9 : 27, c = ns / 2;
    for (int64_t v = threadIdx.x; v < g.NV; v += blockDim.x) {
        int x[3] = {0, 0, 0};
        g.coords(v, x);
        if (!g.interior(x)) continue;
        int64_t r = interior_index<D>(x, n);
        double dsum = 0.0;
        for (int oi = 0; oi < ns; ++oi) {
            if (oi == c) continue;
            double a = (double)A.at(v, oi);
            dsum += a;
            int o[3] = {0, 0, 0}, y[3] = {0, 0, 0};
            off_of(D, oi, o);
            for (int mm = 0; mm < D; ++mm) y[mm] = x[mm] + o[mm];
            if (g.interior(y)) M[r * m + interior_index<D>(y, n)] = a;
        }
        M[r * m + r] = -dsum;
    }
}

// left-looking Cholesky in place (lower triangle), one workgroup
__global__ void k_cholesky(double *M, int64_t m)
{
    __shared__ double red[256];
    for (int64_t j = 0; j < m; ++j) {
        double s = 0.0;
        for (int64_t k = threadIdx.x; k < j; k += blockDim.x) s += M[j * m + k] * M[j * m + k];
        red[threadIdx.x] = s;
        __syncthreads();
        for (int o = 128; o > 0; o >>= 1) {
            if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
            __syncthreads();
        }
        double ljj = sqrt(M[j * m + j] - red[0]);
        __syncthreads();
        for (int64_t i = j + 1 + threadIdx.x; i < m; i += blockDim.x) {
            double t = M[i * m + j];
            for (int64_t k = 0; k < j; ++k) t -= M[i * m + k] * M[j * m + k];
            M[i * m + j] = t / ljj;
        }
        if (threadIdx.x == 0) M[j * m + j] = ljj;
        __syncthreads();
    }
}

// inverse of L L^T, one thread per column j: L y = e_j, then L^T x = y,
// both in place in column j of Ainv (m <= kCinvMax)
__global__ void k_chol_inverse(const double *L, int64_t m, double *Ainv)
{
    const int64_t j = threadIdx.x;
    if (j >= m) return;
    for (int64_t i = 0; i < m; ++i) {
        double s = i == j ? 1.0 : 0.0;
        for (int64_t k = j; k < i; ++k) s -= L[i * m + k] * Ainv[k * m + j];
        Ainv[i * m + j] = i < j ? 0.0 : s / L[i * m + i];
    }
    for (int64_t i = m - 1; i >= 0; --i) {
        double s = Ainv[i * m + j];
        for (int64_t k = i + 1; k < m; ++k) s -= L[k * m + i] * Ainv[k * m + j];
        Ainv[i * m + j] = s / L[i * m + i];
    }
}

// 3D BoxMG weights of the interior fine vertices whose odd axes are the set
// bits of ODD, one thread each, the 27 offsets unrolled.  The neighbour u of
// the collapsed row has odd coordinates only where x is odd and the offset
// is 0, and its weights vanish structurally along its even axes, so the
// corner of every term is fixed at compile time; the sums run in
// boxmg_row's order and give the same bits.
template <typename T, int ODD>
__global__ __launch_bounds__(256) void k_weights3_class(HalfRow<3, T> A, int nf, T *W)
{
    constexpr int p0 = ODD & 1, p1 = (ODD >> 1) & 1, p2 = (ODD >> 2) & 1;
    const int nc = nf / 2;
    const int c0 = p0 ? nc : nc - 1, c1 = p1 ? nc : nc - 1, c2 = p2 ? nc : nc - 1;
    const int64_t idx = block_index<3>() * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)c0 * c1 * c2) return;
    const int i0 = (int)(idx % c0), i1 = (int)((idx / c0) % c1), i2 = (int)(idx / ((int64_t)c0 * c1));
    const int x0 = 2 * i0 + (p0 ? 1 : 2), x1 = 2 * i1 + (p1 ? 1 : 2), x2 = 2 * i2 + (p2 ? 1 : 2);
    const int64_t nv = A.nv, nv2 = nv * nv, NV = A.NV;
    const int64_t v = x0 + nv * x1 + nv2 * x2;
    double dsum = 0.0;
    unroll<27>([&](auto OI) {
        constexpr int oi = decltype(OI)::value;
        if constexpr (oi != 13) dsum += (double)A.at(v, oi);
    });
    double acc[8], diag = 0.0;
#pragma unroll
    for (int B = 0; B < 8; ++B) acc[B] = 0.0;
    unroll<27>([&](auto OI) {
        constexpr int oi = decltype(OI)::value;
        constexpr int o0 = oi % 3 - 1, o1 = oi / 3 % 3 - 1, o2 = oi / 9 - 1;
        constexpr int m0 = p0 ? o0 : 0, m1 = p1 ? o1 : 0, m2 = p2 ? o2 : 0;  // collapsed offset
        const double a = oi == 13 ? -dsum : (double)A.at(v, oi);
        if constexpr (m0 == 0 && m1 == 0 && m2 == 0) {
            diag += a;
        } else {
            // u = x + m: odd exactly where x is odd and m is 0
            constexpr int q0 = p0 && m0 == 0, q1 = p1 && m1 == 0, q2 = p2 && m2 == 0;
            const int64_t uv = v + m0 + m1 * nv + m2 * nv2;
            unroll<8>([&](auto BU) {
                constexpr int Bu = decltype(BU)::value;
                constexpr int b0 = Bu & 1, b1 = (Bu >> 1) & 1, b2 = (Bu >> 2) & 1;
                if constexpr ((!b0 || q0) && (!b1 || q1) && (!b2 || q2)) {
                    // corner of x's box: floor((p + m) / 2) + b per axis
                    constexpr int B = ((floor_half(p0 + m0) + b0) << 0) | ((floor_half(p1 + m1) + b1) << 1) |
                                      ((floor_half(p2 + m2) + b2) << 2);
                    const double wu = (double)W[(int64_t)Bu * NV + uv];
                    if (wu != 0.0) acc[B] -= a * wu;
                }
            });
        }
    });
#pragma unroll
    for (int B = 0; B < 8; ++B) W[(int64_t)B * NV + v] = (T)(acc[B] / diag);
}

template <int D, typename T>
static void weights_launch(const HalfRow<D, T> &A, int nf, int64_t NV, T *W, hipStream_t st)
{
    dim3 gv(grid_for(NV, 256));
    if constexpr (D == 2) {
        hipLaunchKernelGGL((k_weights2<T, 0>), gv, dim3(256), 0, st, A, nf, W);
        hipLaunchKernelGGL((k_weights2<T, 1>), gv, dim3(256), 0, st, A, nf, W);
    } else {
        hipLaunchKernelGGL((k_weights<D, T>), gv, dim3(256), 0, st, A, nf, 0, W);
        const int64_t nc = nf / 2;
        // pass k: the interior vertices with k odd coordinates, one launch per
        // odd set (nc odd and nc - 1 even interior coordinates per axis)
        const int64_t n1 = nc * (nc - 1) * (nc - 1), n2 = nc * nc * (nc - 1), n3 = nc * nc * nc;
        if (n1 > 0) {
            hipLaunchKernelGGL((k_weights3_class<T, 1>), dim3(grid_for(n1, 256)), dim3(256), 0, st, A, nf, W);
            hipLaunchKernelGGL((k_weights3_class<T, 2>), dim3(grid_for(n1, 256)), dim3(256), 0, st, A, nf, W);
            hipLaunchKernelGGL((k_weights3_class<T, 4>), dim3(grid_for(n1, 256)), dim3(256), 0, st, A, nf, W);
        }
        if (n2 > 0) {
            hipLaunchKernelGGL((k_weights3_class<T, 3>), dim3(grid_for(n2, 256)), dim3(256), 0, st, A, nf, W);
            hipLaunchKernelGGL((k_weights3_class<T, 5>), dim3(grid_for(n2, 256)), dim3(256), 0, st, A, nf, W);
            hipLaunchKernelGGL((k_weights3_class<T, 6>), dim3(grid_for(n2, 256)), dim3(256), 0, st, A, nf, W);
        }
        if (n3 > 0) hipLaunchKernelGGL((k_weights3_class<T, 7>), dim3(grid_for(n3, 256)), dim3(256), 0, st, A, nf, W);
    }
}

template <int D, typename T>
static void galerkin_launch(const HalfRow<D, T> &A, const T *W, int nf, int64_t NVc, T *Sc, hipStream_t st)
{
    constexpr int CPB = gal_cpb<D>(), ns = D == 2 ? 9 : 27;
    const int nc = nf / 2;
    if constexpr (D == 3) {
        if (nc >= 4) {
            // interior vertices unrolled, the boundary surface by groups
            const int64_t ni = (int64_t)(nc - 1) * (nc - 1) * (nc - 1);
            if (W) hipLaunchKernelGGL((k_galerkin3_int<T, false>), dim3(grid_for(ni, 256)), dim3(256), 0, st, A, W, nf, Sc);
            else hipLaunchKernelGGL((k_galerkin3_int<T, true>), dim3(grid_for(ni, 256)), dim3(256), 0, st, A, W, nf, Sc);
            hipLaunchKernelGGL((k_galerkin_p<D, T, true>), dim3(grid_for(bnd_count3(nc), CPB)), dim3(CPB * ns), 0, st,
                               A, W, nf, Sc);
            return;
        }
    }
    hipLaunchKernelGGL((k_galerkin_p<D, T>), dim3(grid_for(NVc, CPB)), dim3(CPB * ns), 0, st, A, W, nf, Sc);
}

// weights, Galerkin products and the coarsest matrix in FP64 arithmetic; the
// mixed form stores the levels in FP32 (its finest level: the FP32 decode of
// the store, kept current by every change of the store)
// one wavefront per 64-vertex tile of W (3D): 1 if every structurally
// nonzero weight of the tile's vertices equals the d-linear weight
template <typename T> __global__ __launch_bounds__(256) void k_wgeo_tiles(const T *W, int n, uint8_t *flags)
{
    Grid<3> g(n);
    const int64_t ntile = (g.NV + 63) / 64;
    const int64_t t = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (t >= ntile) return;
    const int64_t v = t * 64 + (threadIdx.x & 63);
    bool geo = true;
    if (v < g.NV) {
        int x[3];
        g.coords(v, x);
        double w[8];
        geo_weights<3, double>(x, w);
        const int odd = (x[0] & 1) | ((x[1] & 1) << 1) | ((x[2] & 1) << 2);
        for (int B = 0; B < 8; ++B)
            if (!(B & ~odd) && W[(int64_t)B * g.NV + v] != (T)w[B]) geo = false;
    }
    const bool all = __all(geo);
    if ((threadIdx.x & 63) == 0) flags[t] = all ? 1 : 0;
}

template <typename T> static void wgeo_launch(const T *W, int n, int64_t NV, uint8_t *flags, hipStream_t st)
{
    if (!flags) return;
    const int64_t ntile = (NV + 63) / 64;
    hipLaunchKernelGGL((k_wgeo_tiles<T>), dim3(grid_for(ntile, 4)), dim3(256), 0, st, W, n, flags);
}

template <int D, typename T> static int coarsen_t(mgd_hier *h, OpSet &o, T *const *S, hipStream_t st)
{
    o.dz_ok = 0;
    mgd_ctx *ctx = h->ctx;
    for (int l = 0; l + 1 < h->nlev; ++l) {
        HalfRow<D, T> A{S[l], h->NV[l], (int64_t)h->nl[l] + 1};
        T *W = (T *)o.W[l];
        if (h->transfer == MGD_BOXMG) {
            weights_launch<D, T>(A, h->nl[l], h->NV[l], W, st);
            if (D == 3) wgeo_launch<T>(W, h->nl[l], h->NV[l], o.wgeo[l], st);
        }
        galerkin_launch<D, T>(A, (const T *)(h->transfer == MGD_BOXMG ? W : nullptr), h->nl[l], h->NV[l + 1],
                              S[l + 1], st);
    }
    int lc = h->nlev - 1;
    HalfRow<D, T> Ac{S[lc], h->NV[lc], (int64_t)h->nl[lc] + 1};
    hipLaunchKernelGGL((k_dense_assemble<D, T>), dim3(1), dim3(256), 0, st, Ac, h->nl[lc], h->m_coarse, o.chol);
    hipLaunchKernelGGL(k_cholesky, dim3(1), dim3(256), 0, st, o.chol, h->m_coarse);
    if (o.cinv) hipLaunchKernelGGL(k_chol_inverse, dim3(1), dim3((unsigned)kCinvMax), 0, st, o.chol, h->m_coarse, o.cinv);
    HIPCHK(ctx, hipGetLastError());
    return MGD_OK;
}

// ---- geometric hierarchy of a provisional operator (Sec. 1: multigrid
// starts from crude fine grid stencils with geometric coarse grid and
// inter-grid transfer operators, cheap to set up): every coarser level is
// the Q1 rediscretisation with cell values that average the 2^d child
// cells' (the finest level's: the centre samples), transfer weights are
// d-linear, and the coarsest matrix is factored as usual.

// coarse cell values: the mean of the 2^d children on the nf-grid (FP64 sum)
template <int D> __global__ void k_avg_children(const float *ef, int nf, float *ec)
{
    const int nc = nf / 2;
    int64_t NC = 1;
    for (int m = 0; m < D; ++m) NC *= nc;
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= NC) return;
    int X[3] = {0, 0, 0};
    int64_t t = c;
    for (int m = 0; m < D; ++m) { X[m] = (int)(t % nc); t /= nc; }
    double sum = 0.0;
    for (int B = 0; B < (1 << D); ++B) {
        int64_t f = 0, st = 1;
        for (int m = 0; m < D; ++m) {
            f += (int64_t)(2 * X[m] + ((B >> m) & 1)) * st;
            st *= nf;
        }
        sum += (double)ef[f];
    }
    ec[c] = (float)(sum / (double)(1 << D));
}

// half stencils of the cell-value rediscretisation on the n-grid (the
// store's base couplings), computed in FP64 and stored as T
template <int D, typename T> __global__ void k_base_stencils(const float *ec, int n, T *S)
{
    Grid<D> g(n);
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= g.NV) return;
    int x[3] = {0, 0, 0};
    g.coords(v, x);
    BaseCells<D> bc;
    bc.load(ec, n, x);
#pragma unroll
    for (int j = 0; j < n_half(D); ++j) S[(int64_t)j * g.NV + v] = (T)bc.coupling(j, nullptr);
}

template <int D, typename T> __global__ void k_geo_weights_t(int n, T *W)
{
    Grid<D> g(n);
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= g.NV) return;
    int x[3] = {0, 0, 0};
    g.coords(v, x);
    double w[1 << D];
    geo_weights<D, double>(x, w);
    for (int B = 0; B < (1 << D); ++B) W[(int64_t)B * g.NV + v] = (T)w[B];
}

template <int D, typename T>
static int coarsen_geometric_t(mgd_hier *h, OpSet &o, T *const *S, const float *eps_c0, float *scratch, hipStream_t st)
{
    o.dz_ok = 0;
    // cell values of level l in scratch, alternating between two halves
    int64_t nc1 = 1;
    for (int m = 0; m < D; ++m) nc1 *= h->nl[0] / 2;
    const float *ef = eps_c0;
    for (int l = 1; l < h->nlev; ++l) {
        int64_t ncl = 1;
        for (int m = 0; m < D; ++m) ncl *= h->nl[l];
        float *ec = scratch + ((l & 1) ? 0 : nc1);
        hipLaunchKernelGGL(k_avg_children<D>, dim3(grid_for(ncl, 256)), dim3(256), 0, st, ef, h->nl[l - 1], ec);
        hipLaunchKernelGGL((k_base_stencils<D, T>), dim3(grid_for(h->NV[l], 256)), dim3(256), 0, st,
                           (const float *)ec, h->nl[l], S[l]);
        if (h->transfer == MGD_BOXMG) {
            hipLaunchKernelGGL((k_geo_weights_t<D, T>), dim3(grid_for(h->NV[l - 1], 256)), dim3(256), 0, st,
                               h->nl[l - 1], (T *)o.W[l - 1]);
            if (D == 3) wgeo_launch<T>((const T *)o.W[l - 1], h->nl[l - 1], h->NV[l - 1], o.wgeo[l - 1], st);
        }
        ef = ec;
    }
    int lc = h->nlev - 1;
    HalfRow<D, T> Ac{S[lc], h->NV[lc], (int64_t)h->nl[lc] + 1};
    hipLaunchKernelGGL((k_dense_assemble<D, T>), dim3(1), dim3(256), 0, st, Ac, h->nl[lc], h->m_coarse, o.chol);
    hipLaunchKernelGGL(k_cholesky, dim3(1), dim3(256), 0, st, o.chol, h->m_coarse);
    if (o.cinv) hipLaunchKernelGGL(k_chol_inverse, dim3(1), dim3((unsigned)kCinvMax), 0, st, o.chol, h->m_coarse, o.cinv);
    HIPCHK(h->ctx, hipGetLastError());
    return MGD_OK;
}

int coarsen_geometric(mgd_hier *h, OpSet &o, const float *eps_c0, float *scratch, hipStream_t st)
{
    if (h->precision == MGD_FP64)
        return h->dim == 2 ? coarsen_geometric_t<2, double>(h, o, o.S64, eps_c0, scratch, st)
                           : coarsen_geometric_t<3, double>(h, o, o.S64, eps_c0, scratch, st);
    return h->dim == 2 ? coarsen_geometric_t<2, float>(h, o, o.S32, eps_c0, scratch, st)
                       : coarsen_geometric_t<3, float>(h, o, o.S32, eps_c0, scratch, st);
}

int coarsen_ops(mgd_hier *h, OpSet &o, hipStream_t st)
{
    if (h->precision == MGD_FP64)
        return h->dim == 2 ? coarsen_t<2, double>(h, o, o.S64, st) : coarsen_t<3, double>(h, o, o.S64, st);
    return h->dim == 2 ? coarsen_t<2, float>(h, o, o.S32, st) : coarsen_t<3, float>(h, o, o.S32, st);
}

template <typename TI> __global__ void k_w_to_f64(const TI *in, int64_t cnt, double *out)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < cnt) out[i] = (double)in[i];
}

template <int D> __global__ void k_geo_weights_all(int n, double *W)
{
    Grid<D> g(n);
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= g.NV) return;
    int x[3] = {0, 0, 0};
    g.coords(v, x);
    double w[1 << D];
    geo_weights<D, double>(x, w);
    for (int B = 0; B < (1 << D); ++B) W[(int64_t)B * g.NV + v] = w[B];
}

int weights_f64(mgd_hier *h, const OpSet &o, int level, double *out, hipStream_t st)
{
    int64_t NV = h->NV[level];
    int64_t cnt = NV << h->dim;
    if (h->transfer == MGD_BOXMG) {
        if (h->precision == MGD_FP64)
            HIPCHK(h->ctx, hipMemcpyAsync(out, o.W[level], cnt * 8, hipMemcpyDeviceToDevice, st));
        else
            hipLaunchKernelGGL((k_w_to_f64<float>), dim3(grid_for(cnt, 256)), dim3(256), 0, st, (const float *)o.W[level], cnt, out);
    } else {
        if (h->dim == 2) hipLaunchKernelGGL(k_geo_weights_all<2>, dim3(grid_for(NV, 256)), dim3(256), 0, st, h->nl[level], out);
        else hipLaunchKernelGGL(k_geo_weights_all<3>, dim3(grid_for(NV, 256)), dim3(256), 0, st, h->nl[level], out);
    }
    HIPCHK(h->ctx, hipGetLastError());
    return MGD_OK;
}
