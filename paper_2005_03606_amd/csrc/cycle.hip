// Multigrid cycle kernels (paper Sec. 4 and 4.1): damped Jacobi
// u <- u + omega D^{-1} (f - A u), residual, restriction R = P^T,
// prolongation, on any operator view: FP64 / FP32 half stencils or the
// compressed surplus store decoded on the fly; plus the FP64 outer residual
// and the vector kernels of the outer iteration, with deterministic
// (fixed-order) reductions.
#include "common.h"

// ------------------------------------------------------------ operator views
template <typename T> struct OpHalf {
    const T *S;
    int64_t NV;
    __device__ inline T c(int64_t v, int j, const int *) const { return S[(int64_t)j * NV + v]; }
};

// compressed fine store: base from the centre samples (in T) + decoded delta
template <int D, typename T> struct OpComp {
    StoreView sv;
    int n;
    T hp;
    __device__ inline T c(int64_t v, int j, const int *x) const
    {
        // x: coordinates of v
        int o[3] = {half_off(D, j, 0), half_off(D, j, 1), D == 3 ? half_off(D, j, 2) : 0};
        int nz = (o[0] != 0) + (o[1] != 0) + (o[2] != 0);
        T base = (T)0;
        if (!(D == 3 && nz == 1)) {
            T sum = (T)0;
            for (int B = (1 << D) - 1; B >= 0; --B) {
                bool ok = true;
                int64_t cc = 0, stride = 1;
                for (int m = 0; m < D; ++m) {
                    int bm = (B >> m) & 1, cm = x[m] - bm, wm = bm + o[m];
                    if (cm < 0 || cm >= n || wm < 0 || wm > 1) ok = false;
                    cc += (int64_t)cm * stride;
                    stride *= n;
                }
                if (ok) sum += (T)sv.eps_c[cc];
            }
            base = sum * (T)kref_unit(D, nz) * hp;
        }
        return base + (T)sv.delta(v, j, n_half(D));
    }
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
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
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

// fc[X] = sum_v P[v][X] r[v] over the 3^d fine vertices around 2X (interior X)
template <int D, typename T>
__global__ void k_restrict(const T *W, int nf, const T *r, T *fc)
{
    Grid<D> gf(nf), gc(nf / 2);
    int64_t V = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (V >= gc.NV) return;
    int X[3] = {0, 0, 0};
    gc.coords(V, X);
    if (!gc.interior(X)) { fc[V] = (T)0; return; }
    T s = (T)0;
    constexpr int ns = D == 2 ? 9 : 27;
    for (int sv = 0; sv < ns; ++sv) {
        int x[3] = {0, 0, 0}, t = sv;
        for (int m = 0; m < D; ++m) { x[m] = 2 * X[m] + t % 3 - 1; t /= 3; }
        int64_t v = gf.vid(x);
        s += wt<D, T, T>(W, gf.NV, v, x, X) * r[v];
    }
    fc[V] = s;
}

// u[v] += sum_B P[v][corner B] e[corner B] (interior fine v)
template <int D, typename T>
__global__ void k_prolong(const T *W, int nf, const T *ec, T *u)
{
    Grid<D> gf(nf), gc(nf / 2);
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= gf.NV) return;
    int x[3] = {0, 0, 0};
    gf.coords(v, x);
    if (!gf.interior(x)) return;
    T s = (T)0;
    for (int B = 0; B < (1 << D); ++B) {
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

template <typename T> __global__ void k_fill(T *a, int64_t n, T val)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = val;
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
    int n;
    const void *u;     // iterate (SWEEP/RESID: float; OUTER: double) / z (PMATVEC: float)
    const void *f;     // rhs (float / double)
    void *out;         // float / double
    const double *pold;
    double *pnew;
    const double *s;   // device scalars (beta at s[5])
    double *partial;
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
    const int x0 = blockIdx.x * BX, y0 = blockIdx.y * BY;
    const int tid = threadIdx.x;
    // centre samples of cells x in [x0-2, x0+64], y in [y0-2, y0+3]
    for (int k = tid; k < (BY + 2) * (BX + 3); k += 256) {
        int cx = x0 - 2 + k % (BX + 3), cy = y0 - 2 + k / (BX + 3);
        s_eps[k / (BX + 3)][k % (BX + 3)] = (cx >= 0 && cx < n && cy >= 0 && cy < n) ? a.sv.eps_c[(int64_t)cy * n + cx] : 0.0f;
    }
    // iterate with a one-vertex halo
    double beta = KIND == ST_PMATVEC ? a.s[5] : 0.0;
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
            TC e00 = (TC)s_eps[ly][lx], e10 = (TC)s_eps[ly][lx + 1];       // (vx-1, vy-1), (vx, vy-1)
            TC e01 = (TC)s_eps[ly + 1][lx], e11 = (TC)s_eps[ly + 1][lx + 1]; // (vx-1, vy), (vx, vy)
            const TC k6 = (TC)(-1.0 / 6.0), k3 = (TC)(-1.0 / 3.0);
            TC base[4] = {(e10 + e11) * k6, e01 * k3, (e01 + e11) * k6, e11 * k3};
            int64_t t = v >> 6;
            int tt = a.sv.tier[t];
            if (tt == 0) {
                for (int j = 0; j < 4; ++j) c[j] = base[j];
            } else {
                const uint8_t *bp = a.sv.payload + (size_t)a.sv.off[t] * 64;
                int l = (int)(v & 63);
                float sc = e8m0_to_float(bp[l]);
                for (int j = 0; j < 4; ++j) {
                    float d;
                    if (tt == 2) d = (float)__builtin_bit_cast(_Float16, ((const uint16_t *)(bp + 64 + j * 128))[l]) * sc;
                    else if (tt == 1) d = e4m3_to_float(bp[64 + j * 64 + l]) * sc;
                    else d = ((const float *)(bp + 64 + j * 256))[l];
                    c[j] = base[j] + (TC)d;
                }
            }
        }
        for (int j = 0; j < 4; ++j) s_c[j][ly][lx] = c[j];
    }
    __syncthreads();
    const int tx = tid & 63, ty = tid >> 6;
    const int vx = x0 + tx, vy = y0 + ty;
    double part = 0.0;
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
            part = r * r;
        } else {  // PMATVEC
            a.pnew[v] = (double)uc;
            double ap = inner ? (double)Au : 0.0;
            ((double *)a.out)[v] = ap;
            part = (double)uc * ap;
        }
    }
    if (KIND == ST_OUTER || KIND == ST_PMATVEC) {
        double sum = block_sum<256>(part, red);
        if (tid == 0) a.partial[blockIdx.y * gridDim.x + blockIdx.x] = sum;
    }
}

static inline dim3 stage2_grid(int n) { return dim3((unsigned)((n + 1 + 63) / 64), (unsigned)((n + 1 + 3) / 4)); }

// ------------------------------------------------------------ dispatch
int store_set_base(mgd_hier *h, OpSet &o, const float *eps_c, hipStream_t st);
StoreView store_view(const mgd_hier *h, const OpSet &o);

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
        dim3 g2 = stage2_grid(n);
        if (mode == 1) hipLaunchKernelGGL((k_stage2<float, ST_RESID>), g2, dim3(256), 0, st, sa);
        else if (zero_guess) hipLaunchKernelGGL((k_stage2<float, ST_SWEEP0>), g2, dim3(256), 0, st, sa);
        else hipLaunchKernelGGL((k_stage2<float, ST_SWEEP>), g2, dim3(256), 0, st, sa);
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
    else if (level > 0) go(OpHalf<float>{o.S32[level], h->NV[level]});
    else go(OpComp<D, float>{store_view(h, o), h->n, (float)(D == 2 ? 1.0 : 1.0 / h->n)});
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

int cycle_smooth(mgd_hier *h, const OpSet &o, int level, void *u, const void *f, void *tmp, int sweeps,
                 double omega, bool zero_guess, hipStream_t st)
{
    // ping-pong u -> tmp -> u; an odd count ends with a copy back
    for (int k = 0; k < sweeps; ++k) {
        const void *src = (k % 2 == 0) ? u : tmp;
        void *dst = (k % 2 == 0) ? tmp : u;
        int rc = sweep(h, o, level, src, f, dst, omega, 0, zero_guess && k == 0, nullptr, st);
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
        if (h->dim == 2) hipLaunchKernelGGL((k_restrict<2, double>), gr, dim3(256), 0, st, W, nf, (const double *)r, (double *)fc);
        else hipLaunchKernelGGL((k_restrict<3, double>), gr, dim3(256), 0, st, W, nf, (const double *)r, (double *)fc);
    } else {
        const float *W = box ? (const float *)o.W[level] : nullptr;
        if (h->dim == 2) hipLaunchKernelGGL((k_restrict<2, float>), gr, dim3(256), 0, st, W, nf, (const float *)r, (float *)fc);
        else hipLaunchKernelGGL((k_restrict<3, float>), gr, dim3(256), 0, st, W, nf, (const float *)r, (float *)fc);
    }
    HIPCHK(h->ctx, hipGetLastError());
    return MGD_OK;
}

int cycle_prolong(mgd_hier *h, const OpSet &o, int level, const void *ec, void *u, hipStream_t st)
{
    int nf = h->nl[level];
    dim3 gr(grid_for(h->NV[level], 256));
    bool box = h->transfer == MGD_BOXMG;
    if (h->precision == MGD_FP64) {
        const double *W = box ? (const double *)o.W[level] : nullptr;
        if (h->dim == 2) hipLaunchKernelGGL((k_prolong<2, double>), gr, dim3(256), 0, st, W, nf, (const double *)ec, (double *)u);
        else hipLaunchKernelGGL((k_prolong<3, double>), gr, dim3(256), 0, st, W, nf, (const double *)ec, (double *)u);
    } else {
        const float *W = box ? (const float *)o.W[level] : nullptr;
        if (h->dim == 2) hipLaunchKernelGGL((k_prolong<2, float>), gr, dim3(256), 0, st, W, nf, (const float *)ec, (float *)u);
        else hipLaunchKernelGGL((k_prolong<3, float>), gr, dim3(256), 0, st, W, nf, (const float *)ec, (float *)u);
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
// a given u) down to the dense coarsest solve and back up, in one workgroup:
// each step is a strided loop over the level's vertices, steps separated by
// workgroup barriers (global writes of the workgroup are visible after them).
struct TailLevel {
    const void *S, *W;
    void *u, *f, *r, *t;
    int n;
    int64_t NV;
};
struct TailArgs {
    int first, last, nu1, nu2, zero_guess;
    double omega;
    const double *chol;
    int64_t m;
    double *work;
    TailLevel L[MGD_MAXLEV];
};

template <int D, typename T>
__device__ void tail_sweep(const TailLevel &lv, const T *u, T *out, bool zero, T omega)
{
    OpHalf<T> A{(const T *)lv.S, lv.NV};
    Grid<D> g(lv.n);
    const T *f = (const T *)lv.f;
    for (int64_t v = threadIdx.x; v < g.NV; v += blockDim.x) {
        int x[3] = {0, 0, 0};
        g.coords(v, x);
        if (!g.interior(x)) { out[v] = (T)0; continue; }
        T Au, Dv;
        if (zero) {
            constexpr int H = n_half(D);
            T dsum = (T)0;
            for (int j = 0; j < H; ++j) {
                int64_t lin = half_lin(D, j, g.nv);
                dsum += A.c(v, j, x) + A.c(v - lin, j, x);
            }
            Dv = -dsum;
            Au = (T)0;
        } else {
            apply_row<D, OpHalf<T>, T>(A, g, v, x, u, Au, Dv);
        }
        out[v] = (zero ? (T)0 : u[v]) + omega * (f[v] - Au) / Dv;
    }
    __syncthreads();
}

template <int D, typename T> __device__ void tail_smooth(const TailLevel &lv, int sweeps, bool zero, T omega)
{
    T *u = (T *)lv.u, *t = (T *)lv.t;
    for (int k = 0; k < sweeps; ++k) {
        if (k % 2 == 0) tail_sweep<D, T>(lv, u, t, zero && k == 0, omega);
        else tail_sweep<D, T>(lv, t, u, false, omega);
    }
    if (sweeps % 2 == 1) {
        for (int64_t v = threadIdx.x; v < lv.NV; v += blockDim.x) u[v] = t[v];
        __syncthreads();
    }
    if (sweeps == 0 && zero) {
        for (int64_t v = threadIdx.x; v < lv.NV; v += blockDim.x) u[v] = (T)0;
        __syncthreads();
    }
}

template <int D, typename T> __device__ void tail_residual_restrict(const TailLevel &lv, const TailLevel &lc)
{
    OpHalf<T> A{(const T *)lv.S, lv.NV};
    Grid<D> g(lv.n), gc(lc.n);
    const T *u = (const T *)lv.u, *f = (const T *)lv.f;
    T *r = (T *)lv.r;
    for (int64_t v = threadIdx.x; v < g.NV; v += blockDim.x) {
        int x[3] = {0, 0, 0};
        g.coords(v, x);
        if (!g.interior(x)) { r[v] = (T)0; continue; }
        T Au, Dv;
        apply_row<D, OpHalf<T>, T>(A, g, v, x, u, Au, Dv);
        r[v] = f[v] - Au;
    }
    __syncthreads();
    const T *W = (const T *)lv.W;
    T *fc = (T *)lc.f, *uc = (T *)lc.u;
    constexpr int ns = D == 2 ? 9 : 27;
    for (int64_t V = threadIdx.x; V < gc.NV; V += blockDim.x) {
        int X[3] = {0, 0, 0};
        gc.coords(V, X);
        uc[V] = (T)0;
        if (!gc.interior(X)) { fc[V] = (T)0; continue; }
        T s = (T)0;
        for (int sv = 0; sv < ns; ++sv) {
            int x[3] = {0, 0, 0}, t = sv;
            for (int m = 0; m < D; ++m) { x[m] = 2 * X[m] + t % 3 - 1; t /= 3; }
            int64_t v = g.vid(x);
            s += wt<D, T, T>(W, g.NV, v, x, X) * r[v];
        }
        fc[V] = s;
    }
    __syncthreads();
}

template <int D, typename T> __device__ void tail_prolong(const TailLevel &lv, const TailLevel &lc)
{
    Grid<D> g(lv.n), gc(lc.n);
    const T *W = (const T *)lv.W, *ec = (const T *)lc.u;
    T *u = (T *)lv.u;
    for (int64_t v = threadIdx.x; v < g.NV; v += blockDim.x) {
        int x[3] = {0, 0, 0};
        g.coords(v, x);
        if (!g.interior(x)) continue;
        T s = (T)0;
        for (int B = 0; B < (1 << D); ++B) {
            int X[3] = {0, 0, 0};
            bool ok = true;
            for (int m = 0; m < D; ++m) {
                X[m] = (x[m] >> 1) + ((B >> m) & 1);
                if (X[m] > gc.n) ok = false;
            }
            if (!ok) continue;
            T w = wt<D, T, T>(W, g.NV, v, x, X);
            if (w != (T)0) s += w * ec[gc.vid(X)];
        }
        u[v] += s;
    }
    __syncthreads();
}

template <int BS> __device__ inline double block_sum_tail(double v, double *red)
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

// dense solve on the coarsest interior, FP64 triangular substitutions
template <int D, typename T> __device__ void tail_coarse(const TailLevel &lv, const double *L, int64_t m, double *work,
                                                         double *red)
{
    Grid<D> g(lv.n);
    const T *f = (const T *)lv.f;
    T *u = (T *)lv.u;
    for (int64_t v = threadIdx.x; v < g.NV; v += blockDim.x) {
        int x[3] = {0, 0, 0};
        g.coords(v, x);
        if (!g.interior(x)) continue;
        int64_t k = 0, st = 1;
        for (int mm = 0; mm < D; ++mm) { k += (int64_t)(x[mm] - 1) * st; st *= (lv.n - 1); }
        work[k] = (double)f[v];
    }
    __syncthreads();
    for (int64_t i = 0; i < m; ++i) {
        double s = 0.0;
        for (int64_t k = threadIdx.x; k < i; k += blockDim.x) s += L[i * m + k] * work[k];
        s = block_sum_tail<1024>(s, red);
        if (threadIdx.x == 0) work[i] = (work[i] - s) / L[i * m + i];
        __syncthreads();
    }
    for (int64_t i = m - 1; i >= 0; --i) {
        double s = 0.0;
        for (int64_t k = i + 1 + threadIdx.x; k < m; k += blockDim.x) s += L[k * m + i] * work[k];
        s = block_sum_tail<1024>(s, red);
        if (threadIdx.x == 0) work[i] = (work[i] - s) / L[i * m + i];
        __syncthreads();
    }
    for (int64_t v = threadIdx.x; v < g.NV; v += blockDim.x) {
        int x[3] = {0, 0, 0};
        g.coords(v, x);
        T val = (T)0;
        if (g.interior(x)) {
            int64_t k = 0, st = 1;
            for (int mm = 0; mm < D; ++mm) { k += (int64_t)(x[mm] - 1) * st; st *= (lv.n - 1); }
            val = (T)work[k];
        }
        u[v] = val;
    }
    __syncthreads();
}

template <int D, typename T> __global__ __launch_bounds__(1024) void k_tail(TailArgs a)
{
    __shared__ double red[1024];
    T omega = (T)a.omega;
    for (int l = a.first; l < a.last; ++l) {
        bool zero = l > a.first || a.zero_guess;
        tail_smooth<D, T>(a.L[l], a.nu1, zero, omega);
        tail_residual_restrict<D, T>(a.L[l], a.L[l + 1]);
    }
    tail_coarse<D, T>(a.L[a.last], a.chol, a.m, a.work, red);
    for (int l = a.last - 1; l >= a.first; --l) {
        tail_prolong<D, T>(a.L[l], a.L[l + 1]);
        tail_smooth<D, T>(a.L[l], a.nu2, false, omega);
    }
}

// first level handled by the tail kernel (levels with few vertices)
static int tail_first(const mgd_hier *h)
{
    const int64_t kTailNV = 5000;
    int l = h->nlev - 1;
    while (l > 0 && h->NV[l - 1] <= kTailNV) --l;
    if (h->precision == MGD_MIXED && l == 0) l = h->nlev > 1 ? 1 : 0;  // level 0 is the compressed store
    return l;
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
    a.chol = o.chol;
    a.m = h->m_coarse;
    a.work = h->partial;
    for (int l = first; l <= a.last; ++l) {
        TailLevel &L = a.L[l];
        L.S = h->precision == MGD_FP64 ? (const void *)o.S64[l] : (const void *)o.S32[l];
        L.W = h->transfer == MGD_BOXMG ? o.W[l] : nullptr;
        L.u = l == first ? u : h->u[l];
        L.f = l == first ? const_cast<void *>(f) : h->f[l];
        L.r = h->r[l];
        L.t = h->t[l];
        L.n = h->nl[l];
        L.NV = h->NV[l];
    }
    if (h->precision == MGD_FP64) {
        if (h->dim == 2) hipLaunchKernelGGL((k_tail<2, double>), dim3(1), dim3(1024), 0, st, a);
        else hipLaunchKernelGGL((k_tail<3, double>), dim3(1), dim3(1024), 0, st, a);
    } else {
        if (h->dim == 2) hipLaunchKernelGGL((k_tail<2, float>), dim3(1), dim3(1024), 0, st, a);
        else hipLaunchKernelGGL((k_tail<3, float>), dim3(1), dim3(1024), 0, st, a);
    }
    HIPCHK(h->ctx, hipGetLastError());
    return MGD_OK;
}

// multiplicative V(nu1,nu2) correction scheme from level l down
static int vcycle_rec(mgd_hier *h, const OpSet &o, int l, void *u, const void *f, double omega, int nu1, int nu2,
                      bool zero_guess, hipStream_t st)
{
    int rc;
    if (l == tail_first(h)) return launch_tail(h, o, l, u, f, omega, nu1, nu2, zero_guess, st);
    if (nu1 > 0) {
        if ((rc = cycle_smooth(h, o, l, u, f, h->t[l], nu1, omega, zero_guess, st))) return rc;
    } else if (zero_guess) {
        if ((rc = fill_zero(h, u, h->NV[l], st))) return rc;
    }
    if ((rc = cycle_residual(h, o, l, u, f, h->r[l], st))) return rc;
    if ((rc = cycle_restrict(h, o, l, h->r[l], h->f[l + 1], st))) return rc;
    if ((rc = vcycle_rec(h, o, l + 1, h->u[l + 1], h->f[l + 1], omega, nu1, nu2, true, st))) return rc;
    if ((rc = cycle_prolong(h, o, l, h->u[l + 1], u, st))) return rc;
    if (nu2 > 0)
        if ((rc = cycle_smooth(h, o, l, u, f, h->t[l], nu2, omega, false, st))) return rc;
    return MGD_OK;
}

int vcycle_ops(mgd_hier *h, const OpSet &o, void *u, const void *f, double omega, int nu1, int nu2, bool zero_guess,
               hipStream_t st)
{
    return vcycle_rec(h, o, 0, u, f, omega, nu1, nu2, zero_guess, st);
}

// ------------------------------------------------------------ FP64 outer
template <int D> struct OpComp64 {
    StoreView sv;
    int n;
    __device__ inline double c(int64_t v, int j, const int *x) const
    {
#pragma clang fp contract(off)
        return base_coupling64<D>(sv.eps_c, n, x, j, nullptr) + (double)sv.delta(v, j, n_half(D));
    }
};

template <int D, class Op>
__global__ __launch_bounds__(256) void k_outer_residual(Op A, int n, const double *u, const double *f, double *r,
                                                        double *partial, float *rf)
{
    __shared__ double red[256];
    Grid<D> g(n);
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double rr = 0.0;
    if (v < g.NV) {
        int x[3] = {0, 0, 0};
        g.coords(v, x);
        double rv = 0.0;
        if (g.interior(x)) {
            double Au, Dv;
            apply_row<D, Op, double>(A, g, v, x, u, Au, Dv);
            rv = f[v] - Au;
            rr = rv * rv;
        }
        r[v] = rv;
        if (rf) rf[v] = (float)rv;
    }
    double s = block_sum<256>(rr, red);
    if (threadIdx.x == 0 && partial) partial[blockIdx.x] = s;
}

// out[k] = sum of partial[k*stride .. k*stride+cnt), fixed order, one block;
// post 1: CG beta from the scalars (see k_beta), post 2: CG alpha
enum { RED_PLAIN = 0, RED_BETA = 1, RED_ALPHA = 2 };
__global__ void k_reduce(const double *partial, int64_t cnt, int nvec, int64_t stride, double *out, double *sc,
                         int post)
{
    __shared__ double red[1024];
    for (int k = 0; k < nvec; ++k) {
        double s = 0.0;
        for (int64_t i = threadIdx.x; i < cnt; i += 1024) s += partial[k * stride + i];
        double t = block_sum<1024>(s, red);
        if (threadIdx.x == 0) out[k] = t;
    }
    if (threadIdx.x == 0 && post == RED_BETA) {
        // sc: [0] zr_old, [1] zr, [2] zdr, [3] pAp, [4] rr, [5] beta, [6] alpha, [7] restart
        sc[5] = sc[7] != 0.0 ? 0.0 : sc[2] / sc[0];
        sc[0] = sc[1];
        sc[7] = 0.0;
    }
    if (threadIdx.x == 0 && post == RED_ALPHA) sc[6] = sc[1] / sc[3];
}

template <int D>
static int outer_residual_t(mgd_hier *h, const OpSet &o, const double *u, const double *f, double *r,
                            double *partial, hipStream_t st)
{
    dim3 gr(grid_for(h->NV[0], 256));
    if (h->precision == MGD_FP64)
        hipLaunchKernelGGL((k_outer_residual<D, OpHalf<double>>), gr, dim3(256), 0, st,
                           OpHalf<double>{o.S64[0], h->NV[0]}, h->n, u, f, r, partial, (float *)nullptr);
    else
        hipLaunchKernelGGL((k_outer_residual<D, OpComp64<D>>), gr, dim3(256), 0, st,
                           OpComp64<D>{store_view(h, o), h->n}, h->n, u, f, r, partial, (float *)h->f[0]);
    HIPCHK(h->ctx, hipGetLastError());
    return MGD_OK;
}

// r = f - A u (finest operator as stored, FP64); if norm2_dev: ||r||^2 there
int outer_residual(mgd_hier *h, const OpSet &o, const double *u, const double *f, double *r, double *norm2_dev,
                   hipStream_t st)
{
    if (h->dim == 2 && h->precision == MGD_MIXED) {
        StageArgs<double> sa;
        memset(&sa, 0, sizeof(sa));
        sa.sv = store_view(h, o);
        sa.n = h->n;
        sa.u = u;
        sa.f = f;
        sa.out = r;
        sa.partial = h->partial;
        sa.rf = (float *)h->f[0];
        dim3 g2 = stage2_grid(h->n);
        hipLaunchKernelGGL((k_stage2<double, ST_OUTER>), g2, dim3(256), 0, st, sa);
        if (norm2_dev) {
            int64_t nb = (int64_t)g2.x * g2.y;
            hipLaunchKernelGGL(k_reduce, dim3(1), dim3(1024), 0, st, (const double *)h->partial, nb, 1, nb, norm2_dev, nullptr, 0);
        }
        HIPCHK(h->ctx, hipGetLastError());
        return MGD_OK;
    }
    double *partial = norm2_dev ? h->partial : nullptr;
    int rc = h->dim == 2 ? outer_residual_t<2>(h, o, u, f, r, partial, st) : outer_residual_t<3>(h, o, u, f, r, partial, st);
    if (rc) return rc;
    if (norm2_dev) {
        int64_t nb = grid_for(h->NV[0], 256);
        hipLaunchKernelGGL(k_reduce, dim3(1), dim3(1024), 0, st, (const double *)h->partial, nb, 1, nb, norm2_dev, nullptr, 0);
        HIPCHK(h->ctx, hipGetLastError());
    }
    return MGD_OK;
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

// partials of z.r and z.(r - r_old)
template <typename T>
__global__ __launch_bounds__(256) void k_dots_zr(const T *z, const double *r, const double *rold, int64_t n,
                                                 double *partial, int64_t nb)
{
    __shared__ double red[256];
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double a = 0.0, b = 0.0;
    if (i < n) {
        double zz = (double)z[i];
        a = zz * r[i];
        b = zz * (r[i] - rold[i]);
    }
    double sa = block_sum<256>(a, red), sb = block_sum<256>(b, red);
    if (threadIdx.x == 0) { partial[blockIdx.x] = sa; partial[nb + blockIdx.x] = sb; }
}


// p_new = z + beta p_old on every vertex; Ap = A p_new on the interior,
// with partials of p_new . Ap
template <int D, class Op, typename TZ>
__global__ __launch_bounds__(256) void k_p_matvec(Op A, int n, const TZ *z, const double *pold, double *pnew,
                                                  double *Ap, const double *s, double *partial)
{
    __shared__ double red[256];
    Grid<D> g(n);
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double beta = s[5], prod = 0.0;
    if (v < g.NV) {
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
            prod = pv * apv;
        } else {
            Ap[v] = 0.0;
        }
    }
    double sum = block_sum<256>(prod, red);
    if (threadIdx.x == 0) partial[blockIdx.x] = sum;
}

// x += alpha p; r_old = r; r -= alpha Ap; partials of r.r
__global__ __launch_bounds__(256) void k_cg_update(double *x, const double *p, double *r, double *rold,
                                                   const double *Ap, int64_t n, const double *s, double *partial,
                                                   float *rf)
{
    __shared__ double red[256];
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double alpha = s[6], rr = 0.0;
    if (i < n) {
        x[i] += alpha * p[i];
        double ri = r[i];
        rold[i] = ri;
        ri -= alpha * Ap[i];
        r[i] = ri;
        if (rf) rf[i] = (float)ri;
        rr = ri * ri;
    }
    double sum = block_sum<256>(rr, red);
    if (threadIdx.x == 0) partial[blockIdx.x] = sum;
}

struct PcgBufs {
    double *r, *rold, *p0, *p1, *Ap;
};

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

// z.r, z.(r - r_old) -> s[1], s[2]; then beta
int pcg_beta(mgd_hier *h, const void *z, const double *r, const double *rold, double *s, hipStream_t st)
{
    int64_t n = h->NV[0], nb = grid_for(n, 256);
    double *part = h->partial;
    if (h->precision == MGD_FP64) hipLaunchKernelGGL(k_dots_zr<double>, dim3(nb), dim3(256), 0, st, (const double *)z, r, rold, n, part, nb);
    else hipLaunchKernelGGL(k_dots_zr<float>, dim3(nb), dim3(256), 0, st, (const float *)z, r, rold, n, part, nb);
    hipLaunchKernelGGL(k_reduce, dim3(1), dim3(1024), 0, st, (const double *)part, nb, 2, nb, s + 1, s, (int)RED_BETA);
    HIPCHK(h->ctx, hipGetLastError());
    return MGD_OK;
}

template <int D, typename TZ>
static int pcg_matvec_t(mgd_hier *h, const OpSet &o, const TZ *z, const double *pold, double *pnew, double *Ap,
                        double *s, hipStream_t st)
{
    int64_t n = h->NV[0], nb = grid_for(n, 256);
    double *part = h->partial;
    if (h->precision == MGD_FP64)
        hipLaunchKernelGGL((k_p_matvec<D, OpHalf<double>, TZ>), dim3(nb), dim3(256), 0, st,
                           OpHalf<double>{o.S64[0], h->NV[0]}, h->n, z, pold, pnew, Ap, (const double *)s, part);
    else
        hipLaunchKernelGGL((k_p_matvec<D, OpComp64<D>, TZ>), dim3(nb), dim3(256), 0, st,
                           OpComp64<D>{store_view(h, o), h->n}, h->n, z, pold, pnew, Ap, (const double *)s, part);
    hipLaunchKernelGGL(k_reduce, dim3(1), dim3(1024), 0, st, (const double *)part, nb, 1, nb, s + 3, s, (int)RED_ALPHA);
    HIPCHK(h->ctx, hipGetLastError());
    return MGD_OK;
}

int pcg_matvec(mgd_hier *h, const OpSet &o, const void *z, const double *pold, double *pnew, double *Ap, double *s,
               hipStream_t st)
{
    if (h->dim == 2 && h->precision == MGD_MIXED) {
        StageArgs<double> sa;
        memset(&sa, 0, sizeof(sa));
        sa.sv = store_view(h, o);
        sa.n = h->n;
        sa.u = z;
        sa.pold = pold;
        sa.pnew = pnew;
        sa.out = Ap;
        sa.s = s;
        sa.partial = h->partial;
        dim3 g2 = stage2_grid(h->n);
        int64_t nb = (int64_t)g2.x * g2.y;
        hipLaunchKernelGGL((k_stage2<double, ST_PMATVEC>), g2, dim3(256), 0, st, sa);
        hipLaunchKernelGGL(k_reduce, dim3(1), dim3(1024), 0, st, (const double *)h->partial, nb, 1, nb, s + 3, s, (int)RED_ALPHA);
        HIPCHK(h->ctx, hipGetLastError());
        return MGD_OK;
    }
    if (h->precision == MGD_FP64)
        return h->dim == 2 ? pcg_matvec_t<2, double>(h, o, (const double *)z, pold, pnew, Ap, s, st)
                           : pcg_matvec_t<3, double>(h, o, (const double *)z, pold, pnew, Ap, s, st);
    return h->dim == 2 ? pcg_matvec_t<2, float>(h, o, (const float *)z, pold, pnew, Ap, s, st)
                       : pcg_matvec_t<3, float>(h, o, (const float *)z, pold, pnew, Ap, s, st);
}

int pcg_update(mgd_hier *h, double *x, const double *p, double *r, double *rold, const double *Ap, double *s,
               hipStream_t st)
{
    int64_t n = h->NV[0], nb = grid_for(n, 256);
    double *part = h->partial;
    float *rf = h->precision == MGD_MIXED ? (float *)h->f[0] : nullptr;
    hipLaunchKernelGGL(k_cg_update, dim3(nb), dim3(256), 0, st, x, p, r, rold, Ap, n, (const double *)s, part, rf);
    hipLaunchKernelGGL(k_reduce, dim3(1), dim3(1024), 0, st, (const double *)part, nb, 1, nb, s + 4, nullptr, 0);
    HIPCHK(h->ctx, hipGetLastError());
    return MGD_OK;
}

int vec_fill_f64(mgd_ctx *ctx, double *a, int64_t n, double v, hipStream_t st)
{
    hipLaunchKernelGGL(k_fill<double>, dim3(grid_for(n, 256)), dim3(256), 0, st, a, n, v);
    HIPCHK(ctx, hipGetLastError());
    return MGD_OK;
}
