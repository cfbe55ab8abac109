// Additive adaFAC-x correction (paper Sec. 4.1, eq. mg:adaFAC-x) on a
// device-resident hierarchy, as a correction scheme: the right-hand side
// r_0 is restricted to every level, every level above the coarsest forms
// its update from its own residual alone,
//     e_l = S_l r_l - P~ S_{l+1} R~ r_l,   S_l = omega diag(A_l)^{-1},
// the coarsest level solves exactly, and the updates are summed through the
// prolongations, e = sum_l P_0 .. P_{l-1} e_l.
//   adaFAC-PI:  R~ = injection (the fine residual at the coarse vertex),
//               P~ = P.  All levels' updates are independent: two launches
//               over every level at once (the auxiliary term of each coarse
//               vertex, then every level's update).
//   adaFAC-Jac: P~ = (I - S_l A_l) P, R~ = P~^T (one damped Jacobi step
//               smooths the auxiliary prolongation): a few passes per level.
#include <algorithm>

#include "common.h"

namespace {

struct AdaLevel {
    int n;
    int64_t NV;
    const void *S;   // half stencils [H][NV] of this level (cycle type)
    const void *W;   // BoxMG weights [2^d][NV] toward level + 1, or null (d-linear)
    const void *r;   // this level's residual
    void *e;         // this level's update
    void *q;         // coarse levels: S_l applied to the injected finer residual
    int64_t block0;  // first block of this level in a launch over several levels
};

struct AdaArgs {
    int nlev, first, last;  // levels first .. last - 1 take part in this launch
    double omega;
    AdaLevel L[MGD_MAXLEV];
};

template <int D> __device__ inline void coords(int64_t v, int nv, int *x)
{
    x[0] = (int)(v % nv);
    const int64_t t = v / nv;
    if (D == 2) {
        x[1] = (int)t;
    } else {
        x[1] = (int)(t % nv);
        x[2] = (int)(t / nv);
    }
}

template <int D> __device__ inline bool interior(const int *x, int n)
{
    for (int m = 0; m < D; ++m)
        if (x[m] == 0 || x[m] == n) return false;
    return true;
}

// diagonal of a row: minus the sum of its couplings (own and lower slots)
template <int D, typename T> __device__ inline T diag(const T *S, int64_t NV, int nv, int64_t v)
{
    constexpr int H = n_half(D);
    T s = (T)0;
#pragma unroll
    for (int j = 0; j < H; ++j) {
        s += S[(int64_t)j * NV + v];
        s += S[(int64_t)j * NV + v - half_lin(D, j, nv)];
    }
    return -s;
}

// (A u)_v for an interior v
template <int D, typename T> __device__ inline T apply(const T *S, int64_t NV, int nv, int64_t v, const T *u)
{
    constexpr int H = n_half(D);
    T acc = (T)0, dsum = (T)0;
#pragma unroll
    for (int j = 0; j < H; ++j) {
        const int64_t lin = half_lin(D, j, nv);
        const T a = S[(int64_t)j * NV + v], b = S[(int64_t)j * NV + v - lin];
        acc += a * u[v + lin] + b * u[v - lin];
        dsum += a + b;
    }
    return acc - dsum * u[v];
}

// prolongation weight of fine vertex x toward coarse vertex X (its box corner B)
template <int D, typename T>
__device__ inline T weight(const T *W, int64_t NV, int64_t v, const int *x, const int *X)
{
    int B = 0;
    for (int m = 0; m < D; ++m) {
        const int b = X[m] - (x[m] >> 1);
        if (b < 0 || b > 1) return (T)0;
        B |= b << m;
    }
    if (W) return W[(int64_t)B * NV + v];
    T p = (T)1;
    for (int m = 0; m < D; ++m) {
        const int dd = x[m] - 2 * X[m];
        p *= dd == 0 ? (T)1 : (dd == 1 || dd == -1) ? (T)0.5 : (T)0;
    }
    return p;
}

__device__ inline int level_of(const AdaArgs &a, int64_t b)
{
    int l = a.first;
    while (l + 1 < a.last && b >= a.L[l + 1].block0) ++l;
    return l;
}

// adaFAC-PI, auxiliary term: q_c[V] = omega r_{c-1}[2V] / D_c[V] on every
// coarse level c (first = 1)
template <int D, typename T> __global__ __launch_bounds__(256) void k_ada_q(AdaArgs a)
{
    const int c = level_of(a, blockIdx.x);
    const AdaLevel &lc = a.L[c], &lf = a.L[c - 1];
    const int64_t V = (int64_t)(blockIdx.x - lc.block0) * blockDim.x + threadIdx.x;
    if (V >= lc.NV) return;
    const int nvc = lc.n + 1, nvf = lf.n + 1;
    int X[3] = {0, 0, 0};
    coords<D>(V, nvc, X);
    T q = (T)0;
    if (interior<D>(X, lc.n)) {
        const int64_t vf = D == 2 ? 2 * X[0] + (int64_t)nvf * 2 * X[1]
                                  : 2 * X[0] + (int64_t)nvf * (2 * X[1] + (int64_t)nvf * 2 * X[2]);
        q = (T)a.omega * ((const T *)lf.r)[vf] / diag<D, T>((const T *)lc.S, lc.NV, nvc, V);
    }
    ((T *)lc.q)[V] = q;
}

// adaFAC-PI, level updates: e_l = omega r_l / D_l - P q_{l+1} on every level
// above the coarsest (first = 0)
template <int D, typename T> __global__ __launch_bounds__(256) void k_ada_e(AdaArgs a)
{
    const int l = level_of(a, blockIdx.x);
    const AdaLevel &lv = a.L[l], &lc = a.L[l + 1];
    const int64_t v = (int64_t)(blockIdx.x - lv.block0) * blockDim.x + threadIdx.x;
    if (v >= lv.NV) return;
    const int nv = lv.n + 1, nvc = lc.n + 1;
    int x[3] = {0, 0, 0};
    coords<D>(v, nv, x);
    T e = (T)0;
    if (interior<D>(x, lv.n)) {
        e = (T)a.omega * ((const T *)lv.r)[v] / diag<D, T>((const T *)lv.S, lv.NV, nv, v);
        T s = (T)0;
        for (int B = 0; B < (1 << D); ++B) {
            int X[3] = {0, 0, 0};
            bool ok = true;
            for (int m = 0; m < D; ++m) {
                X[m] = (x[m] >> 1) + ((B >> m) & 1);
                if (X[m] > lc.n) ok = false;
            }
            if (!ok) continue;
            const T w = weight<D, T>((const T *)lv.W, lv.NV, v, x, X);
            if (w == (T)0) continue;
            const int64_t V = D == 2 ? X[0] + (int64_t)nvc * X[1] : X[0] + (int64_t)nvc * (X[1] + (int64_t)nvc * X[2]);
            s += w * -((const T *)lc.q)[V];
        }
        e += s;
    }
    ((T *)lv.e)[v] = e;
}

// y = omega x / D on one level's interior (0 elsewhere)
template <int D, typename T>
__global__ __launch_bounds__(256) void k_ada_scale(const T *S, int n, const T *xin, T *y, double omega)
{
    const int nv = n + 1;
    int64_t NV = 1;
    for (int m = 0; m < D; ++m) NV *= nv;
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= NV) return;
    int x[3] = {0, 0, 0};
    coords<D>(v, nv, x);
    y[v] = interior<D>(x, n) ? (T)omega * xin[v] / diag<D, T>(S, NV, nv, v) : (T)0;
}

// adaFAC-Jac, level update: e = y - (t - omega D^{-1} A t), t = P a
template <int D, typename T>
__global__ __launch_bounds__(256) void k_ada_jac_fin(const T *S, int n, const T *t, T *e, double omega)
{
    const int nv = n + 1;
    int64_t NV = 1;
    for (int m = 0; m < D; ++m) NV *= nv;
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= NV) return;
    int x[3] = {0, 0, 0};
    coords<D>(v, nv, x);
    if (!interior<D>(x, n)) {
        e[v] = (T)0;
        return;
    }
    const T At = apply<D, T>(S, NV, nv, v, t);
    e[v] = e[v] - (t[v] - (T)omega * At / diag<D, T>(S, NV, nv, v));
}

template <typename T> __global__ void k_ada_fill(T *a, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = (T)0;
}

// coarsest level: e = A^{-1} r on its interior (FP64: the precomputed inverse,
// or forward and backward substitution with the Cholesky factor)
template <int D, typename T>
__global__ __launch_bounds__(1024) void k_ada_coarse(int n, const T *r, T *e, const double *chol, const double *cinv,
                                                     int m)
{
    extern __shared__ double work[];
    const int nv = n + 1, nin = n - 1;
    int NV = 1;
    for (int k = 0; k < D; ++k) NV *= nv;
    auto vof = [&](int k) {
        int v = 0, st = 1, t = k;
        for (int mm = 0; mm < D; ++mm) {
            v += (1 + t % nin) * st;
            t /= nin;
            st *= nv;
        }
        return v;
    };
    for (int k = threadIdx.x; k < m; k += (int)blockDim.x) work[k] = (double)r[vof(k)];
    for (int v = threadIdx.x; v < NV; v += (int)blockDim.x) e[v] = (T)0;
    __syncthreads();
    if (cinv) {
        for (int i = threadIdx.x; i < m; i += (int)blockDim.x) {
            double s = 0.0;
            for (int k = 0; k < m; ++k) s += cinv[(int64_t)i * m + k] * work[k];
            e[vof(i)] = (T)s;
        }
        return;
    }
    for (int i = 0; i < m; ++i) {  // L y = b
        const double yi = work[i] / chol[(int64_t)i * m + i];
        __syncthreads();
        if (threadIdx.x == 0) work[i] = yi;
        for (int k = i + 1 + threadIdx.x; k < m; k += (int)blockDim.x) work[k] -= chol[(int64_t)k * m + i] * yi;
        __syncthreads();
    }
    for (int i = m - 1; i >= 0; --i) {  // L^T x = y
        const double xi = work[i] / chol[(int64_t)i * m + i];
        __syncthreads();
        if (threadIdx.x == 0) work[i] = xi;
        for (int k = threadIdx.x; k < i; k += (int)blockDim.x) work[k] -= chol[(int64_t)i * m + k] * xi;
        __syncthreads();
    }
    for (int k = threadIdx.x; k < m; k += (int)blockDim.x) e[vof(k)] = (T)work[k];
}

template <int D, typename T>
int adafac_t(mgd_hier *h, const OpSet &o, const void *rhs, double omega, int variant, void **result, hipStream_t st)
{
    const int L = h->nlev;
    AdaArgs a;
    memset(&a, 0, sizeof(a));
    a.nlev = L;
    a.omega = omega;
    for (int l = 0; l < L; ++l) {
        AdaLevel &lv = a.L[l];
        lv.n = h->nl[l];
        lv.NV = h->NV[l];
        lv.S = h->precision == MGD_FP64 ? (const void *)o.S64[l] : (const void *)o.S32[l];
        lv.W = (h->transfer == MGD_BOXMG && l + 1 < L) ? o.W[l] : nullptr;
        lv.r = l == 0 ? rhs : h->r[l];
        lv.e = h->u[l];
        lv.q = h->t[l];
    }
    int rc;
    // residuals of every level
    for (int l = 0; l + 1 < L; ++l)
        if ((rc = cycle_restrict(h, o, l, a.L[l].r, h->r[l + 1], st))) return rc;
    if (L > 1 && variant == 1) {
        int64_t b = 0;
        for (int c = 1; c < L; ++c) {
            a.L[c].block0 = b;
            b += grid_for(a.L[c].NV, 256);
        }
        a.first = 1;
        a.last = L;
        hipLaunchKernelGGL((k_ada_q<D, T>), dim3((unsigned)b), dim3(256), 0, st, a);
        b = 0;
        for (int l = 0; l + 1 < L; ++l) {
            a.L[l].block0 = b;
            b += grid_for(a.L[l].NV, 256);
        }
        a.first = 0;
        a.last = L - 1;
        hipLaunchKernelGGL((k_ada_e<D, T>), dim3((unsigned)b), dim3(256), 0, st, a);
        HIPCHK(h->ctx, hipGetLastError());
    } else if (L > 1) {
        for (int l = 0; l + 1 < L; ++l) {
            const AdaLevel &lv = a.L[l], &lc = a.L[l + 1];
            const T *S = (const T *)lv.S;
            T *y = (T *)lv.e, *w = (T *)h->t[l], *ac = (T *)h->f[l + 1];
            const dim3 gv(grid_for(lv.NV, 256)), gc(grid_for(lc.NV, 256));
            hipLaunchKernelGGL((k_ada_scale<D, T>), gv, dim3(256), 0, st, S, lv.n, (const T *)lv.r, y, omega);
            if ((rc = cycle_residual(h, o, l, y, lv.r, w, st))) return rc;          // w = r - A y
            if ((rc = cycle_restrict(h, o, l, w, ac, st))) return rc;              // a = R w
            hipLaunchKernelGGL((k_ada_scale<D, T>), gc, dim3(256), 0, st, (const T *)lc.S, lc.n, (const T *)ac, ac,
                               omega);                                              // a = S_{l+1} a
            hipLaunchKernelGGL((k_ada_fill<T>), gv, dim3(256), 0, st, w, lv.NV);
            if ((rc = cycle_prolong(h, o, l, ac, w, st))) return rc;                // t = P a
            hipLaunchKernelGGL((k_ada_jac_fin<D, T>), gv, dim3(256), 0, st, S, lv.n, (const T *)w, y, omega);
            HIPCHK(h->ctx, hipGetLastError());
        }
    }
    // coarsest level, exactly
    const AdaLevel &lc = a.L[L - 1];
    const int m = (int)h->m_coarse;
    const unsigned thr = (unsigned)std::min<int64_t>(1024, std::max<int64_t>(64, ((lc.NV + 63) / 64) * 64));
    hipLaunchKernelGGL((k_ada_coarse<D, T>), dim3(1), dim3(thr), (size_t)std::max(m, 1) * 8, st, lc.n,
                       (const T *)lc.r, (T *)lc.e, (const double *)o.chol, (const double *)o.cinv, m);
    HIPCHK(h->ctx, hipGetLastError());
    // e = sum of the prolonged updates, from the coarsest level up
    for (int l = L - 2; l >= 0; --l)
        if ((rc = cycle_prolong(h, o, l, h->u[l + 1], h->u[l], st))) return rc;
    *result = h->u[0];
    return MGD_OK;
}

}  // namespace

// one additive adaFAC cycle from a zero correction: *result = B rhs
// (variant 1: adaFAC-PI, 2: adaFAC-Jac), in the hierarchy's cycle type
int adafac_ops(mgd_hier *h, const OpSet &o, const void *rhs, double omega, int variant, void **result,
               hipStream_t st)
{
    if (variant != 1 && variant != 2) return mgd_fail(h->ctx, MGD_EINVAL, "adaFAC variant %d", variant);
    if (h->m_coarse > 1500) return mgd_fail(h->ctx, MGD_EINVAL, "coarsest level too large");
    if (h->precision == MGD_FP64)
        return h->dim == 2 ? adafac_t<2, double>(h, o, rhs, omega, variant, result, st)
                           : adafac_t<3, double>(h, o, rhs, omega, variant, result, st);
    return h->dim == 2 ? adafac_t<2, float>(h, o, rhs, omega, variant, result, st)
                       : adafac_t<3, float>(h, o, rhs, omega, variant, result, st);
}
