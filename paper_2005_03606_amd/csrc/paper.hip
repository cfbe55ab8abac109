// The paper's flexible-precision format (Sec. 5.5) for the hierarchical
// surplus of element matrices, one cell per thread: the full surplus
// matrix, the byte count p3 (0: only the marker, 2..7: truncated, 8: the
// double) and the encoded entries.  Every step is exact integer or IEEE
// arithmetic (no contraction), so the result is the same bits as any
// correct implementation of the same definition.
#include "common.h"

// p-byte datum of x (2 <= p <= 7): p - 1 little-endian bytes with the sign
// in the top bit and the leading 8 (p - 1) - 1 fraction bits, then the
// unbiased exponent as a signed char clamped to [-128, 127]; zero has
// exponent -128 and a zero fraction
__device__ inline void p3_put(double x, int p, uint8_t *out)
{
    const uint64_t b = (uint64_t)__double_as_longlong(x);
    const int m = 8 * (p - 1) - 1;
    int e = (int)((b >> 52) & 0x7ff) - 1023;
    uint64_t frac = b & ((1ull << 52) - 1);
    if (x == 0.0) { e = -128; frac = 0; }
    e = e < -128 ? -128 : (e > 127 ? 127 : e);
    const uint64_t word = ((b >> 63) << m) | (frac >> (52 - m));
    for (int k = 0; k < p - 1; ++k) out[k] = (uint8_t)(word >> (8 * k));
    out[p - 1] = (uint8_t)(int8_t)e;
}

// the value a p-byte datum stands for
__device__ inline double p3_get(const uint8_t *in, int p)
{
    const int m = 8 * (p - 1) - 1;
    uint64_t word = 0;
    for (int k = 0; k < p - 1; ++k) word |= (uint64_t)in[k] << (8 * k);
    const int sign = (int)(word >> m) & 1;
    const uint64_t mt = word & ((1ull << m) - 1);
    const int e = (int8_t)in[p - 1];
    if (e == -128 && mt == 0) return sign ? -0.0 : 0.0;
    const double v = ldexp(1.0 + ldexp((double)mt, -m), e);
    return sign ? -v : v;
}

template <int D>
__global__ __launch_bounds__(256) void k_p3_encode(const double *K, const double *K1, int64_t count, double tau,
                                                   uint8_t *p3_out, uint8_t *bytes_out)
{
#pragma clang fp contract(off)
    constexpr int nl = 1 << D, nn = nl * nl, U = n_pairs(D);
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= count) return;
    double E[nn];
    for (int a = 0; a < nl; ++a)
        for (int b = a + 1; b < nl; ++b) {
            const int pi = pair_index(D, a, b);
            const double d = K[c * U + pi] - K1[c * U + pi];
            E[a * nl + b] = d;
            E[b * nl + a] = d;
        }
    for (int a = 0; a < nl; ++a) {
        double sum = 0.0;
        for (int b = 0; b < nl; ++b)
            if (b != a) sum = sum - E[a * nl + b];
        E[a * nl + a] = sum;
    }
    double fro = 0.0;
    for (int i = 0; i < nn; ++i) fro = fro + E[i] * E[i];
    int p = 8;
    if (sqrt(fro) < tau) {
        p = 0;
    } else {
        for (int q = 2; q < 8; ++q) {
            double err = 0.0;
            for (int i = 0; i < nn; ++i) {
                uint8_t buf[8];
                p3_put(E[i], q, buf);
                const double dd = fabs(p3_get(buf, q) - E[i]);
                if (dd > err) err = dd;
            }
            if (err <= tau) { p = q; break; }
        }
    }
    p3_out[c] = (uint8_t)p;
    uint8_t *o = bytes_out + c * (nn * 8);
    for (int i = 0; i < nn && p > 0; ++i) {
        if (p == 8) {
            const uint64_t b = (uint64_t)__double_as_longlong(E[i]);
            for (int k = 0; k < 8; ++k) o[i * 8 + k] = (uint8_t)(b >> (8 * k));
        } else {
            p3_put(E[i], p, o + i * p);
        }
    }
}

int launch_p3_encode(mgd_ctx *ctx, int dim, const double *K, const double *K1, int64_t count, double tau,
                     uint8_t *p3_out, uint8_t *bytes_out, hipStream_t st)
{
    const dim3 g(grid_for(count, 256));
    if (dim == 2) hipLaunchKernelGGL(k_p3_encode<2>, g, dim3(256), 0, st, K, K1, count, tau, p3_out, bytes_out);
    else hipLaunchKernelGGL(k_p3_encode<3>, g, dim3(256), 0, st, K, K1, count, tau, p3_out, bytes_out);
    HIPCHK(ctx, hipGetLastError());
    return MGD_OK;
}
