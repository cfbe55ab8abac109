// Hierarchical surplus store with dynamic precision (paper Sec. 5.5):
// the fine couplings are kept as their difference from the centre-sample
// base (eps_c K_ref assembled), per vertex at the cheapest tier that meets
// the storage tolerance, packed in 64-vertex tiles of one tier each.
#include "common.h"

// ------------------------------------------------------ bit-level encoders
// round-to-nearest-even into binary16 (|y| <= 65504 by construction)
__device__ inline uint32_t f32_to_f16_bits(float y)
{
    uint32_t b = __float_as_uint(y), sg = (b >> 16) & 0x8000u, a = b & 0x7fffffffu;
    if (a < 0x38800000u) {  // below 2^-14: multiples of 2^-24
        uint32_t q = (uint32_t)rintf(__uint_as_float(a) * 16777216.0f);
        return sg | q;
    }
    uint32_t h = a - 0x38000000u;  // exponent bias 127 -> 15
    h = (h + 0x0FFFu + ((h >> 13) & 1u)) >> 13;
    return sg | h;
}

// round-to-nearest-even into OCP FP8 E4M3FN (|y| <= 448 by construction)
__device__ inline uint32_t f32_to_e4m3_bits(float y)
{
    uint32_t b = __float_as_uint(y), sg = (b >> 24) & 0x80u, a = b & 0x7fffffffu;
    if (a < 0x3C800000u) {  // below 2^-6: multiples of 2^-9
        uint32_t q = (uint32_t)rintf(__uint_as_float(a) * 512.0f);
        return sg | q;
    }
    uint32_t h = a - 0x3C000000u;  // exponent bias 127 -> 7
    h = (h + 0x7FFFFu + ((h >> 20) & 1u)) >> 20;
    if (h > 0x7Eu) h = 0x7Eu;
    return sg | h;
}

__device__ inline double f16_bits_value(uint32_t h) { return (double)(float)__builtin_bit_cast(_Float16, (uint16_t)h); }

// smallest e with mx <= fmax(t) 2^e, from the FP32 fields of mx
__device__ inline int scale_exponent(float mx, int t)
{
    if (t == 3 || !(mx > 0.0f)) return 0;
    int Ef = t == 1 ? 8 : 15;
    uint32_t mf = t == 1 ? 0x600000u : 0x7FE000u;  // 448 = 1.75 2^8, 65504 = (2 - 2^-10) 2^15
    uint32_t a = __float_as_uint(mx);
    int Ea;
    uint32_t ma;
    if (a >= 0x00800000u) {
        Ea = (int)(a >> 23) - 127;
        ma = a & 0x7FFFFFu;
    } else {
        int lz = __clz((int)a) - 8;
        ma = (a << lz) & 0x7FFFFFu;
        Ea = -126 - lz;
    }
    int e = Ea - Ef + (ma > mf ? 1 : 0);
    return e < -127 ? -127 : (e > 127 ? 127 : e);
}

// code of delta at tier t with scale 2^e, and its decoded value (exact, FP64)
__device__ inline uint32_t quantise(float d, int t, int e, double *dec)
{
#pragma clang fp contract(off)
    if (t == 3) {
        *dec = (double)d;
        return __float_as_uint(d);
    }
    float y = d * __uint_as_float((uint32_t)(127 - e) << 23 | 0u);  // d * 2^-e
    if (127 - e <= 0) y = (float)ldexp((double)d, -e);
    uint32_t c;
    double v;
    if (t == 2) {
        c = f32_to_f16_bits(y);
        v = f16_bits_value(c);
    } else {
        c = f32_to_e4m3_bits(y);
        v = (double)e4m3_to_float(c);
    }
    *dec = ldexp(v, e);
    return c;
}

// ------------------------------------------------------------ kernels
template <int D>
__global__ void k_deltas(const float *S32, const float *eps_c, int n, int64_t NV, double tau_abs,
                         double tau_rel, int tmin, int tmax, float *delta, uint8_t *vtier)
{
    // the surplus is defined by unfused FP64 operations (no FMA contraction)
#pragma clang fp contract(off)
    Grid<D> g(n);
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= NV) return;
    int x[3] = {0, 0, 0};
    g.coords(v, x);
    constexpr int H = n_half(D);
    float d[H];
    double ref = 0.0;
    float mx = 0.0f;
    BaseCells<D> bc;
    bc.load(eps_c, n, x);
#pragma unroll
    for (int j = 0; j < H; ++j) {
        double b = bc.coupling(j, &ref);
        d[j] = (float)((double)S32[(int64_t)j * NV + v] - b);
        delta[(int64_t)j * NV + v] = d[j];
        mx = fmaxf(mx, fabsf(d[j]));
    }
    double tau = tau_rel * ref;
    if (tau_abs > tau) tau = tau_abs;
    int tier = tmax;
    if ((double)mx <= tau) tier = 0;
    else {
        for (int t = tmin; t <= tmax; ++t) {
            if (t == 0) continue;
            int e = scale_exponent(mx, t);
            double err = 0.0;
            for (int j = 0; j < H; ++j) {
                double dec;
                quantise(d[j], t, e, &dec);
                err = fmax(err, fabs(dec - (double)d[j]));
            }
            if (err <= tau) { tier = t; break; }
        }
    }
    vtier[v] = (uint8_t)tier;
}

__global__ void k_tile_tier(const uint8_t *vtier, int64_t NV, int64_t ntile, int H, uint8_t *tier, uint32_t *units)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ntile) return;
    int m = 0;
    for (int64_t v = t * 64; v < NV && v < t * 64 + 64; ++v) m = vtier[v] > m ? vtier[v] : m;
    tier[t] = (uint8_t)m;
    units[t] = tile_units(m, H);
}

// single-block exclusive scan of uint32 sizes, in place; total to *total
__global__ void k_scan_u32(uint32_t *a, int64_t n, uint32_t *total)
{
    __shared__ uint32_t buf[1024];
    __shared__ uint32_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int64_t base = 0; base < n; base += 1024) {
        int64_t i = base + threadIdx.x;
        uint32_t v = i < n ? a[i] : 0;
        buf[threadIdx.x] = v;
        __syncthreads();
        for (int o = 1; o < 1024; o <<= 1) {
            uint32_t t = threadIdx.x >= o ? buf[threadIdx.x - o] : 0;
            __syncthreads();
            buf[threadIdx.x] += t;
            __syncthreads();
        }
        if (i < n) a[i] = carry + buf[threadIdx.x] - v;
        __syncthreads();
        if (threadIdx.x == 1023) carry += buf[1023];
        __syncthreads();
    }
    if (threadIdx.x == 0) *total = carry;
}

// one lane per (tile, vertex slot); lanes past NV write zeros
template <int D>
__global__ void k_encode(const float *delta, int64_t NV, int64_t ntile, const uint8_t *tier,
                         const uint32_t *toff, uint8_t *payload)
{
    int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t t = gid >> 6;
    if (t >= ntile) return;
    int l = (int)(gid & 63), tt = tier[t];
    if (tt == 0) return;
    constexpr int H = n_half(D);
    int64_t v = gid;
    uint8_t *base = payload + (size_t)toff[t] * 64;
    int eb = tier_bytes(tt);
    if (v >= NV) {
        base[l] = 0;
        for (int j = 0; j < H; ++j)
            for (int b = 0; b < eb; ++b) base[64 + ((size_t)j * 64 + l) * eb + b] = 0;
        return;
    }
    float d[H], mx = 0.0f;
    for (int j = 0; j < H; ++j) {
        d[j] = delta[(int64_t)j * NV + v];
        mx = fmaxf(mx, fabsf(d[j]));
    }
    int e = scale_exponent(mx, tt);
    base[l] = (uint8_t)(e + 127);
    for (int j = 0; j < H; ++j) {
        double dec;
        uint32_t c = quantise(d[j], tt, e, &dec);
        uint8_t *slot = base + 64 + (size_t)j * 64 * eb;
        if (eb == 1) slot[l] = (uint8_t)c;
        else if (eb == 2) ((uint16_t *)slot)[l] = (uint16_t)c;
        else ((uint32_t *)slot)[l] = c;
    }
}

// the decoded store, i.e. the mixed form's operator: base + delta summed in
// FP64 and rounded once to FP32 (written as FP32 or widened to FP64)
template <int D, typename TO>
__global__ void k_decode_store(StoreView sv, int n, TO *out)
{
#pragma clang fp contract(off)
    Grid<D> g(n);
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= g.NV) return;
    int x[3] = {0, 0, 0};
    g.coords(v, x);
    constexpr int H = n_half(D);
    BaseCells<D> bc;
    bc.load(sv.eps_c, n, x);
#pragma unroll
    for (int j = 0; j < H; ++j) {
        double b = bc.coupling(j, nullptr);
        out[(int64_t)j * g.NV + v] = (TO)(float)(b + (double)sv.delta(v, j, H));
    }
}

int decode_store_f32(mgd_hier *h, OpSet &o, hipStream_t st);

template <typename TI> __global__ void k_to_f64(const TI *in, int64_t cnt, double *out)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < cnt) out[i] = (double)in[i];
}

// ------------------------------------------------------------ host side
int compress_into(mgd_hier *h, OpSet &o, const float *S32, const float *eps_c,
                  const mgd_tier_policy *pol, float *delta, uint8_t *vtier, hipStream_t st)
{
    mgd_ctx *ctx = h->ctx;
    int64_t NV = h->NV[0], nc = 1;
    for (int m = 0; m < h->dim; ++m) nc *= h->n;
    if (eps_c != o.eps_c)
        HIPCHK(ctx, hipMemcpyAsync(o.eps_c, eps_c, sizeof(float) * nc, hipMemcpyDeviceToDevice, st));
    dim3 gv(grid_for(NV, 256));
    if (h->dim == 2)
        hipLaunchKernelGGL(k_deltas<2>, gv, dim3(256), 0, st, S32, o.eps_c, h->n, NV, pol->tau_abs,
                           pol->tau_rel, pol->min_tier, pol->max_tier, delta, vtier);
    else
        hipLaunchKernelGGL(k_deltas<3>, gv, dim3(256), 0, st, S32, o.eps_c, h->n, NV, pol->tau_abs,
                           pol->tau_rel, pol->min_tier, pol->max_tier, delta, vtier);
    hipLaunchKernelGGL(k_tile_tier, dim3(grid_for(o.ntile, 256)), dim3(256), 0, st, vtier, NV, o.ntile,
                       h->H, o.tier, o.toff);
    hipLaunchKernelGGL(k_scan_u32, dim3(1), dim3(1024), 0, st, o.toff, o.ntile, o.units_total);
    dim3 ge(grid_for(o.ntile * 64, 256));
    if (h->dim == 2)
        hipLaunchKernelGGL(k_encode<2>, ge, dim3(256), 0, st, delta, NV, o.ntile, o.tier, o.toff, o.payload);
    else
        hipLaunchKernelGGL(k_encode<3>, ge, dim3(256), 0, st, delta, NV, o.ntile, o.tier, o.toff, o.payload);
    HIPCHK(ctx, hipGetLastError());
    return decode_store_f32(h, o, st);  // the FP32 finest operator follows the store
}

// every tile at tier 0: the operator is exactly the centre-sample base
int store_set_base(mgd_hier *h, OpSet &o, const float *eps_c, hipStream_t st)
{
    mgd_ctx *ctx = h->ctx;
    int64_t nc = 1;
    for (int m = 0; m < h->dim; ++m) nc *= h->n;
    if (eps_c != o.eps_c)
        HIPCHK(ctx, hipMemcpyAsync(o.eps_c, eps_c, sizeof(float) * nc, hipMemcpyDeviceToDevice, st));
    HIPCHK(ctx, hipMemsetAsync(o.tier, 0, o.ntile, st));
    HIPCHK(ctx, hipMemsetAsync(o.toff, 0, sizeof(uint32_t) * o.ntile, st));
    HIPCHK(ctx, hipMemsetAsync(o.units_total, 0, sizeof(uint32_t), st));
    return decode_store_f32(h, o, st);
}

StoreView store_view(const mgd_hier *h, const OpSet &o)
{
    StoreView sv;
    sv.tier = o.tier; sv.off = o.toff; sv.payload = o.payload; sv.eps_c = o.eps_c;
    sv.n = h->n; sv.NV = h->NV[0];
    return sv;
}

// decoded level-0 operator of the mixed path, FP32 (Galerkin input, unfused
// kernels, the 3D outer operator); kept current with every change of the store
int decode_store_f32(mgd_hier *h, OpSet &o, hipStream_t st)
{
    o.dz_ok = 0;
    StoreView sv = store_view(h, o);
    dim3 gv(grid_for(h->NV[0], 256));
    if (h->dim == 2) hipLaunchKernelGGL((k_decode_store<2, float>), gv, dim3(256), 0, st, sv, h->n, o.S32[0]);
    else hipLaunchKernelGGL((k_decode_store<3, float>), gv, dim3(256), 0, st, sv, h->n, o.S32[0]);
    HIPCHK(h->ctx, hipGetLastError());
    return MGD_OK;
}

int decode_level_f64(mgd_hier *h, const OpSet &o, int level, double *out, hipStream_t st)
{
    int64_t NV = h->NV[level], cnt = NV * h->H;
    if (h->precision == MGD_FP64) {
        HIPCHK(h->ctx, hipMemcpyAsync(out, o.S64[level], sizeof(double) * cnt, hipMemcpyDeviceToDevice, st));
        return MGD_OK;
    }
    if (level == 0) {
        StoreView sv = store_view(h, o);
        dim3 gv(grid_for(NV, 256));
        if (h->dim == 2) hipLaunchKernelGGL((k_decode_store<2, double>), gv, dim3(256), 0, st, sv, h->n, out);
        else hipLaunchKernelGGL((k_decode_store<3, double>), gv, dim3(256), 0, st, sv, h->n, out);
    } else {
        hipLaunchKernelGGL((k_to_f64<float>), dim3(grid_for(cnt, 256)), dim3(256), 0, st, o.S32[level], cnt, out);
    }
    HIPCHK(h->ctx, hipGetLastError());
    return MGD_OK;
}

int opset_alloc(mgd_hier *h, OpSet &o)
{
    mgd_ctx *ctx = h->ctx;
    int rc;
    int nlw = 1 << h->dim;
    for (int l = 0; l < h->nlev; ++l) {
        size_t cnt = (size_t)h->NV[l] * h->H;
        if (h->precision == MGD_FP64) {
            if ((rc = dev_alloc(ctx, (void **)&o.S64[l], cnt * 8))) return rc;
        } else {
            if ((rc = dev_alloc(ctx, (void **)&o.S32[l], cnt * 4))) return rc;
        }
        if (h->transfer == MGD_BOXMG && l + 1 < h->nlev)
            if ((rc = dev_alloc(ctx, &o.W[l], (size_t)h->NV[l] * nlw * h->vec_bytes()))) return rc;
        if (h->dim == 3 && (rc = dev_alloc(ctx, &o.Dz[l], (size_t)h->NV[l] * h->vec_bytes()))) return rc;
        if (h->dim == 3 && h->transfer == MGD_BOXMG && l + 1 < h->nlev &&
            (rc = dev_alloc(ctx, (void **)&o.wgeo[l], (size_t)(h->NV[l] + 63) / 64)))
            return rc;
    }
    o.dz_ok = 0;
    if (h->precision == MGD_MIXED) {
        int64_t nc = 1;
        for (int m = 0; m < h->dim; ++m) nc *= h->n;
        o.ntile = (h->NV[0] + 63) / 64;
        o.payload_cap_units = o.ntile * tile_units(3, h->H);
        if ((rc = dev_alloc(ctx, (void **)&o.tier, o.ntile))) return rc;
        if ((rc = dev_alloc(ctx, (void **)&o.toff, o.ntile * 4))) return rc;
        if ((rc = dev_alloc(ctx, (void **)&o.payload, (size_t)o.payload_cap_units * 64))) return rc;
        if ((rc = dev_alloc(ctx, (void **)&o.eps_c, nc * 4))) return rc;
        if ((rc = dev_alloc(ctx, (void **)&o.units_total, 64))) return rc;
        if (h->dim == 3 && items4_fit(3, h->n) &&
            (rc = dev_alloc(ctx, (void **)&o.imask, (size_t)(h->n / 4) * h->NV[0] / (h->n + 1))))
            return rc;
        HIPCHK(ctx, hipMemset(o.tier, 0, o.ntile));
        HIPCHK(ctx, hipMemset(o.toff, 0, o.ntile * 4));
        HIPCHK(ctx, hipMemset(o.units_total, 0, 4));
    }
    int64_t m = h->m_coarse;
    if ((rc = dev_alloc(ctx, (void **)&o.chol, (size_t)(m > 0 ? m * m : 1) * 8))) return rc;
    if (m <= kCinvMax && (rc = dev_alloc(ctx, (void **)&o.cinv, (size_t)(m > 0 ? m * m : 1) * 8))) return rc;
    return MGD_OK;
}

void opset_free(OpSet &o)
{
    for (int l = 0; l < MGD_MAXLEV; ++l) {
        dev_free(o.S64[l]); dev_free(o.S32[l]); dev_free(o.W[l]); dev_free(o.Dz[l]); dev_free(o.wgeo[l]);
        o.S64[l] = nullptr; o.S32[l] = nullptr; o.W[l] = nullptr; o.Dz[l] = nullptr; o.wgeo[l] = nullptr;
    }
    dev_free(o.tier); dev_free(o.toff); dev_free(o.payload); dev_free(o.eps_c);
    dev_free(o.units_total); dev_free(o.chol); dev_free(o.cinv); dev_free(o.imask);
    o = OpSet();
}
