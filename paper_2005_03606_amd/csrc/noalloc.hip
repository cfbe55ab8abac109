// Allocation-free entry point: mgd_compress_stencils_noalloc keeps the
// compression's working buffers (the surplus [H][NV] FP32 and the vertex
// tiers [NV]) in a static device array instead of the hierarchy's
// buffers, so a caller that cannot allocate device memory (HIP graph
// capture, a tight serving loop) can re-compress a level-0 store.
//
// The array is file scope and __device__: every GPU the library runs on
// holds its own copy, at its own address, until the process ends.  Host
// code must not pass the array's name to a kernel (on the host it names a
// host-side stand-in); scratch_init looks up this device's address once,
// at context creation, and kernels receive that address.
#include <mutex>

#include "common.h"

// 64 MiB: the surplus and tiers of up to kScratchBytes / (4 H + 1) vertices
// (3D: ~1.27 M vertices, e.g. 107^3 cells; 2D: ~3.9 M, e.g. 1976^2 cells)
constexpr size_t kScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

static std::mutex g_scratch_mu;
static unsigned char *g_scratch_addr[64] = {};  // per device, looked up once

int scratch_init(mgd_ctx *ctx)
{
    if (ctx->device < 0 || ctx->device >= 64) return mgd_fail(ctx, MGD_EINVAL, "device index %d", ctx->device);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_addr[ctx->device]) {
        void *p = nullptr;
        // the context's device is current (mgd_create set it)
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return mgd_fail(ctx, MGD_EHIP, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
        g_scratch_addr[ctx->device] = (unsigned char *)p;
    }
    ctx->scratch = g_scratch_addr[ctx->device];
    return MGD_OK;
}

extern "C" int mgd_compress_stencils_noalloc(mgd_ctx *ctx, mgd_hier *h, const float *S32, const float *eps_c,
                                             const mgd_tier_policy *pol, hipStream_t stream)
{
    if (!ctx || !h || !S32 || !eps_c || !pol) return MGD_EINVAL;
    if (h->ctx != ctx) return mgd_fail(ctx, MGD_EINVAL, "hierarchy belongs to another context");
    if (h->precision != MGD_MIXED) return mgd_fail(ctx, MGD_EINVAL, "compress needs a MGD_MIXED hierarchy");
    if (pol->min_tier < 1 || pol->max_tier > 3 || pol->min_tier > pol->max_tier)
        return mgd_fail(ctx, MGD_EINVAL, "tiers must satisfy 1 <= min_tier <= max_tier <= 3");
    if (!(pol->tau_abs >= 0.0) || !(pol->tau_rel >= 0.0)) return mgd_fail(ctx, MGD_EINVAL, "tau must be >= 0");
    if (!ctx->scratch) return mgd_fail(ctx, MGD_EINVAL, "context has no scratch address");
    // surplus at offset 0, tiers after it on a 256-byte boundary
    const size_t delta_bytes = (size_t)h->NV[0] * h->H * 4;
    const size_t tier_off = (delta_bytes + 255) & ~(size_t)255;
    const size_t need = tier_off + (size_t)h->NV[0];
    if (need > kScratchBytes)
        return mgd_fail(ctx, MGD_EINVAL, "level 0 has %lld vertices: the allocation-free compression holds at most "
                        "%lld (%zu scratch bytes, %d surplus slots per vertex)", (long long)h->NV[0],
                        (long long)(kScratchBytes / (4 * (size_t)h->H + 1)), kScratchBytes, h->H);
    HIPCHK(ctx, hipSetDevice(ctx->device));
    float *delta = (float *)ctx->scratch;
    uint8_t *vtier = ctx->scratch + tier_off;
    return compress_into(h, h->ops, S32, eps_c, pol, delta, vtier, stream);
}
