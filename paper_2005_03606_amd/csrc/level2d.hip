// Fused 2D V-cycle level steps (paper Sec. 4): the pre-smoothing half of a
// level (two damped Jacobi sweeps followed by the residual) and the
// post-smoothing half (prolongation of the coarse correction followed by two
// sweeps), each one pass over the level.  A block owns a 64 x BY tile of
// vertices; it stages the operator, the right-hand side and the iterate of
// the tile plus a halo of K vertices (K = number of stencil applications) in
// LDS and applies the stencil K times on shrinking regions, so the level's
// data crosses HBM once per half-cycle instead of once per sweep.  The
// operator comes from FP32 / FP64 half stencils or, on the finest level of
// the mixed form, from the compressed surplus store (centre-sample base plus
// the decoded FP8 / FP16 / FP32 surplus, Sec. 5.5).  Tiles are numbered so
// that each XCD (workgroups go round-robin over the 8 XCDs) receives a
// contiguous band of tile rows and neighbouring tiles share halo rows in one
// L2.  At the outer level of the conjugate-gradient iteration the post half
// also forms the block partials of the two dot products of the Polak-Ribiere
// coefficient (summed in fixed order by one reduction launch afterwards).
#include "common.h"

enum { L2_PRE = 0, L2_POST = 1, L2_PMV = 2, L2_PRER = 3 };

template <typename T> struct Lev2Args {
    const T *S;       // half stencils [4][NV] (unless the store is used)
    const float *Sf;  // PMV with an FP32 iterate: the FP32 half stencils (mixed form, store not used)
    StoreView sv;     // compressed finest-level store
    int n;            // cells per axis of this level
    const T *u;       // PRE: start iterate (unless zero); POST: iterate before prolongation
    const T *f;       // right-hand side
    T *u_out;         // smoothed iterate on the tile
    T *r_out;         // PRE: residual after smoothing
    const T *ec;      // POST: coarse correction on the (n/2)-grid
    const T *W;       // POST: BoxMG weights [4][NV] of this level, or null (d-linear)
    T omega;
    // POST at the outer level: partials of z.r and z.(r - r_old), z = u_out
    const double *r64, *rold64;
    double *partial;
    // PMV (CG, FP64): p = z + beta p_old, Ap = A p; beta from the dot partials
    const void *z;
    const double *pold;
    double *pnew, *Ap;
    CgScalars cg;
};

// sum of v over the block (256 threads)
__device__ inline double lev2_block_sum(double v, double *red)
{
    red[threadIdx.x] = v;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    double r = red[0];
    __syncthreads();
    return r;
}

// fixed-order sum of cnt partials by the block (the same value in every block)
__device__ inline double sum_partials2(const double *p, int64_t cnt, double *red)
{
    double v = 0.0;
    for (int64_t i = threadIdx.x; i < cnt; i += 256) v += p[i];
    return lev2_block_sum(v, red);
}

// surplus entry j of vertex lane l of a payload tile (tier 1: FP8 E4M3,
// 2: FP16, 3: FP32), from the aligned 32-bit word w holding it and the
// vertex's scale word sw
__device__ inline float lev2_decode(int tier, int l, uint32_t sw, uint32_t w)
{
    const float sc = e8m0_to_float((sw >> ((l & 3) * 8)) & 0xffu);
    if (tier == 2) return (float)__builtin_bit_cast(_Float16, (uint16_t)((w >> ((l & 1) * 16)) & 0xffffu)) * sc;
    if (tier == 1) return e4m3_to_float((w >> ((l & 3) * 8)) & 0xffu) * sc;
    if (tier == 3) return __uint_as_float(w);
    return 0.0f;
}

// byte offset, within its tile's payload, of the word holding entry j of
// vertex lane l (tier-0 vertices: 0)
__device__ inline uint32_t lev2_word(int tier, int l, int j)
{
    const int tb = tier == 3 ? 4 : tier;
    return tier ? (uint32_t)((64 + j * 64 * tb + l * tb) & ~3) : 0u;
}

// Thread layout: lane = column, wave = row (stride 4) when staging; in the
// stencil applications lane = column 1 + lane of the halo region, each wave
// a contiguous band of rows, with the 3 x 3 iterate window carried in
// registers from row to row.
template <typename T, int BY, int KIND, bool COMP, bool ZERO, bool DOTS, bool ZF = false>
__global__ __launch_bounds__(256) void k_lev2(Lev2Args<T> a)
{
    constexpr bool PMV = KIND == L2_PMV, RST = KIND == L2_PRER;  // RST: pre half + restriction
    constexpr bool PREK = KIND == L2_PRE || RST;
    constexpr int K = PREK ? 3 : KIND == L2_POST ? 2 : 1;  // stencil applications
    // halos: K vertices on the high side, K (K + 1 when restricting: the
    // residual is needed one vertex below the tile) on the low side; the
    // first application spans at most 64 columns (one lane each)
    constexpr int HL = RST ? K + 1 : K, HH = K;
    constexpr int BX = RST ? 58 : 66 - 2 * K;           // tile width (even when restricting)
    constexpr int UW = BX + HL + HH, UH = BY + HL + HH; // iterate / rhs region
    constexpr int CH = UH - 1, EW = UW + 1, EH = UH;    // couplings, centre samples
    constexpr int XU = UW - 64, XE = EW - 64;           // columns beyond the 64 lanes
    constexpr int RU = (UH + 3) / 4, RC = (CH + 3) / 4, RE = (EH + 3) / 4;
    constexpr int RA = (UH - 2 + 3) / 4;                // rows per wave, first application
    constexpr int RL = BY / 4;                          // rows per wave, last application (symmetric halos)
    static_assert(BY % 4 == 0, "tile height must be a multiple of 4");
    static_assert(!RST || (BX / 2) * (BY / 2) <= 256, "restriction: one thread per coarse vertex of the tile");
    static_assert(UW - 2 <= 64 && XU >= 0 && XU <= 3, "halo region must fit the lane layout");
    constexpr int UH2 = PMV ? 1 : UH;                   // arrays the product does not use
    __shared__ T sC[4][CH][UW];
    __shared__ T sU0[UH][UW], sU1[UH2][UW];
    __shared__ T sF[UH2][UW], sWD[UH2][UW];
    __shared__ float sE[COMP ? EH : 1][COMP ? EW : 1];
    __shared__ double red[DOTS || PMV ? 256 : 1];

    const int n = a.n, nv = n + 1;
    const uint32_t NV = (uint32_t)nv * (uint32_t)nv;
    const int ntx = (nv + BX - 1) / BX, nty = (nv + BY - 1) / BY, nt = ntx * nty;
    const int per = (nt + 7) / 8;
    const int tile = (int)(blockIdx.x & 7) * per + (int)(blockIdx.x >> 3);
    if (tile >= nt) return;  // whole block: padding of the XCD-banded numbering
    const int x0 = (tile % ntx) * BX, y0 = (tile / ntx) * BY;
    const int gx = x0 - HL, gy = y0 - HL;  // global coordinates of local (0, 0)
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    auto in_dom = [&](int x, int y) { return x >= 0 && x <= n && y >= 0 && y <= n; };
    double beta = 0.0;
    if (PMV) {
        // Polak-Ribiere coefficient from the dot partials, every block in the same order
        const double zr = sum_partials2(a.cg.p1, a.cg.n1, red), zdr = sum_partials2(a.cg.p1 + a.cg.n1, a.cg.n1, red);
        beta = a.cg.s[7] != 0.0 ? 0.0 : zdr / a.cg.s[a.cg.zr_old];
        if (blockIdx.x == 0 && tid == 0) a.cg.s[a.cg.zr_new] = zr;
    }
    auto vid = [&](int x, int y) { return (uint32_t)y * (uint32_t)nv + (uint32_t)x; };

    // ---------------- phase 1: all global loads into registers, no branches
    // between them (out-of-range items read index 0 and are zeroed after)
    // (a) iterate, rhs, prolongation on the U region: main columns 0..63 by
    // lane, rows by wave; the XU extra columns one item per thread
    constexpr int NPU = KIND == L2_POST ? RU + 1 : 1;
    T fr[RU + 1], ur[RU + 1], wr[NPU][4], er[NPU][4];
    const T *Wsrc = a.W ? a.W : a.ec;
    auto load_u = [&](int s, int lx, int ly, bool ok) {
        const int vx = gx + lx, vy = gy + ly;
        const bool dom = ok && in_dom(vx, vy);
        const uint32_t v = dom ? vid(vx, vy) : 0u;
        if (PMV) {
            const double zl = ZF ? (double)((const float *)a.z)[v] : ((const double *)a.z)[v];
            const double pl = a.pold[v];
            ur[s] = dom ? (T)(zl + beta * pl) : (T)0;
            fr[s] = (T)0;
            return;
        }
        const T fl = a.f[v];
        fr[s] = dom ? fl : (T)0;
        if (KIND == L2_POST || !ZERO) {
            const T ul = a.u[v];
            ur[s] = dom ? ul : (T)0;
        } else {
            ur[s] = (T)0;
        }
        if (KIND == L2_POST) {
            // u += P e: weights of v toward the corners (x>>1)+bx, (y>>1)+by of
            // its coarse box; only corners along odd axes can be non-zero
            const bool inner = dom && vx > 0 && vx < n && vy > 0 && vy < n;
            const uint32_t nc1 = (uint32_t)(n / 2 + 1);
            const int bxm = vx & 1, bym = vy & 1;
#pragma unroll
            for (int B = 0; B < 4; ++B) {
                const int bx = B & 1, by = B >> 1;
                const bool use = inner && bx <= bxm && by <= bym;
                const uint32_t ic = use ? (uint32_t)((vy >> 1) + by) * nc1 + (uint32_t)((vx >> 1) + bx) : 0u;
                const T e = a.ec[ic];
                const T wl = Wsrc[a.W && use ? (uint32_t)B * NV + v : 0u];
                const T w = a.W ? wl : (T)((bxm ? 0.5 : 1.0) * (bym ? 0.5 : 1.0));
                wr[s][B] = use ? w : (T)0;
                er[s][B] = use ? e : (T)0;
            }
        }
    };
#pragma unroll
    for (int j = 0; j < RU; ++j) load_u(j, lane, wave + 4 * j, wave + 4 * j < UH);
    load_u(RU, 64 + tid % XU, tid / XU, tid < XU * UH);

    // (b) couplings on the C region (half stencils), or the store's centre
    // samples, tier bytes, offsets and payload words
    constexpr int NCR = COMP ? 1 : RC + 1;
    T cr[NCR][4];
    constexpr int NER = COMP ? RE + 1 : 1, NTR = COMP ? RC + 1 : 1;
    float epr[NER];
    int tt[NTR];
    uint32_t oo[NTR], sw[NTR], wv[NTR][4];
    if (!COMP) {
        auto load_c = [&](int s, int lx, int ly, bool ok) {
            const int vx = gx + lx, vy = gy + ly;
            const bool dom = ok && in_dom(vx, vy);
            const uint32_t v = dom ? vid(vx, vy) : 0u;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                T c;
                if constexpr (PMV && ZF) c = (T)a.Sf[(uint32_t)j * NV + v];
                else c = a.S[(uint32_t)j * NV + v];
                cr[s][j] = dom ? c : (T)0;
            }
        };
#pragma unroll
        for (int j = 0; j < RC; ++j) load_c(j, lane, wave + 4 * j, wave + 4 * j < CH);
        load_c(RC, 64 + tid % XU, tid / XU, tid < XU * CH);
    } else {
        auto load_e = [&](int s, int lx, int ly, bool ok) {
            const int cx = gx - 1 + lx, cy = gy - 1 + ly;
            const bool in = ok && cx >= 0 && cx < n && cy >= 0 && cy < n;
            const float e = a.sv.eps_c[in ? (uint32_t)cy * (uint32_t)n + (uint32_t)cx : 0u];
            epr[s] = in ? e : 0.0f;
        };
#pragma unroll
        for (int j = 0; j < RE; ++j) load_e(j, lane, wave + 4 * j, wave + 4 * j < EH);
        load_e(RE, 64 + tid % XE, tid / XE, tid < XE * EH);
        auto load_t = [&](int s, int lx, int ly, bool ok) {
            const int vx = gx + lx, vy = gy + ly;
            const bool dom = ok && in_dom(vx, vy);
            const uint32_t t = dom ? vid(vx, vy) >> 6 : 0u;
            const int tl = a.sv.tier[t];
            const uint32_t ol = a.sv.off[t];
            tt[s] = dom ? tl : 0;
            oo[s] = ol;
        };
#pragma unroll
        for (int j = 0; j < RC; ++j) load_t(j, lane, wave + 4 * j, wave + 4 * j < CH);
        load_t(RC, 64 + tid % XU, tid / XU, tid < XU * CH);
        // payload words: the vertex's scale byte and its four entries, read as
        // the aligned 32-bit words holding them (tiles are 64-byte aligned);
        // offsets in bytes from the payload start (tier-0 items read word 0)
        const uint32_t *P32 = (const uint32_t *)a.sv.payload;
        auto load_p = [&](int s, int lx, int ly) {
            const uint32_t l = vid(gx + lx, gy + ly) & 63u;
            const int tier = tt[s];
            const uint32_t tb = tier == 3 ? 4u : (uint32_t)tier;
            const uint32_t base = tier ? oo[s] * 64u : 0u;
            const uint32_t o0 = tier ? base + 64u + ((l * tb) & ~3u) : 0u, step = 64u * tb;
            sw[s] = P32[(base + (l & ~3u)) >> 2];
#pragma unroll
            for (int j = 0; j < 4; ++j) wv[s][j] = P32[(o0 + (uint32_t)j * step) >> 2];
        };
#pragma unroll
        for (int j = 0; j < RC; ++j) load_p(j, lane, wave + 4 * j);
        load_p(RC, 64 + tid % XU, tid / XU);
    }
    // DOTS: the outer residual and its previous value on this wave's rows of
    // the last application
    double dr[DOTS ? RL : 1], dro[DOTS ? RL : 1];
    if (DOTS) {
        const int vx = gx + 1 + lane;
#pragma unroll
        for (int r = 0; r < RL; ++r) {
            const int vy = gy + HL + wave * RL + r;
            const bool ok = lane + 1 >= HL && lane + 1 < HL + BX && in_dom(vx, vy);
            const uint32_t v = ok ? vid(vx, vy) : 0u;
            const double x1 = a.r64[v], x2 = a.rold64[v];
            dr[r] = ok ? x1 : 0.0;
            dro[r] = ok ? x2 : 0.0;
        }
    }

    // RST: the restriction weights of this thread's coarse vertex (9 fine neighbours)
    T wres[RST ? 9 : 1];
    if (RST) {
        constexpr int CW = BX / 2;
        const int cx = tid % CW, cy = tid / CW, nc = n / 2;
        const int X = x0 / 2 + cx, Y = y0 / 2 + cy;
        const bool use = tid < CW * (BY / 2) && X > 0 && X < nc && Y > 0 && Y < nc;
#pragma unroll
        for (int sv = 0; sv < 9; ++sv) {
            const int ox = sv % 3 - 1, oy = sv / 3 - 1;
            const int B = (ox < 0 ? 1 : 0) | (oy < 0 ? 2 : 0);  // X - (x >> 1) is 1 exactly where o = -1
            const uint32_t v = use ? vid(2 * X + ox, 2 * Y + oy) : 0u;
            const T wl = Wsrc[a.W && use ? (uint32_t)B * NV + v : 0u];
            const T geo = (T)((ox ? 0.5 : 1.0) * (oy ? 0.5 : 1.0));
            wres[sv] = use ? (a.W ? wl : geo) : (T)0;
        }
    }

    // ---------------- stores into LDS
    auto store_u = [&](int s, int lx, int ly, bool ok) {
        if (!ok) return;
        T uv = ur[s];
        if (KIND == L2_POST) {
            T sum = (T)0;
#pragma unroll
            for (int B = 0; B < 4; ++B)
                if (wr[s][B] != (T)0) sum += wr[s][B] * er[s][B];
            uv += sum;
        }
        if (!PMV) sF[ly][lx] = fr[s];
        sU0[ly][lx] = uv;
    };
#pragma unroll
    for (int j = 0; j < RU; ++j) store_u(j, lane, wave + 4 * j, wave + 4 * j < UH);
    store_u(RU, 64 + tid % XU, tid / XU, tid < XU * UH);
    if (!COMP) {
#pragma unroll
        for (int j = 0; j < RC; ++j)
            if (wave + 4 * j < CH)
                for (int q = 0; q < 4; ++q) sC[q][wave + 4 * j][lane] = cr[j][q];
        if (tid < XU * CH)
            for (int q = 0; q < 4; ++q) sC[q][tid / XU][64 + tid % XU] = cr[RC][q];
    } else {
#pragma unroll
        for (int j = 0; j < RE; ++j)
            if (wave + 4 * j < EH) sE[wave + 4 * j][lane] = epr[j];
        if (tid < XE * EH) sE[tid / XE][64 + tid % XE] = epr[RE];
    }
    __syncthreads();

    // ---------------- phase 2 (store): centre-sample base + decoded surplus
    if (COMP) {
        const double k6 = -1.0 / 6.0, k3 = -1.0 / 3.0;
        auto decode = [&](int s, int lx, int ly, bool ok) {
            // base + surplus in FP64 without fused multiply-add, rounded once
            // to FP32: the store's decode, bit for bit
#pragma clang fp contract(off)
            if (!ok) return;
            const uint32_t l = vid(gx + lx, gy + ly) & 63u;
            // cells around the vertex: (x, y-1), (x-1, y), (x, y) at sE[ly][lx+1], sE[ly+1][lx], sE[ly+1][lx+1]
            const double e10 = sE[ly][lx + 1], e01 = sE[ly + 1][lx], e11 = sE[ly + 1][lx + 1];
            float d[4] = {0.0f, 0.0f, 0.0f, 0.0f};
            const int tier = tt[s];
            if (tier == 2) {
                const float sc = e8m0_to_float((sw[s] >> ((l & 3u) * 8u)) & 0xffu);
                const uint32_t sh = (l & 1u) * 16u;
#pragma unroll
                for (int q = 0; q < 4; ++q) d[q] = (float)__builtin_bit_cast(_Float16, (uint16_t)(wv[s][q] >> sh)) * sc;
            } else if (tier == 1) {
                const float sc = e8m0_to_float((sw[s] >> ((l & 3u) * 8u)) & 0xffu);
                const uint32_t sh = (l & 3u) * 8u;
#pragma unroll
                for (int q = 0; q < 4; ++q) d[q] = e4m3_to_float((wv[s][q] >> sh) & 0xffu) * sc;
            } else if (tier == 3) {
#pragma unroll
                for (int q = 0; q < 4; ++q) d[q] = __uint_as_float(wv[s][q]);
            }
            sC[0][ly][lx] = (T)(float)((e10 + e11) * k6 + (double)d[0]);
            sC[1][ly][lx] = (T)(float)(e01 * k3 + (double)d[1]);
            sC[2][ly][lx] = (T)(float)((e01 + e11) * k6 + (double)d[2]);
            sC[3][ly][lx] = (T)(float)(e11 * k3 + (double)d[3]);
        };
#pragma unroll
        for (int j = 0; j < RC; ++j) decode(j, lane, wave + 4 * j, wave + 4 * j < CH);
        decode(RC, 64 + tid % XU, tid / XU, tid < XU * CH);
        __syncthreads();
    }

    // ---------------- phase 2b: omega / diagonal on the first application's region
    // this lane's column in every application (lanes beyond the region read
    // a valid column and store nothing)
    const int lx = 1 + lane < UW - 1 ? 1 + lane : UW - 2;
    const int vxc = gx + lx;
    const bool xin = vxc > 0 && vxc < n;
    const T om = a.omega, om1 = (T)1 - a.omega;
#pragma unroll
    for (int j = 0; j < (UH - 2 + 3) / 4; ++j) {
        const int ly = 1 + wave + 4 * j;
        if (!PMV && ly < UH - 1) {
            const int vy = gy + ly;
            const T dsum = ((sC[0][ly][lx] + sC[1][ly][lx]) + (sC[2][ly][lx] + sC[3][ly][lx])) +
                           ((sC[0][ly][lx - 1] + sC[1][ly - 1][lx + 1]) + (sC[2][ly - 1][lx] + sC[3][ly - 1][lx - 1]));
            sWD[ly][lx] = (xin && vy > 0 && vy < n) ? om / -dsum : (T)0;
        }
    }
    if (!PMV) __syncthreads();

    // ---------------- phase 3: K stencil applications on shrinking regions
    double pa = 0.0, pb = 0.0;
#pragma unroll
    for (int k = 1; k <= K; ++k) {
        // application k covers local columns and rows [k, UW - k) x [k, UH - k)
        const bool last = k == K;
        const bool on = 1 + lane == lx && lx >= k && lx < UW - k;
        T(*Ui)[UW] = (k & 1) ? sU0 : sU1;
        T(*Uo)[UW] = (k & 1) ? sU1 : sU0;
        const bool need_u = !(PREK && ZERO && k == 1);
        // this wave's band of rows
        const int rh = UH - 2 * k, q = rh / 4, rr = rh % 4;
        const int ys = k + wave * q + (wave < rr ? wave : rr), cnt = q + (wave < rr ? 1 : 0);
        T um0 = (T)0, um1 = (T)0, um2 = (T)0, uc0 = (T)0, uc1 = (T)0, uc2 = (T)0, pa2 = (T)0;
        if (need_u) {
            um0 = Ui[ys - 1][lx - 1]; um1 = Ui[ys - 1][lx]; um2 = Ui[ys - 1][lx + 1];
            uc0 = Ui[ys][lx - 1]; uc1 = Ui[ys][lx]; uc2 = Ui[ys][lx + 1];
        }
        pa2 = sC[2][ys - 1][lx];
#pragma unroll
        for (int r = 0; r < RA; ++r) {
            if (r < cnt) {
                const int ly = ys + r, vy = gy + ly;
                const bool inner = xin && vy > 0 && vy < n;
                const T a2 = sC[2][ly][lx];
                T val = (T)0;
                if (!need_u) {
                    val = sWD[ly][lx] * sF[ly][lx];
                } else {
                    const T up0 = Ui[ly + 1][lx - 1], up1 = Ui[ly + 1][lx], up2 = Ui[ly + 1][lx + 1];
                    const T a0 = sC[0][ly][lx], a1 = sC[1][ly][lx], a3 = sC[3][ly][lx];
                    const T b0 = sC[0][ly][lx - 1], b1 = sC[1][ly - 1][lx + 1], b2 = pa2, b3 = sC[3][ly - 1][lx - 1];
                    const T acc = a0 * uc2 + a1 * up0 + a2 * up1 + a3 * up2 + b0 * uc0 + b1 * um2 + b2 * um1 + b3 * um0;
                    const T fv = PMV ? (T)0 : sF[ly][lx];
                    if (PMV) {
                        const T Dv = -(((a0 + a1) + (a2 + a3)) + ((b0 + b1) + (b2 + b3)));
                        val = Dv * uc1 + acc;
                    } else if (PREK && last) {
                        const T Dv = -(((a0 + a1) + (a2 + a3)) + ((b0 + b1) + (b2 + b3)));
                        val = fv - (Dv * uc1 + acc);
                    } else {
                        val = om1 * uc1 + sWD[ly][lx] * (fv - acc);
                    }
                    um0 = uc0; um1 = uc1; um2 = uc2;
                    uc0 = up0; uc1 = up1; uc2 = up2;
                }
                pa2 = a2;
                val = inner ? val : (T)0;
                const bool dom = on && in_dom(vxc, vy);
                if (last && RST) {
                    if (on) Uo[ly][lx] = val;  // residual, restricted below
                } else if (last) {
                    if (dom) {
                        const uint32_t v = vid(vxc, vy);
                        if (PMV) {
                            a.pnew[v] = (double)um1;  // the window moved on: row ly's p is um1 now
                            a.Ap[v] = (double)val;
                            pa += (double)um1 * (double)val;
                        } else if (KIND == L2_PRE) {
                            a.r_out[v] = val;
                        } else {
                            a.u_out[v] = val;
                        }
                    }
                    if (DOTS) {
                        const double z = dom ? (double)val : 0.0;
                        pa += z * dr[r];
                        pb += z * (dr[r] - dro[r]);
                    }
                } else {
                    if (on) Uo[ly][lx] = val;
                    // the smoothed iterate of the tile itself (after the last sweep)
                    if (PREK && k == K - 1 && dom && lx >= HL && lx < HL + BX && ly >= HL && ly < HL + BY)
                        a.u_out[vid(vxc, vy)] = val;
                }
            }
        }
        if (!last || RST) __syncthreads();
    }
    if (RST) {
        // fc[X] = sum of P[v][X] r[v] over the 3 x 3 fine vertices around 2X,
        // for the tile's coarse vertices X in [x0/2, x0/2 + BX/2) x [y0/2, y0/2 + BY/2)
        const T(*R)[UW] = sU1;
        constexpr int CW = BX / 2;
        const int nc = n / 2;
        if (tid < CW * (BY / 2)) {
            const int cx = tid % CW, cy = tid / CW;
            const int X = x0 / 2 + cx, Y = y0 / 2 + cy;
            if (X <= nc && Y <= nc) {
                T fc = (T)0;
                if (X > 0 && X < nc && Y > 0 && Y < nc) {
#pragma unroll
                    for (int sv = 0; sv < 9; ++sv) {
                        const int ox = sv % 3 - 1, oy = sv / 3 - 1;
                        fc += wres[sv] * R[HL + 2 * cy + oy][HL + 2 * cx + ox];
                    }
                }
                a.r_out[(uint32_t)Y * (uint32_t)(nc + 1) + (uint32_t)X] = fc;
            }
        }
    }
    if (DOTS) {
        double sa = lev2_block_sum(pa, red), sb = lev2_block_sum(pb, red);
        if (tid == 0) {
            a.partial[tile] = sa;
            a.partial[(int64_t)nt + tile] = sb;
        }
    }
    if (PMV) {
        double sa = lev2_block_sum(pa, red);
        if (tid == 0) a.partial[tile] = sa;
    }
}

// ------------------------------------------------------------ host side
StoreView store_view(const mgd_hier *h, const OpSet &o);


// tiles of a level: 60 (pre half) or 62 (post half) columns by `by` rows
static int lev2_tiles(int n, int kind, int by)
{
    int nv = n + 1, bx = kind == L2_PRE ? 60 : kind == L2_POST ? 62 : kind == L2_PRER ? 58 : 64;
    return ((nv + bx - 1) / bx) * ((nv + by - 1) / by);
}
static dim3 lev2_grid(int n, int kind, int by)
{
    int nt = lev2_tiles(n, kind, by);
    return dim3((unsigned)(8 * ((nt + 7) / 8)));
}

// tile heights: 16 rows in FP32 (about 50 KB of LDS), 8 in FP64
constexpr int kBYf = 16, kBYd = 8;

// The mixed form's finest level: the fused kernels decode the compressed
// store when the level is large enough to stream from HBM, where its fewer
// bytes set the pace.  Smaller levels stay in the 256 MB Infinity Cache
// between passes, the kernels are bound by vector instructions there, and
// they read the FP32 copy of the same operator (the store's decode, kept
// current beside it) instead of decoding per pass.  Either way the tile's
// operator in LDS holds the same values, so the results agree bit for bit.
constexpr int64_t kStoreMinNV = (int64_t)1 << 22;
static bool lev2_store(const mgd_hier *h, int l)
{
    if (h->precision != MGD_MIXED || l != 0) return false;
    if (h->store_path == MGD_STORE_AUTO) return h->NV[0] >= kStoreMinNV;
    return h->store_path == MGD_STORE_DECODE;
}

// 2D, V(2,2), a coarser level below, and 32-bit indices into [4][NV] arrays
bool lev2_ok(const mgd_hier *h, int l, int nu1, int nu2)
{
    return h->dim == 2 && nu1 == 2 && nu2 == 2 && l < h->nlev - 1 && h->NV[l] * 4 < ((int64_t)1 << 31);
}

template <typename T, int BY>
static int lev2_pre_t(mgd_hier *h, const OpSet &o, int l, const T *u, const T *f, T *u_out, T *r_out, double omega,
                      hipStream_t st)
{
    Lev2Args<T> a;
    memset(&a, 0, sizeof(a));
    const bool comp = lev2_store(h, l);
    if (comp) a.sv = store_view(h, o);
    else a.S = (const T *)(h->precision == MGD_FP64 ? (const void *)o.S64[l] : (const void *)o.S32[l]);
    a.n = h->nl[l];
    a.u = u;
    a.f = f;
    a.u_out = u_out;
    a.r_out = r_out;
    a.omega = (T)omega;
    dim3 g = lev2_grid(a.n, L2_PRE, BY);
    if (comp) {
        if (!u) hipLaunchKernelGGL((k_lev2<T, BY, L2_PRE, true, true, false>), g, dim3(256), 0, st, a);
        else hipLaunchKernelGGL((k_lev2<T, BY, L2_PRE, true, false, false>), g, dim3(256), 0, st, a);
    } else {
        if (!u) hipLaunchKernelGGL((k_lev2<T, BY, L2_PRE, false, true, false>), g, dim3(256), 0, st, a);
        else hipLaunchKernelGGL((k_lev2<T, BY, L2_PRE, false, false, false>), g, dim3(256), 0, st, a);
    }
    HIPCHK(h->ctx, hipGetLastError());
    return MGD_OK;
}

template <typename T, int BY>
static int lev2_post_t(mgd_hier *h, const OpSet &o, int l, const T *u, const T *ec, const T *f, T *u_out,
                       double omega, const Lev2Dots *dots, hipStream_t st)
{
    Lev2Args<T> a;
    memset(&a, 0, sizeof(a));
    const bool comp = lev2_store(h, l);
    if (comp) a.sv = store_view(h, o);
    else a.S = (const T *)(h->precision == MGD_FP64 ? (const void *)o.S64[l] : (const void *)o.S32[l]);
    a.n = h->nl[l];
    a.u = u;
    a.ec = ec;
    a.f = f;
    a.u_out = u_out;
    a.W = h->transfer == MGD_BOXMG ? (const T *)o.W[l] : nullptr;
    a.omega = (T)omega;
    dim3 g = lev2_grid(a.n, L2_POST, BY);
    if (dots) {
        a.r64 = dots->r;
        a.rold64 = dots->rold;
        a.partial = h->partial;
        if (comp) hipLaunchKernelGGL((k_lev2<T, BY, L2_POST, true, false, true>), g, dim3(256), 0, st, a);
        else hipLaunchKernelGGL((k_lev2<T, BY, L2_POST, false, false, true>), g, dim3(256), 0, st, a);
        HIPCHK(h->ctx, hipGetLastError());
        // the partials feed the CG matrix-vector kernel, whose every block adds
        // them: long lists (large grids) are first summed to one pair
        const int nt = lev2_tiles(a.n, L2_POST, BY);
        h->p1 = h->partial;
        h->p1_n = nt;
        if (nt > 2048) {
            int rc = compress_partials(h, h->partial, nt, 2, h->scal + 16, st);
            if (rc) return rc;
            h->p1 = h->scal + 16;
            h->p1_n = 1;
        }
        return MGD_OK;
    } else {
        if (comp) hipLaunchKernelGGL((k_lev2<T, BY, L2_POST, true, false, false>), g, dim3(256), 0, st, a);
        else hipLaunchKernelGGL((k_lev2<T, BY, L2_POST, false, false, false>), g, dim3(256), 0, st, a);
    }
    HIPCHK(h->ctx, hipGetLastError());
    return MGD_OK;
}

// CG matrix-vector product on the finest level (2D, FP64): p_new = z + beta
// p_old, Ap = A p_new, one partial of p.Ap per tile into h->partial2
int lev2_pmv(mgd_hier *h, const OpSet &o, const void *z, const double *pold, double *pnew, double *Ap,
             const CgScalars &c, hipStream_t st)
{
    constexpr int BY = 16;
    Lev2Args<double> a;
    memset(&a, 0, sizeof(a));
    const bool mixed = h->precision == MGD_MIXED, comp = lev2_store(h, 0);
    if (comp) a.sv = store_view(h, o);
    else if (mixed) a.Sf = (const float *)o.S32[0];
    else a.S = o.S64[0];
    a.n = h->nl[0];
    a.z = z;
    a.pold = pold;
    a.pnew = pnew;
    a.Ap = Ap;
    a.cg = c;
    a.partial = h->partial2;
    dim3 g = lev2_grid(a.n, L2_PMV, BY);
    if (comp) hipLaunchKernelGGL((k_lev2<double, BY, L2_PMV, true, false, false, true>), g, dim3(256), 0, st, a);
    else if (mixed) hipLaunchKernelGGL((k_lev2<double, BY, L2_PMV, false, false, false, true>), g, dim3(256), 0, st, a);
    else hipLaunchKernelGGL((k_lev2<double, BY, L2_PMV, false, false, false, false>), g, dim3(256), 0, st, a);
    HIPCHK(h->ctx, hipGetLastError());
    h->p2_n = lev2_tiles(a.n, L2_PMV, BY);
    return MGD_OK;
}

// pre half with the restriction: u_out = S^2 u, fc = P^T (f - A u_out) on the coarser level
template <typename T, int BY>
static int lev2_prer_t(mgd_hier *h, const OpSet &o, int l, const T *u, const T *f, T *u_out, T *fc, double omega,
                       hipStream_t st)
{
    Lev2Args<T> a;
    memset(&a, 0, sizeof(a));
    const bool comp = lev2_store(h, l);
    if (comp) a.sv = store_view(h, o);
    else a.S = (const T *)(h->precision == MGD_FP64 ? (const void *)o.S64[l] : (const void *)o.S32[l]);
    a.n = h->nl[l];
    a.u = u;
    a.f = f;
    a.u_out = u_out;
    a.r_out = fc;
    a.W = h->transfer == MGD_BOXMG ? (const T *)o.W[l] : nullptr;
    a.ec = f;  // any valid address for the weight loads that are not needed (d-linear)
    a.omega = (T)omega;
    dim3 g = lev2_grid(a.n, L2_PRER, BY);
    if (comp) {
        if (!u) hipLaunchKernelGGL((k_lev2<T, BY, L2_PRER, true, true, false>), g, dim3(256), 0, st, a);
        else hipLaunchKernelGGL((k_lev2<T, BY, L2_PRER, true, false, false>), g, dim3(256), 0, st, a);
    } else {
        if (!u) hipLaunchKernelGGL((k_lev2<T, BY, L2_PRER, false, true, false>), g, dim3(256), 0, st, a);
        else hipLaunchKernelGGL((k_lev2<T, BY, L2_PRER, false, false, false>), g, dim3(256), 0, st, a);
    }
    HIPCHK(h->ctx, hipGetLastError());
    return MGD_OK;
}

int lev2_prer(mgd_hier *h, const OpSet &o, int l, const void *u, const void *f, void *u_out, void *fc, double omega,
              hipStream_t st)
{
    if (h->precision == MGD_FP64)
        return lev2_prer_t<double, kBYd>(h, o, l, (const double *)u, (const double *)f, (double *)u_out,
                                         (double *)fc, omega, st);
    return lev2_prer_t<float, kBYf>(h, o, l, (const float *)u, (const float *)f, (float *)u_out, (float *)fc, omega,
                                    st);
}

int lev2_pre(mgd_hier *h, const OpSet &o, int l, const void *u, const void *f, void *u_out, void *r_out,
             double omega, hipStream_t st)
{
    if (h->precision == MGD_FP64)
        return lev2_pre_t<double, kBYd>(h, o, l, (const double *)u, (const double *)f, (double *)u_out,
                                        (double *)r_out, omega, st);
    return lev2_pre_t<float, kBYf>(h, o, l, (const float *)u, (const float *)f, (float *)u_out, (float *)r_out,
                                   omega, st);
}

int lev2_post(mgd_hier *h, const OpSet &o, int l, const void *u, const void *ec, const void *f, void *u_out,
              double omega, const Lev2Dots *dots, hipStream_t st)
{
    if (h->precision == MGD_FP64)
        return lev2_post_t<double, kBYd>(h, o, l, (const double *)u, (const double *)ec, (const double *)f,
                                         (double *)u_out, omega, dots, st);
    return lev2_post_t<float, kBYf>(h, o, l, (const float *)u, (const float *)ec, (const float *)f, (float *)u_out,
                                    omega, dots, st);
}
