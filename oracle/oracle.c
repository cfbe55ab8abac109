/*
 * oracle.c -- plain, slow, FP64 reference of delayed approximate matrix
 * assembly in multigrid (Murray & Weinzierl, "Delayed approximate matrix
 * assembly in multigrid with dynamic precisions", arXiv:2005.03606).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark load this file.  It shares no code, table
 * or constant with the HIP library and includes none of its headers.
 *
 * Everything is written as the plain definition, in FP64, with no blocking,
 * fusion or reordering:
 *   - element matrices: Sec. 4.2 eq. (mg:weak-form-of-assembly), eps held
 *     constant on each of the s^d equal sub-cells, sampled at the sub-cell
 *     midpoint, the gradient product integrated exactly on each sub-cell;
 *   - adaptive sample ladder: Sec. 5.2, eq. (termination criterion) with the
 *     doubling ladder s = 1, 2, 4, 8, 16;
 *   - stencils: Sec. 4 (a stencil is one row of A_h, 9 / 27 points);
 *   - hierarchical surplus and reduced-precision storage: Sec. 5.5;
 *   - Galerkin coarse operators A_{l-1} = R A_l P, d-linear P, R = P^T: Sec. 4;
 *   - damped Jacobi S = omega diag^{-1}(A): Sec. 4.1;
 *   - multiplicative correction-scheme V(nu1,nu2) and the normalised-residual
 *     stopping rule: Sec. 4 and Sec. 6.
 *
 * Index conventions (shared with the HIP path only as a documented layout):
 *   cell c = i + N (j + N k), vertex v = i + (N+1)(j + (N+1)k), x fastest;
 *   local vertex a of a cell has bit m = offset along axis m;
 *   stencil offset o in {-1,0,1}^d has index sum_m (o_m+1) 3^m.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define MAXLEV 24

/* ------------------------------------------------------------ materials */
enum { F_CONST = 0, F_SINE = 1, F_THETA = 2, F_BALLS = 3, F_LATTICE = 4, F_BOXES = 5 };

typedef struct {
    int32_t kind, dim, count, pad;
    double p0, p1;
    const double *data;
} orc_field;

/* eps at point x (the material laws are listed in the input generator) */
double orc_eps(const orc_field *f, const double *x)
{
    int d = f->dim;
    if (f->kind == F_CONST)
        return f->p0;
    if (f->kind == F_SINE) {
        double p = 1.0;
        for (int m = 0; m < d; ++m)
            p *= sin(2.0 * M_PI * x[m]);
        return 1.0 + f->p0 * p;
    }
    if (f->kind == F_THETA) {
        /* Sec. 6, eq. (results:theta-setup) */
        double p = 1.0, th = f->p0;
        for (int m = 0; m < d; ++m)
            p *= exp(-th * x[m]) * cos(M_PI * th * x[m]);
        return 1.0 + (0.3 / d) * p;
    }
    if (f->kind == F_BALLS) {
        for (int b = 0; b < f->count; ++b) {
            const double *row = f->data + (size_t)b * (d + 1);
            double r2 = 0.0;
            for (int m = 0; m < d; ++m) {
                double dx = x[m] - row[m];
                r2 += dx * dx;
            }
            if (r2 <= row[d] * row[d])
                return f->p1;
        }
        return f->p0;
    }
    if (f->kind == F_LATTICE) {
        /* d-linear interpolation of lattice values, spacing 1/L */
        int L = f->count;
        int base[3];
        double t[3];
        for (int m = 0; m < d; ++m) {
            double y = x[m] * L;
            int i = (int)floor(y);
            if (i < 0) i = 0;
            if (i > L - 1) i = L - 1;
            base[m] = i;
            t[m] = y - i;
        }
        double g = 0.0;
        for (int a = 0; a < (1 << d); ++a) {
            double w = 1.0;
            int64_t idx = 0, stride = 1;
            for (int m = 0; m < d; ++m) {
                int bit = (a >> m) & 1;
                w *= bit ? t[m] : 1.0 - t[m];
                idx += (int64_t)(base[m] + bit) * stride;
                stride *= (L + 1);
            }
            g += w * f->data[idx];
        }
        return exp(f->p0 * g);
    }
    if (f->kind == F_BOXES) {
        double e = f->p0;
        for (int b = 0; b < f->count; ++b) {
            const double *row = f->data + (size_t)b * (2 * d + 1);
            int in = 1;
            for (int m = 0; m < d; ++m)
                if (!(x[m] >= row[m] && x[m] < row[d + m]))
                    in = 0;
            if (in)
                e = row[2 * d];
        }
        return e;
    }
    return NAN;
}

/* ----------------------------------------------- sub-cell matrices G_q */
/* 1D integrals over the sub-interval [q/s, (q+1)/s] of the reference axis:
 * M[a][b] = int psi_a psi_b, psi_0 = 1 - xi, psi_1 = xi (exact rationals);
 * the derivative product psi_a' psi_b' = sigma_a sigma_b integrates to
 * sigma_a sigma_b / s.                                                   */
static void moments(int s, int q, double M[2][2])
{
    double S3 = (double)s * s * s;
    int qb = s - 1 - q;
    M[1][1] = (3.0 * q * q + 3.0 * q + 1.0) / (3.0 * S3);
    M[0][0] = (3.0 * qb * qb + 3.0 * qb + 1.0) / (3.0 * S3);
    M[0][1] = M[1][0] = (6.0 * q * (s - q) + 3.0 * (s - 2.0 * q) - 2.0) / (6.0 * S3);
}

/* G_q[a][b] = int over sub-cell q of grad phi_a . grad phi_b
 *           = h^{d-2} sum_k (sigma sigma / s)_k prod_{m != k} M_{q_m}      */
void orc_subcell_matrix(int d, int s, const int32_t *q, double h, double *G)
{
    int nl = 1 << d;
    double M[3][2][2];
    for (int m = 0; m < d; ++m)
        moments(s, q[m], M[m]);
    double hp = (d == 2) ? 1.0 : h;
    for (int a = 0; a < nl; ++a)
        for (int b = 0; b < nl; ++b) {
            double sum = 0.0;
            for (int k = 0; k < d; ++k) {
                int ak = (a >> k) & 1, bk = (b >> k) & 1;
                double term = ((ak == bk) ? 1.0 : -1.0) / s;
                for (int m = 0; m < d; ++m) {
                    if (m == k) continue;
                    term *= M[m][(a >> m) & 1][(b >> m) & 1];
                }
                sum += term;
            }
            G[a * nl + b] = hp * sum;
        }
}

/* ------------------------------------------------------ element matrix */
static void cell_coords(int d, int N, int64_t c, int *ci)
{
    for (int m = 0; m < d; ++m) {
        ci[m] = (int)(c % N);
        c /= N;
    }
}

/* K_c(s) = sum_q eps(x_q) G_q, q = qx + s (qy + s qz) ascending,
 * x_q = ((i + (q_x + 1/2)/s) / N, ...).  Sec. 4.2: n^d sub-volumes with
 * eps constant on each; s = 1 is the single centre sample.               */
void orc_element_matrix(const orc_field *f, int d, int N, int s, int64_t c, double *K)
{
    int nl = 1 << d, ci[3];
    cell_coords(d, N, c, ci);
    int64_t nq = 1;
    for (int m = 0; m < d; ++m) nq *= s;
    double h = 1.0 / N, G[64];
    memset(K, 0, sizeof(double) * nl * nl);
    for (int64_t qq = 0; qq < nq; ++qq) {
        int32_t q[3];
        int64_t t = qq;
        double x[3];
        for (int m = 0; m < d; ++m) {
            q[m] = (int32_t)(t % s);
            t /= s;
            x[m] = ((double)ci[m] + ((double)q[m] + 0.5) / (double)s) / (double)N;
        }
        double e = orc_eps(f, x);
        orc_subcell_matrix(d, s, q, h, G);
        for (int i = 0; i < nl * nl; ++i)
            K[i] += e * G[i];
    }
}

/* same, with eps samples given: eps_q[q] for q ascending */
void orc_element_matrix_samples(int d, int N, int s, const double *eps_q, double *K)
{
    int nl = 1 << d;
    int64_t nq = 1;
    for (int m = 0; m < d; ++m) nq *= s;
    double h = 1.0 / N, G[64];
    memset(K, 0, sizeof(double) * nl * nl);
    for (int64_t qq = 0; qq < nq; ++qq) {
        int32_t q[3];
        int64_t t = qq;
        for (int m = 0; m < d; ++m) {
            q[m] = (int32_t)(t % s);
            t /= s;
        }
        orc_subcell_matrix(d, s, q, h, G);
        for (int i = 0; i < nl * nl; ++i)
            K[i] += eps_q[qq] * G[i];
    }
}

void orc_assemble(const orc_field *f, int d, int N, int s, const int64_t *cells, int64_t n, double *K)
{
    int nl = 1 << d;
    for (int64_t i = 0; i < n; ++i)
        orc_element_matrix(f, d, N, s, cells ? cells[i] : i, K + (size_t)i * nl * nl);
}

static double maxabs(const double *a, int n)
{
    double m = 0.0;
    for (int i = 0; i < n; ++i)
        if (fabs(a[i]) > m) m = fabs(a[i]);
    return m;
}

/* Sec. 5.2: start from the centre sample (s = 1); at each step integrate
 * with the next sample count, compare new and old element matrix in the
 * element-wise max norm relative to the old one; below C the cell is done
 * (keep the new matrix), otherwise go on; the last rung s_max ends it.
 * Returns the final s; rel[k] = relative change at rung k (k = 0 for s = 2). */
int orc_ladder_cell(const orc_field *f, int d, int N, int64_t c, int s_max, double C,
                    double *K, double *rel)
{
    int nl = 1 << d, nn = nl * nl;
    double Kn[64];
    orc_element_matrix(f, d, N, 1, c, K);
    int s = 1, k = 0;
    for (int m = 2; m <= s_max; m *= 2, ++k) {
        orc_element_matrix(f, d, N, m, c, Kn);
        double diff[64];
        for (int i = 0; i < nn; ++i)
            diff[i] = Kn[i] - K[i];
        double r = maxabs(diff, nn) / maxabs(K, nn);
        if (rel) rel[k] = r;
        memcpy(K, Kn, sizeof(double) * nn);
        s = m;
        if (r < C)
            break;
    }
    return s;
}

void orc_ladder(const orc_field *f, int d, int N, int s_max, double C, double *K,
                int32_t *s_final, double *rel /* [cells][4] or NULL */)
{
    int64_t nc = 1;
    int nl = 1 << d;
    for (int m = 0; m < d; ++m) nc *= N;
    for (int64_t c = 0; c < nc; ++c)
        s_final[c] = orc_ladder_cell(f, d, N, c, s_max, C, K + (size_t)c * nl * nl,
                                     rel ? rel + c * 4 : NULL);
}

static int64_t npow(int n, int d);

/* The paper's own ladder (Sec. 5.2) as its memory-footprint table applies
 * it (Sec. 6.3): a cell goes from n to n + 1 samples per axis while the
 * element matrix changes by C or more (relative to the old matrix, max
 * norm); once a step changes it by less than C the cell keeps the matrix it
 * had (the table's smooth case stores nothing beyond the n = 1 matrix);
 * n_max ends it.  Returns the final n; rel[k] is the change at the step
 * n = k + 1 -> k + 2.                                                       */
int orc_ladder_cell_inc(const orc_field *f, int d, int N, int64_t c, int n_max, double C, double *K, double *rel)
{
    int nl = 1 << d, nn = nl * nl;
    double Kn[64];
    orc_element_matrix(f, d, N, 1, c, K);
    int s = 1;
    for (int m = 2; m <= n_max; ++m) {
        orc_element_matrix(f, d, N, m, c, Kn);
        double diff[64];
        for (int i = 0; i < nn; ++i)
            diff[i] = Kn[i] - K[i];
        double r = maxabs(diff, nn) / maxabs(K, nn);
        if (rel) rel[m - 2] = r;
        if (r < C)
            break;
        memcpy(K, Kn, sizeof(double) * nn);
        s = m;
    }
    return s;
}

/* ----------------------------------------- the paper's truncated format */
/* Sec. 5.5: a datum in p bytes (2 <= p < 8) holds a sign bit, the leading
 * m = 8 (p - 1) - 1 bits of the IEEE double's 52-bit fraction (truncated,
 * the leading 1 implied) and one byte with the unbiased exponent as a
 * signed char, clamped to [-128, 127]; p = 8 is the double itself.  Zero
 * has no exponent: it is kept exact here (exponent byte -128, fraction 0,
 * and a decoder that maps that pattern to 0).                              */
void orc_p3_encode(double x, int p, uint8_t *out)
{
    if (p >= 8) { memcpy(out, &x, 8); return; }
    uint64_t b;
    memcpy(&b, &x, 8);
    int sign = (int)(b >> 63);
    int eb = (int)((b >> 52) & 0x7ff);
    uint64_t frac = b & ((1ull << 52) - 1);
    int e = eb - 1023;
    if (x == 0.0) { e = -128; frac = 0; }
    if (e < -128) e = -128;
    if (e > 127) e = 127;
    int m = 8 * (p - 1) - 1;
    uint64_t mt = frac >> (52 - m);                     /* truncation */
    uint64_t word = ((uint64_t)sign << m) | mt;         /* p - 1 bytes */
    for (int k = 0; k < p - 1; ++k) out[k] = (uint8_t)(word >> (8 * k));
    out[p - 1] = (uint8_t)(int8_t)e;
}

double orc_p3_decode(const uint8_t *in, int p)
{
    if (p >= 8) { double x; memcpy(&x, in, 8); return x; }
    int m = 8 * (p - 1) - 1;
    uint64_t word = 0;
    for (int k = 0; k < p - 1; ++k) word |= (uint64_t)in[k] << (8 * k);
    int sign = (int)(word >> m) & 1;
    uint64_t mt = word & ((1ull << m) - 1);
    int e = (int8_t)in[p - 1];
    if (e == -128 && mt == 0) return sign ? -0.0 : 0.0;
    double v = ldexp(1.0 + ldexp((double)mt, -m), e);
    return sign ? -v : v;
}

/* bytes per entry for one cell's surplus (K - K(1)), Sec. 5.5: 0 (only the
 * marker) when the surplus' Frobenius norm is below tau, else the fewest
 * bytes p in 2..8 whose truncation error stays within tau in every entry  */
int orc_p3_choose(const double *surplus, int nn, double tau)
{
    double fro = 0.0;
    for (int i = 0; i < nn; ++i) fro += surplus[i] * surplus[i];
    if (sqrt(fro) < tau) return 0;
    for (int p = 2; p < 8; ++p) {
        double err = 0.0;
        uint8_t buf[8];
        for (int i = 0; i < nn; ++i) {
            orc_p3_encode(surplus[i], p, buf);
            double dd = fabs(orc_p3_decode(buf, p) - surplus[i]);
            if (dd > err) err = dd;
        }
        if (err <= tau) return p;
    }
    return 8;
}

/* Table memory-footprint of Sec. 6.3 for the paper's ladder, published one
 * rung per cycle: in cycle k (k = 2 .. cycles) every unfinished cell tries
 * n = k and keeps it unless it changed the matrix by less than C (then the
 * cell is done with n = k - 1); out[k-1] = {max n, mean n, compression},
 * compression =
 * 2^d 2^d 8 bytes per cell over (1 marker byte + 2^d 2^d p bytes of its
 * surplus over the n = 1 matrix) summed over the cells.                   */
void orc_paper_table(const orc_field *f, int d, int N, double C, double tau, int cycles, double *out)
{
    int nl = 1 << d, nn = nl * nl;
    int64_t nc = npow(N, d);
    double *K = malloc(sizeof(double) * nc * nn), *K1 = malloc(sizeof(double) * nc * nn);
    int *n = malloc(sizeof(int) * nc);
    uint8_t *done = malloc(nc);
    for (int64_t c = 0; c < nc; ++c) {
        orc_element_matrix(f, d, N, 1, c, K1 + c * nn);
        memcpy(K + c * nn, K1 + c * nn, sizeof(double) * nn);
        n[c] = 1;
        done[c] = 0;
    }
    for (int k = 1; k <= cycles; ++k) {
        if (k >= 2)
            for (int64_t c = 0; c < nc; ++c) {
                if (done[c]) continue;
                double Kn[64], diff[64];
                orc_element_matrix(f, d, N, k, c, Kn);
                for (int i = 0; i < nn; ++i) diff[i] = Kn[i] - K[c * nn + i];
                double r = maxabs(diff, nn) / maxabs(K + c * nn, nn);
                if (r < C) { done[c] = 1; continue; }  /* keeps K(k - 1) */
                memcpy(K + c * nn, Kn, sizeof(double) * nn);
                n[c] = k;
            }
        int nmax = 0;
        double nsum = 0.0, bytes = 0.0;
        for (int64_t c = 0; c < nc; ++c) {
            double sur[64];
            for (int i = 0; i < nn; ++i) sur[i] = K[c * nn + i] - K1[c * nn + i];
            int p = orc_p3_choose(sur, nn, tau);
            bytes += 1.0 + (double)nn * p;
            if (n[c] > nmax) nmax = n[c];
            nsum += n[c];
        }
        out[3 * (k - 1)] = nmax;
        out[3 * (k - 1) + 1] = nsum / nc;
        out[3 * (k - 1) + 2] = (double)nc * nn * 8.0 / bytes;
    }
    free(K); free(K1); free(n); free(done);
}

/* ------------------------------------------------------------ stencils */
static int64_t npow(int n, int d)
{
    int64_t r = 1;
    for (int m = 0; m < d; ++m) r *= n;
    return r;
}

static int nst(int d) { return d == 2 ? 9 : 27; }

static void offset_of(int d, int idx, int *o)
{
    for (int m = 0; m < d; ++m) {
        o[m] = idx % 3 - 1;
        idx /= 3;
    }
}

/* Full stencils a_v[o] = sum over cells c holding both v and v+o of
 * K_c[loc(v)][loc(v+o)], cells taken in ascending index.  S: [(N+1)^d][3^d]. */
void orc_stencils(int d, int N, const double *K, double *S)
{
    int nl = 1 << d, ns = nst(d), nv = N + 1;
    int64_t NV = npow(nv, d);
    for (int64_t v = 0; v < NV; ++v) {
        int vi[3];
        int64_t t = v;
        for (int m = 0; m < d; ++m) { vi[m] = (int)(t % nv); t /= nv; }
        for (int oi = 0; oi < ns; ++oi) {
            int o[3];
            offset_of(d, oi, o);
            double a = 0.0;
            for (int B = nl - 1; B >= 0; --B) { /* ascending cell index */
                int ok = 1, lv = 0, lw = 0;
                int64_t c = 0, stride = 1;
                for (int m = 0; m < d; ++m) {
                    int bm = (B >> m) & 1;
                    int cm = vi[m] - bm;
                    int wm = bm + o[m];
                    if (cm < 0 || cm >= N || wm < 0 || wm > 1) { ok = 0; break; }
                    lv |= bm << m;
                    lw |= wm << m;
                    c += (int64_t)cm * stride;
                    stride *= N;
                }
                if (ok)
                    a += K[(size_t)c * nl * nl + lv * nl + lw];
            }
            S[(size_t)v * ns + oi] = a;
        }
    }
}

/* Hierarchical surplus base of Sec. 5.5: the stencil coupling assembled from
 * the centre-sample element matrices eps_c K_ref (K_ref: unit-eps Q1 matrix).
 * Off-diagonal couplings of the unit matrix depend only on how many axes two
 * local vertices differ in: 2D -1/6 (one), -1/3 (two); 3D (times h)
 * 0 (one), -1/12 (two), -1/12 (three).  The base coupling for offset o is
 *   ((sum of eps_c over the cells holding v and v+o, ascending) * k(o)) * h^{d-2},
 * evaluated in FP64 in exactly this order.  ref_v = (sum of eps_c over all
 * cells around v, ascending) * h^{d-2} is the magnitude that scales the
 * allowed storage error.                                                  */
static double kref_unit(int d, int nz)
{
    if (d == 2) return nz == 1 ? -1.0 / 6.0 : -1.0 / 3.0;
    return nz == 1 ? 0.0 : -1.0 / 12.0;
}

void orc_base_coupling(int d, int N, const float *eps_c, int64_t v, int oi, double *base, double *ref)
{
    int nv = N + 1, vi[3], o[3], nz = 0;
    int64_t t = v;
    for (int m = 0; m < d; ++m) { vi[m] = (int)(t % nv); t /= nv; }
    offset_of(d, oi, o);
    for (int m = 0; m < d; ++m) nz += o[m] != 0;
    double hp = (d == 2) ? 1.0 : 1.0 / N;
    double sum = 0.0, sall = 0.0;
    for (int B = (1 << d) - 1; B >= 0; --B) {
        int ok = 1, shared = 1;
        int64_t c = 0, stride = 1;
        for (int m = 0; m < d; ++m) {
            int bm = (B >> m) & 1, cm = vi[m] - bm, wm = bm + o[m];
            if (cm < 0 || cm >= N) { ok = 0; break; }
            if (wm < 0 || wm > 1) shared = 0;
            c += (int64_t)cm * stride;
            stride *= N;
        }
        if (!ok) continue;
        sall += (double)eps_c[c];
        if (shared) sum += (double)eps_c[c];
    }
    if (base) *base = (sum * kref_unit(d, nz)) * hp;
    if (ref) *ref = sall * hp;
}

/* ------------------------------------------- reduced-precision encoding */
/* Round x to the nearest value of a binary floating format with `mbits`
 * stored mantissa bits and minimum normal exponent emin (subnormals below),
 * ties to even.  Returns the rounded value (no overflow handling). */
static double round_format(double x, int mbits, int emin)
{
    if (x == 0.0) return x;
    int e;
    frexp(fabs(x), &e); /* |x| = m 2^e, m in [0.5,1): exponent of leading bit is e-1 */
    int E = e - 1;
    if (E < emin) E = emin;
    double spacing = ldexp(1.0, E - mbits);
    return rint(x / spacing) * spacing; /* rint: round half to even */
}

/* IEEE binary16 bits of an exactly representable value */
static uint16_t half_bits(double v)
{
    uint16_t s = signbit(v) ? 0x8000 : 0;
    double a = fabs(v);
    if (a == 0.0) return s;
    int e;
    frexp(a, &e);
    int E = e - 1;
    if (E < -14) { /* subnormal: a = m 2^-24 */
        return s | (uint16_t)llrint(ldexp(a, 24));
    }
    uint16_t mant = (uint16_t)llrint((ldexp(a, -E) - 1.0) * 1024.0);
    return s | (uint16_t)((E + 15) << 10) | mant;
}

/* OCP FP8 E4M3FN bits (bias 7, 3 mantissa bits, max 448, no infinities) */
static uint8_t e4m3_bits(double v)
{
    uint8_t s = signbit(v) ? 0x80 : 0;
    double a = fabs(v);
    if (a == 0.0) return s;
    int e;
    frexp(a, &e);
    int E = e - 1;
    if (E < -6) return s | (uint8_t)llrint(ldexp(a, 9));
    uint8_t mant = (uint8_t)llrint((ldexp(a, -E) - 1.0) * 8.0);
    return s | (uint8_t)((E + 7) << 3) | mant;
}

double orc_half_value(uint16_t b)
{
    int s = b >> 15, E = (b >> 10) & 31, m = b & 1023;
    double v = (E == 0) ? ldexp((double)m, -24) : ldexp(1.0 + m / 1024.0, E - 15);
    return s ? -v : v;
}

double orc_e4m3_value(uint8_t b)
{
    int s = b >> 7, E = (b >> 3) & 15, m = b & 7;
    double v = (E == 0) ? ldexp((double)m, -9) : ldexp(1.0 + m / 8.0, E - 7);
    return s ? -v : v;
}

/* tiers: 0 nothing stored, 1 FP8 E4M3FN, 2 binary16, 3 binary32 */
static double tier_fmax(int tier) { return tier == 1 ? 448.0 : 65504.0; }

/* smallest e with maxabs <= fmax 2^e, clamped to the E8M0 range [-127,127] */
int orc_scale_exponent(double maxabs, int tier)
{
    if (!(maxabs > 0.0) || tier == 3) return 0;
    double fm = tier_fmax(tier);
    int e = ilogb(maxabs) - ilogb(fm) - 1;
    while (maxabs > ldexp(fm, e)) ++e;
    while (e > -127 && maxabs <= ldexp(fm, e - 1)) --e;
    if (e < -127) e = -127;
    if (e > 127) e = 127;
    return e;
}

/* quantised value (already multiplied back by the scale) of delta at a tier */
static double quantise(double delta, int tier, int e)
{
    if (tier == 0) return 0.0;
    if (tier == 3) return delta;
    double y = ldexp(delta, -e);
    double r = (tier == 2) ? round_format(y, 10, -14) : round_format(y, 3, -6);
    double fm = tier_fmax(tier);
    if (r > fm) r = fm;
    if (r < -fm) r = -fm;
    return ldexp(r, e);
}

/* Sec. 5.5: choose the cheapest tier whose maximum error over the stencil
 * stays within tau; below min_tier only the "store nothing" tier is tried. */
int orc_choose_tier(const float *delta, int H, double tau, int min_tier, int max_tier)
{
    double mx = 0.0;
    for (int j = 0; j < H; ++j)
        if (fabs((double)delta[j]) > mx) mx = fabs((double)delta[j]);
    if (mx <= tau) return 0;
    for (int t = min_tier; t <= max_tier; ++t) {
        if (t == 0) continue;
        int e = orc_scale_exponent(mx, t);
        double err = 0.0;
        for (int j = 0; j < H; ++j) {
            double q = quantise((double)delta[j], t, e);
            double dd = fabs(q - (double)delta[j]);
            if (dd > err) err = dd;
        }
        if (err <= tau) return t;
    }
    return max_tier;
}

/* encode one stencil's deltas at a given tier: returns the E8M0 byte and the
 * payload words (FP8 byte, binary16 bits or binary32 bits, per entry)      */
int orc_encode_stencil(const float *delta, int H, int tier, uint32_t *words)
{
    double mx = 0.0;
    for (int j = 0; j < H; ++j)
        if (fabs((double)delta[j]) > mx) mx = fabs((double)delta[j]);
    int e = orc_scale_exponent(mx, tier);
    for (int j = 0; j < H; ++j) {
        double q = quantise((double)delta[j], tier, e);
        if (tier == 1) words[j] = e4m3_bits(ldexp(q, -e));
        else if (tier == 2) words[j] = half_bits(ldexp(q, -e));
        else if (tier == 3) { float fv = delta[j]; memcpy(&words[j], &fv, 4); }
        else words[j] = 0;
    }
    return e + 127;
}

double orc_decode_entry(int tier, int e8, uint32_t word)
{
    if (tier == 0) return 0.0;
    if (tier == 3) { float fv; memcpy(&fv, &word, 4); return fv; }
    double v = (tier == 2) ? orc_half_value((uint16_t)word) : orc_e4m3_value((uint8_t)word);
    return ldexp(v, e8 - 127);
}

static int64_t vid(int d, int nv, const int *vi);

/* ------------------------------------------------- transfer operators P */
static double pw(int dlt) { return dlt == 0 ? 1.0 : (dlt == 1 || dlt == -1) ? 0.5 : 0.0; }

enum { T_GEOMETRIC = 0, T_BOXMG = 1 };

/* Prolongation weights of every fine vertex v toward the 2^d coarse vertices
 * (v_m >> 1) + B_m, B in {0,1}^d (B_m = 1 only matters on odd axes):
 * Pw[v][B].  Geometric: d-linear interpolation (Sec. 4).  BoxMG (Sec. 4,
 * "Rediscretisation ... vs Ritz-Galerkin plus algebraic operators"): an
 * operator-dependent interpolation that takes coarse values over unchanged,
 * and obtains every other fine value from its own stencil row, with the
 * stencil collapsed onto the sub-space (line, plane) that holds the point and
 * the coarse points it interpolates from; points with more odd coordinates use
 * the weights of points with fewer.  Fine boundary vertices keep d-linear
 * weights so that every interior coarse row keeps a zero row sum.          */
static void geometric_weights(int d, const int *vi, double *w)
{
    for (int B = 0; B < (1 << d); ++B) {
        double p = 1.0;
        for (int m = 0; m < d; ++m) {
            int V = (vi[m] >> 1) + ((B >> m) & 1);
            p *= pw(vi[m] - 2 * V);
        }
        w[B] = p;
    }
}

void orc_transfer_weights(int d, int nf, const double *Sf, int kind, double *Pw)
{
    int nv = nf + 1, ns = nst(d), nl = 1 << d;
    int64_t NV = npow(nv, d);
    /* pass k handles fine vertices with k odd coordinates */
    for (int k = 0; k <= d; ++k)
        for (int64_t v = 0; v < NV; ++v) {
            int vi[3], odd = 0, bnd = 0;
            int64_t t = v;
            for (int m = 0; m < d; ++m) {
                vi[m] = (int)(t % nv);
                t /= nv;
                odd += vi[m] & 1;
                if (vi[m] == 0 || vi[m] == nv - 1) bnd = 1;
            }
            if (odd != k) continue;
            double *w = Pw + (size_t)v * nl;
            if (kind == T_GEOMETRIC || bnd || k == 0) {
                geometric_weights(d, vi, w);
                continue;
            }
            /* row of v restricted to the odd axes: offsets along even axes are
             * summed (collapsed); each odd-axis neighbour u = v + o contributes
             * its own weights (already final: it has fewer odd coordinates,
             * or is a coarse vertex) */
            double acc[8] = {0}, diag = 0.0;
            for (int oi = 0; oi < ns; ++oi) {
                int o[3];
                offset_of(d, oi, o);
                double a = Sf[(size_t)v * ns + oi];
                int self = 1, ui[3];
                for (int m = 0; m < d; ++m) {
                    int om = (vi[m] & 1) ? o[m] : 0; /* collapse even axes */
                    ui[m] = vi[m] + om;
                    if (om != 0) self = 0;
                }
                if (self) { diag += a; continue; }
                const double *wu = Pw + (size_t)vid(d, nv, ui) * nl;
                /* map u's corner B' to v's corner B (same coarse box) */
                for (int Bu = 0; Bu < nl; ++Bu) {
                    if (wu[Bu] == 0.0) continue;
                    int B = 0;
                    for (int m = 0; m < d; ++m) {
                        int Vm = (ui[m] >> 1) + ((Bu >> m) & 1);
                        B |= (Vm - (vi[m] >> 1)) << m;
                    }
                    acc[B] -= a * wu[Bu];
                }
            }
            for (int B = 0; B < nl; ++B)
                w[B] = acc[B] / diag;
        }
}

/* ---------------------------------------------------- Galerkin: P^T A P */
/* Sec. 4: Ritz-Galerkin coarse operator A_{l-1} = R A_l P with R = P^T,
 * over the full vertex set (boundary vertices included, so that interior
 * rows keep zero row sums).  Sf: [(nf+1)^d][3^d], Sc: [(nf/2+1)^d][3^d].   */
void orc_galerkin(int d, int nf, const double *Sf, const double *Pw, double *Sc)
{
    int nc = nf / 2, ns = nst(d), nvf = nf + 1, nvc = nc + 1, nl = 1 << d;
    int64_t NVf = npow(nvf, d), NVc = npow(nvc, d);
    memset(Sc, 0, sizeof(double) * NVc * ns);
    for (int64_t v = 0; v < NVf; ++v) {
        int vi[3];
        int64_t t = v;
        for (int m = 0; m < d; ++m) { vi[m] = (int)(t % nvf); t /= nvf; }
        for (int Bv = 0; Bv < nl; ++Bv) {
            double pV = Pw[(size_t)v * nl + Bv];
            if (pV == 0.0) continue;
            int Vi[3], okV = 1;
            for (int m = 0; m < d; ++m) {
                Vi[m] = (vi[m] >> 1) + ((Bv >> m) & 1);
                if (Vi[m] >= nvc) okV = 0;
            }
            if (!okV) continue;
            for (int oi = 0; oi < ns; ++oi) {
                int o[3], wi[3], okw = 1;
                offset_of(d, oi, o);
                for (int m = 0; m < d; ++m) {
                    wi[m] = vi[m] + o[m];
                    if (wi[m] < 0 || wi[m] >= nvf) okw = 0;
                }
                if (!okw) continue;
                double a = Sf[(size_t)v * ns + oi];
                int64_t w = vid(d, nvf, wi);
                for (int Bw = 0; Bw < nl; ++Bw) {
                    double pW = Pw[(size_t)w * nl + Bw];
                    if (pW == 0.0) continue;
                    int so = 0, okW = 1, mul = 1;
                    for (int m = 0; m < d; ++m) {
                        int Wm = (wi[m] >> 1) + ((Bw >> m) & 1);
                        if (Wm >= nvc) okW = 0;
                        so += (Wm - Vi[m] + 1) * mul;
                        mul *= 3;
                    }
                    if (!okW) continue;
                    Sc[(size_t)vid(d, nvc, Vi) * ns + so] += pV * a * pW;
                }
            }
        }
    }
}

/* --------------------------------------------------- grid operations */
static int is_interior(int d, int nv, int64_t v, int *vi)
{
    int in = 1;
    for (int m = 0; m < d; ++m) {
        vi[m] = (int)(v % nv);
        v /= nv;
        if (vi[m] == 0 || vi[m] == nv - 1) in = 0;
    }
    return in;
}

static int64_t vid(int d, int nv, const int *vi)
{
    int64_t v = 0, stride = 1;
    for (int m = 0; m < d; ++m) { v += (int64_t)vi[m] * stride; stride *= nv; }
    return v;
}

/* (A u)_v over the full stencil */
static double apply_row(int d, int n, const double *S, const double *u, int64_t v)
{
    int nv = n + 1, ns = nst(d), vi[3];
    int64_t t = v;
    for (int m = 0; m < d; ++m) { vi[m] = (int)(t % nv); t /= nv; }
    double s = 0.0;
    for (int oi = 0; oi < ns; ++oi) {
        int o[3], wi[3], ok = 1;
        offset_of(d, oi, o);
        for (int m = 0; m < d; ++m) {
            wi[m] = vi[m] + o[m];
            if (wi[m] < 0 || wi[m] >= nv) ok = 0;
        }
        if (ok) s += S[(size_t)v * ns + oi] * u[vid(d, nv, wi)];
    }
    return s;
}

/* r = f - A u on interior vertices, 0 on the boundary */
void orc_residual(int d, int n, const double *S, const double *u, const double *f, double *r)
{
    int64_t NV = npow(n + 1, d);
    int vi[3];
    for (int64_t v = 0; v < NV; ++v)
        r[v] = is_interior(d, n + 1, v, vi) ? f[v] - apply_row(d, n, S, u, v) : 0.0;
}

/* one damped Jacobi sweep, Sec. 4.1: u_out = u + omega diag^{-1} (f - A u) */
void orc_jacobi(int d, int n, const double *S, const double *u, const double *f, double omega, double *u_out)
{
    int64_t NV = npow(n + 1, d);
    int vi[3], c = nst(d) / 2;
    for (int64_t v = 0; v < NV; ++v) {
        if (!is_interior(d, n + 1, v, vi)) { u_out[v] = 0.0; continue; }
        double r = f[v] - apply_row(d, n, S, u, v);
        u_out[v] = u[v] + omega * r / S[(size_t)v * nst(d) + c];
    }
}

/* restriction R = P^T onto interior coarse vertices (boundary rows 0) */
void orc_restrict(int d, int nf, const double *Pw, const double *r, double *fc)
{
    int nc = nf / 2, nvc = nc + 1, nvf = nf + 1, nl = 1 << d;
    int64_t NVc = npow(nvc, d), NVf = npow(nvf, d);
    memset(fc, 0, sizeof(double) * NVc);
    for (int64_t v = 0; v < NVf; ++v) {
        int vi[3];
        int64_t t = v;
        for (int m = 0; m < d; ++m) { vi[m] = (int)(t % nvf); t /= nvf; }
        for (int B = 0; B < nl; ++B) {
            double p = Pw[(size_t)v * nl + B];
            if (p == 0.0) continue;
            int Vi[3], ok = 1;
            for (int m = 0; m < d; ++m) {
                Vi[m] = (vi[m] >> 1) + ((B >> m) & 1);
                if (Vi[m] >= nvc) ok = 0;
            }
            if (ok) fc[vid(d, nvc, Vi)] += p * r[v];
        }
    }
    int Vi[3];
    for (int64_t V = 0; V < NVc; ++V)
        if (!is_interior(d, nvc, V, Vi)) fc[V] = 0.0;
}

/* u += P e on interior fine vertices */
void orc_prolong_add(int d, int nf, const double *Pw, const double *ec, double *u)
{
    int nvc = nf / 2 + 1, nvf = nf + 1, nl = 1 << d;
    int64_t NVf = npow(nvf, d);
    for (int64_t v = 0; v < NVf; ++v) {
        int vi[3];
        if (!is_interior(d, nvf, v, vi)) continue;
        double s = 0.0;
        for (int B = 0; B < nl; ++B) {
            double p = Pw[(size_t)v * nl + B];
            if (p == 0.0) continue;
            int Wi[3];
            for (int m = 0; m < d; ++m) Wi[m] = (vi[m] >> 1) + ((B >> m) & 1);
            s += p * ec[vid(d, nvc, Wi)];
        }
        u[v] += s;
    }
}

/* ---------------------------------------------------- dense coarse solve */
/* interior-interior dense matrix of a level, row-major [m][m] */
int64_t orc_dense_matrix(int d, int n, const double *S, double *A)
{
    int nv = n + 1, ns = nst(d);
    int64_t NV = npow(nv, d), m = npow(n - 1, d);
    int64_t *map = malloc(sizeof(int64_t) * NV);
    int64_t k = 0;
    int vi[3];
    for (int64_t v = 0; v < NV; ++v)
        map[v] = is_interior(d, nv, v, vi) ? k++ : -1;
    if (A) {
        memset(A, 0, sizeof(double) * m * m);
        for (int64_t v = 0; v < NV; ++v) {
            if (map[v] < 0) continue;
            is_interior(d, nv, v, vi);
            for (int oi = 0; oi < ns; ++oi) {
                int o[3], wi[3];
                offset_of(d, oi, o);
                for (int mm = 0; mm < d; ++mm) wi[mm] = vi[mm] + o[mm];
                int64_t w = vid(d, nv, wi);
                if (map[w] >= 0)
                    A[map[v] * m + map[w]] += S[(size_t)v * ns + oi];
            }
        }
    }
    free(map);
    return m;
}

/* Cholesky A = L L^T in place (lower triangle); returns 0 on success */
int orc_cholesky(int64_t m, double *A)
{
    for (int64_t j = 0; j < m; ++j) {
        double s = A[j * m + j];
        for (int64_t k = 0; k < j; ++k) s -= A[j * m + k] * A[j * m + k];
        if (!(s > 0.0)) return -1;
        double ljj = sqrt(s);
        A[j * m + j] = ljj;
        for (int64_t i = j + 1; i < m; ++i) {
            double t = A[i * m + j];
            for (int64_t k = 0; k < j; ++k) t -= A[i * m + k] * A[j * m + k];
            A[i * m + j] = t / ljj;
        }
    }
    return 0;
}

void orc_cholesky_solve(int64_t m, const double *L, double *b)
{
    for (int64_t i = 0; i < m; ++i) {
        double s = b[i];
        for (int64_t k = 0; k < i; ++k) s -= L[i * m + k] * b[k];
        b[i] = s / L[i * m + i];
    }
    for (int64_t i = m - 1; i >= 0; --i) {
        double s = b[i];
        for (int64_t k = i + 1; k < m; ++k) s -= L[k * m + i] * b[k];
        b[i] = s / L[i * m + i];
    }
}

/* ------------------------------------------------------------ hierarchy */
typedef struct {
    int d, nlev;
    int n[MAXLEV];
    double *S[MAXLEV];
    double *u[MAXLEV], *f[MAXLEV], *r[MAXLEV], *t[MAXLEV];
    double *Pw[MAXLEV]; /* weights of level l's vertices toward level l+1 */
    int transfer;
    double *L; /* Cholesky factor of the coarsest interior matrix */
    int64_t m;
    int64_t *imap; /* coarsest interior vertex list */
} orc_mg;

/* levels: n_0 = N, halve while even and n/2 >= coarsest */
static int level_count(int N, int coarsest)
{
    int k = 1, n = N;
    while (n % 2 == 0 && n / 2 >= coarsest && k < MAXLEV) { n /= 2; ++k; }
    return k;
}

static void mg_coarsen(orc_mg *g)
{
    for (int l = 1; l < g->nlev; ++l) {
        orc_transfer_weights(g->d, g->n[l - 1], g->S[l - 1], g->transfer, g->Pw[l - 1]);
        orc_galerkin(g->d, g->n[l - 1], g->S[l - 1], g->Pw[l - 1], g->S[l]);
    }
    int lc = g->nlev - 1, d = g->d, n = g->n[lc];
    free(g->L);
    g->m = orc_dense_matrix(d, n, g->S[lc], NULL);
    g->L = malloc(sizeof(double) * (g->m > 0 ? g->m * g->m : 1));
    orc_dense_matrix(d, n, g->S[lc], g->L);
    orc_cholesky(g->m, g->L);
}

orc_mg *orc_mg_create(int d, int N, int coarsest, int transfer, const double *S0)
{
    orc_mg *g = calloc(1, sizeof(orc_mg));
    g->d = d;
    g->transfer = transfer;
    g->nlev = level_count(N, coarsest);
    int n = N, ns = nst(d);
    for (int l = 0; l < g->nlev; ++l, n /= 2) {
        int64_t NV = npow(n + 1, d);
        g->n[l] = n;
        g->S[l] = calloc((size_t)NV * ns, sizeof(double));
        g->u[l] = calloc(NV, sizeof(double));
        g->f[l] = calloc(NV, sizeof(double));
        g->r[l] = calloc(NV, sizeof(double));
        g->t[l] = calloc(NV, sizeof(double));
        g->Pw[l] = calloc((size_t)NV << d, sizeof(double));
    }
    memcpy(g->S[0], S0, sizeof(double) * npow(N + 1, d) * ns);
    mg_coarsen(g);
    return g;
}

void orc_mg_set_fine(orc_mg *g, const double *S0)
{
    memcpy(g->S[0], S0, sizeof(double) * npow(g->n[0] + 1, g->d) * nst(g->d));
    mg_coarsen(g);
}

/* Geometric hierarchy of a provisional operator (Sec. 1: multigrid starts
 * from crude fine grid stencils with geometric coarse grid and inter-grid
 * transfer operators): S0 on the finest level; level l >= 1 is the Q1
 * rediscretisation whose cell values average the 2^d child cells' (the
 * finest level's: eps_c0, one value per fine cell, cell index x fastest);
 * d-linear transfer weights; the coarsest matrix factored as usual. */
void orc_mg_set_geometric(orc_mg *g, const double *S0, const double *eps_c0)
{
    int d = g->d, nl = 1 << d;
    memcpy(g->S[0], S0, sizeof(double) * npow(g->n[0] + 1, d) * nst(d));
    double *ef = malloc(sizeof(double) * npow(g->n[0], d));
    memcpy(ef, eps_c0, sizeof(double) * npow(g->n[0], d));
    for (int l = 1; l < g->nlev; ++l) {
        int nf = g->n[l - 1], nc = g->n[l];
        int64_t NC = npow(nc, d);
        orc_transfer_weights(d, nf, g->S[l - 1], T_GEOMETRIC, g->Pw[l - 1]);
        double *ec = malloc(sizeof(double) * NC);
        double *K = malloc(sizeof(double) * NC * nl * nl);
        double G[64];
        int32_t q0[3] = {0, 0, 0};
        orc_subcell_matrix(d, 1, q0, 1.0 / nc, G); /* unit-eps Q1 element matrix */
        for (int64_t c = 0; c < NC; ++c) {
            int X[3] = {0, 0, 0};
            int64_t t = c;
            for (int m = 0; m < d; ++m) { X[m] = (int)(t % nc); t /= nc; }
            double sum = 0.0;
            for (int B = 0; B < nl; ++B) {
                int64_t fi = 0, st = 1;
                for (int m = 0; m < d; ++m) {
                    fi += (int64_t)(2 * X[m] + ((B >> m) & 1)) * st;
                    st *= nf;
                }
                sum += ef[fi];
            }
            ec[c] = sum / nl;
            for (int i = 0; i < nl * nl; ++i) K[c * nl * nl + i] = ec[c] * G[i];
        }
        orc_stencils(d, nc, K, g->S[l]);
        free(K);
        free(ef);
        ef = ec;
    }
    free(ef);
    int lc = g->nlev - 1, n = g->n[lc];
    free(g->L);
    g->m = orc_dense_matrix(d, n, g->S[lc], NULL);
    g->L = malloc(sizeof(double) * (g->m > 0 ? g->m * g->m : 1));
    orc_dense_matrix(d, n, g->S[lc], g->L);
    orc_cholesky(g->m, g->L);
}

int orc_mg_levels(const orc_mg *g) { return g->nlev; }
int orc_mg_level_n(const orc_mg *g, int l) { return g->n[l]; }
const double *orc_mg_level_stencils(const orc_mg *g, int l) { return g->S[l]; }
const double *orc_mg_level_weights(const orc_mg *g, int l) { return g->Pw[l]; }

void orc_mg_destroy(orc_mg *g)
{
    if (!g) return;
    for (int l = 0; l < g->nlev; ++l) {
        free(g->S[l]); free(g->u[l]); free(g->f[l]); free(g->r[l]); free(g->t[l]); free(g->Pw[l]);
    }
    free(g->L);
    free(g);
}

static void coarse_solve(orc_mg *g, int l)
{
    int d = g->d, n = g->n[l], nv = n + 1, vi[3];
    int64_t NV = npow(nv, d), k = 0;
    double *b = malloc(sizeof(double) * (g->m > 0 ? g->m : 1));
    for (int64_t v = 0; v < NV; ++v)
        if (is_interior(d, nv, v, vi)) b[k++] = g->f[l][v];
    orc_cholesky_solve(g->m, g->L, b);
    k = 0;
    for (int64_t v = 0; v < NV; ++v)
        g->u[l][v] = is_interior(d, nv, v, vi) ? b[k++] : 0.0;
    free(b);
}

/* multiplicative correction-scheme V(nu1,nu2) on level l: u[l] improved for
 * rhs f[l]; coarser levels start from zero */
static void vcycle(orc_mg *g, int l, double omega, int nu1, int nu2)
{
    int d = g->d, n = g->n[l];
    int64_t NV = npow(n + 1, d);
    if (l == g->nlev - 1) { coarse_solve(g, l); return; }
    for (int i = 0; i < nu1; ++i) {
        orc_jacobi(d, n, g->S[l], g->u[l], g->f[l], omega, g->t[l]);
        memcpy(g->u[l], g->t[l], sizeof(double) * NV);
    }
    orc_residual(d, n, g->S[l], g->u[l], g->f[l], g->r[l]);
    orc_restrict(d, n, g->Pw[l], g->r[l], g->f[l + 1]);
    memset(g->u[l + 1], 0, sizeof(double) * npow(g->n[l + 1] + 1, d));
    vcycle(g, l + 1, omega, nu1, nu2);
    orc_prolong_add(d, n, g->Pw[l], g->u[l + 1], g->u[l]);
    for (int i = 0; i < nu2; ++i) {
        orc_jacobi(d, n, g->S[l], g->u[l], g->f[l], omega, g->t[l]);
        memcpy(g->u[l], g->t[l], sizeof(double) * NV);
    }
}

/* one V-cycle on the finest level: u <- V(u; f) */
void orc_mg_vcycle(orc_mg *g, double *u, const double *f, double omega, int nu1, int nu2)
{
    int64_t NV = npow(g->n[0] + 1, g->d);
    memcpy(g->u[0], u, sizeof(double) * NV);
    memcpy(g->f[0], f, sizeof(double) * NV);
    vcycle(g, 0, omega, nu1, nu2);
    memcpy(u, g->u[0], sizeof(double) * NV);
}

/* ------------------------------------------------- additive adaFAC-x cycle */
/* Sec. 4.1, eq. (mg:adaFAC-x), written as a correction scheme on the same
 * hierarchy: the fine residual r_0 = f - A_0 u is restricted to every level
 * (r_l = R r_{l-1}); every level l above the coarsest computes its update
 * at once from r_l alone,
 *     e_l = S_l r_l - P~ S_{l+1} R~ r_l,     S_l = omega diag(A_l)^{-1},
 * the second term an auxiliary coarse step that damps the update by what the
 * concurrently running coarser levels will add; the coarsest level solves
 * exactly; the updates are summed through the prolongations,
 * u += sum_l P_0 .. P_{l-1} e_l.
 * variant 1 (adaFAC-PI): R~ = injection (the fine value at the coarse
 *   vertex), P~ = P;
 * variant 2 (adaFAC-Jac): P~ = (I - S_l A_l) P, the prolongation smoothed
 *   by one damped Jacobi step, and R~ = P~^T.                               */
static void level_diag_scale(int d, int n, const double *S, const double *r, double omega, double *out)
{
    int64_t NV = npow(n + 1, d);
    int vi[3], c = nst(d) / 2;
    for (int64_t v = 0; v < NV; ++v)
        out[v] = is_interior(d, n + 1, v, vi) ? omega * r[v] / S[(size_t)v * nst(d) + c] : 0.0;
}

void orc_mg_adafac(orc_mg *g, double *u, const double *f, double omega, int variant)
{
    int d = g->d, L = g->nlev;
    int64_t NV0 = npow(g->n[0] + 1, d);
    /* residuals of every level: g->r[l] */
    orc_residual(d, g->n[0], g->S[0], u, f, g->r[0]);
    for (int l = 1; l < L; ++l)
        orc_restrict(d, g->n[l - 1], g->Pw[l - 1], g->r[l - 1], g->r[l]);
    /* level updates: g->u[l] */
    for (int l = 0; l < L - 1; ++l) {
        int n = g->n[l], nc = g->n[l + 1];
        int64_t NV = npow(n + 1, d), NVc = npow(nc + 1, d);
        double *e = g->u[l], *a = g->f[l + 1], *t = g->t[l];
        level_diag_scale(d, n, g->S[l], g->r[l], omega, e);          /* S_l r_l */
        if (variant == 1) {
            /* R~ r_l: the fine residual at each interior coarse vertex */
            int Vi[3];
            for (int64_t V = 0; V < NVc; ++V) {
                if (!is_interior(d, nc + 1, V, Vi)) { a[V] = 0.0; continue; }
                int wi[3];
                for (int m = 0; m < d; ++m) wi[m] = 2 * Vi[m];
                a[V] = g->r[l][vid(d, n + 1, wi)];
            }
            level_diag_scale(d, nc, g->S[l + 1], a, omega, a);       /* S_{l+1} R~ r_l */
            for (int64_t V = 0; V < NVc; ++V) a[V] = -a[V];
            orc_prolong_add(d, n, g->Pw[l], a, e);                    /* e -= P a */
        } else {
            /* R~ r = P^T (I - A D^{-1} omega) r */
            double *y = malloc(sizeof(double) * NV), *w = malloc(sizeof(double) * NV);
            level_diag_scale(d, n, g->S[l], g->r[l], omega, y);      /* y = S_l r */
            orc_residual(d, n, g->S[l], y, g->r[l], w);               /* w = r - A y */
            orc_restrict(d, n, g->Pw[l], w, a);                       /* a = R w */
            level_diag_scale(d, nc, g->S[l + 1], a, omega, a);       /* a = S_{l+1} R~ r */
            /* P~ a = (I - S_l A_l) P a */
            memset(t, 0, sizeof(double) * NV);
            orc_prolong_add(d, n, g->Pw[l], a, t);                    /* t = P a */
            memset(y, 0, sizeof(double) * NV);
            orc_residual(d, n, g->S[l], t, y, w);                     /* w = -A t */
            level_diag_scale(d, n, g->S[l], w, omega, y);            /* y = -S_l A t */
            int vi[3];
            for (int64_t v = 0; v < NV; ++v)
                if (is_interior(d, n + 1, v, vi)) e[v] -= t[v] + y[v];
            free(y);
            free(w);
        }
    }
    /* coarsest level: exact solve of A_{L-1} e = r_{L-1} */
    memcpy(g->f[L - 1], g->r[L - 1], sizeof(double) * npow(g->n[L - 1] + 1, d));
    coarse_solve(g, L - 1);
    /* u += sum_l P_0 .. P_{l-1} e_l, summed from the coarsest level up */
    for (int l = L - 2; l >= 0; --l)
        orc_prolong_add(d, g->n[l], g->Pw[l], g->u[l + 1], g->u[l]);
    int vi[3];
    for (int64_t v = 0; v < NV0; ++v)
        if (is_interior(d, g->n[0] + 1, v, vi)) u[v] += g->u[0][v];
}

double orc_norm_interior(int d, int n, const double *r)
{
    int64_t NV = npow(n + 1, d);
    int vi[3];
    double s = 0.0;
    for (int64_t v = 0; v < NV; ++v)
        if (is_interior(d, n + 1, v, vi)) s += r[v] * r[v];
    return sqrt(s);
}

/* ----------------------------------------------------------------- solve */
typedef struct {
    int32_t s_fixed;    /* >0: integrate every cell with this s; 0: ladder */
    int32_t s_max;
    int32_t lazy;       /* 0: whole ladder before cycling; 1: rung k applied before cycle k */
    int32_t nu1, nu2;
    int32_t coarsest;
    int32_t max_cycles;
    int32_t transfer;   /* 0 geometric d-linear, 1 BoxMG */
    int32_t outer;      /* 0 stationary (u += V r), 1 conjugate gradients with V as preconditioner */
    int32_t start;      /* after an operator change: 0 carry the iterate over (Sec. 5.1-5.3),
                           1 the carried iterate or the zero start, whichever has the smaller residual */
    int32_t cycle;      /* 0 multiplicative V(nu1,nu2); 1 additive adaFAC-PI, 2 adaFAC-Jac (one cycle
                           per iteration, stationary outer iteration only) */
    int32_t pad;
    double C, omega, tol, div_factor;
} orc_opts;

typedef struct {
    int32_t cycles, status, nlev, pad;
    double r0, r_final;
    int64_t cells_at_s[5]; /* cells whose final s is 1,2,4,8,16 */
    int64_t integrations;  /* cell integrations performed */
    double hist[512];      /* normalised residual at the start of each cycle */
} orc_report;

enum { ORC_OK = 0, ORC_ENOCONV = -4, ORC_EDIVERGED = -5 };

/* Solve A u = f from u (in/out).  Up-front: every cell climbs its ladder to
 * the end before the first cycle (eq. level-operator-sequence-explicit-
 * assembly, all markers final).  Lazy (deterministic schedule): cycle 0 runs
 * on the centre-sample operator and rung k (s = 2^k) of every unfinished
 * cell is integrated and published before cycle k (Sec. 5.1-5.3); cycles
 * on the centre-sample operator use a geometric hierarchy (Sec. 1).  The
 * residual is measured at the start of each cycle with the operator current
 * then, normalised by the first one (Sec. 6); after an operator change the
 * iteration carries its iterate over (Sec. 5.1-5.3: the smoother continues
 * on whatever operator is current), or, with op->start = 1, continues from
 * the carried iterate or from the zero start, whichever has the smaller
 * residual on the new operator; the run stops
 * when every cell is final and the normalised residual is at most tol (for
 * CG the recursion's residual, confirmed with f - A u itself); the
 * stationary iteration aborts when the residual exceeds div_factor times its
 * reference, CG only on a non-finite residual.                             */
int orc_solve(const orc_field *fld, int d, int N, const double *f, double *u, const orc_opts *op, orc_report *rep)
{
    int nl = 1 << d, nn = nl * nl;
    int64_t nc = npow(N, d), NV = npow(N + 1, d);
    double *K = malloc(sizeof(double) * nc * nn);
    double *S = malloc(sizeof(double) * NV * nst(d));
    double *r = malloc(sizeof(double) * NV);
    int32_t *sfin = malloc(sizeof(int32_t) * nc);
    uint8_t *done = malloc(nc);
    int64_t integ = 0;
    memset(rep, 0, sizeof(*rep));

    int ladder = op->s_fixed <= 0;
    if (!ladder) {
        orc_assemble(fld, d, N, op->s_fixed, NULL, nc, K);
        integ += nc;
        for (int64_t c = 0; c < nc; ++c) { sfin[c] = op->s_fixed; done[c] = 1; }
    } else if (!op->lazy) {
        for (int64_t c = 0; c < nc; ++c) {
            double rel[4];
            sfin[c] = orc_ladder_cell(fld, d, N, c, op->s_max, op->C, K + c * nn, rel);
            int steps = 0;
            for (int m = 1; m < sfin[c]; m *= 2) ++steps;
            integ += 1 + steps;
            done[c] = 1;
        }
    } else {
        orc_assemble(fld, d, N, 1, NULL, nc, K);
        integ += nc;
        for (int64_t c = 0; c < nc; ++c) { sfin[c] = 1; done[c] = op->s_max < 2; }
    }
    orc_stencils(d, N, K, S);
    orc_mg *g = orc_mg_create(d, N, op->coarsest, op->transfer, S);
    if (ladder && op->lazy) {
        /* the provisional (centre-sample) operator starts on a geometric
         * hierarchy; every publish rebuilds the hierarchy of op->transfer */
        double *ec = malloc(sizeof(double) * nc);
        for (int64_t c = 0; c < nc; ++c) {
            int ci[3];
            double x[3] = {0.0, 0.0, 0.0};
            cell_coords(d, N, c, ci);
            for (int m = 0; m < d; ++m) x[m] = (ci[m] + 0.5) / N;
            ec[c] = orc_eps(fld, x);
        }
        orc_mg_set_geometric(g, S, ec);
        free(ec);
    }
    rep->nlev = g->nlev;
    int status = ORC_ENOCONV, k, rung = 1;
    double r0 = 0.0, rk = 0.0;
    /* outer Krylov state: conjugate gradients with one V-cycle as the
     * preconditioner B; beta in the Polak-Ribiere form z.(r - r_old)/(z_old.r_old)
     * and a restart whenever the operator changes */
    double *z = calloc(NV, sizeof(double)), *p = calloc(NV, sizeof(double));
    double *Ap = calloc(NV, sizeof(double)), *rold = calloc(NV, sizeof(double));
    double *zero = calloc(NV, sizeof(double));
    double zr_old = 0.0, r_ref = 0.0;
    int restart = 1;
    int vi[3];
    for (k = 0; k <= op->max_cycles; ++k) {
        if (ladder && op->lazy && k >= 1 && (1 << rung) <= op->s_max) {
            int m = 1 << rung;
            double Kn[64];
            int changed = 0;
            for (int64_t c = 0; c < nc; ++c) {
                if (done[c]) continue;
                orc_element_matrix(fld, d, N, m, c, Kn);
                ++integ;
                double diff[64];
                for (int i = 0; i < nn; ++i) diff[i] = Kn[i] - K[c * nn + i];
                double rel = maxabs(diff, nn) / maxabs(K + c * nn, nn);
                memcpy(K + c * nn, Kn, sizeof(double) * nn);
                sfin[c] = m;
                if (rel < op->C || 2 * m > op->s_max) done[c] = 1;
                changed = 1;
            }
            ++rung;
            if (changed) {
                orc_stencils(d, N, K, S);
                orc_mg_set_fine(g, S);
                restart = 1;
            }
        }
        if (op->outer == 0 || restart)
            orc_residual(d, N, g->S[0], u, f, r);
        rk = orc_norm_interior(d, N, r);
        /* start after an operator change.  The paper carries the iterate
         * over (start = 0: nothing to do).  The optional rule (start = 1)
         * keeps the carried iterate unless its residual on the new operator
         * exceeds that of the zero start (the interior set to zero, boundary
         * values kept), in which case the iteration restarts from there */
        if (restart && k > 0 && op->start == 1) {
            double *uz = malloc(sizeof(double) * NV), *rz = malloc(sizeof(double) * NV);
            for (int64_t v = 0; v < NV; ++v) uz[v] = is_interior(d, N + 1, v, vi) ? 0.0 : u[v];
            orc_residual(d, N, g->S[0], uz, f, rz);
            double rzn = orc_norm_interior(d, N, rz);
            if (rk > rzn) {
                memcpy(u, uz, sizeof(double) * NV);
                memcpy(r, rz, sizeof(double) * NV);
                rk = rzn;
            }
            free(uz);
            free(rz);
        }
        if (k == 0) r0 = rk;
        /* the divergence guard (Sec. 6.2) watches the solver, not operator
         * updates: its reference is re-taken whenever the operator changes */
        if (k == 0 || restart) r_ref = rk > r0 ? rk : r0;
        double rel = r0 > 0.0 ? rk / r0 : 0.0;
        if (k < 512) rep->hist[k] = rel;
        int all_done = 1, fresh = restart;
        for (int64_t c = 0; c < nc && all_done; ++c) all_done = done[c];
        if (all_done && rel <= op->tol) {
            /* the stopping rule is on f - A u (Sec. 6); the CG recursion's
             * residual drifts from it by rounding, so a recursion-based
             * convergence is confirmed with the residual itself, and if that
             * is still above the tolerance CG restarts from it */
            if (op->outer == 0 || restart) { status = ORC_OK; break; }
            orc_residual(d, N, g->S[0], u, f, r);
            double rt = orc_norm_interior(d, N, r);
            if (rt <= op->tol * r0) { rk = rt; status = ORC_OK; break; }
            fresh = 1;
        }
        /* the guard watches the stationary iteration; the CG residual norm is
         * not monotone, so CG stops only on a non-finite residual */
        if (op->outer == 0 ? !(rk <= op->div_factor * r_ref) : !isfinite(rk)) { status = ORC_EDIVERGED; break; }
        if (k == op->max_cycles) break;
        if (op->outer == 0) {
            if (op->cycle == 0) orc_mg_vcycle(g, u, f, op->omega, op->nu1, op->nu2);
            else orc_mg_adafac(g, u, f, op->omega, op->cycle);
            restart = 0;
            continue;
        }
        memset(z, 0, sizeof(double) * NV);
        orc_mg_vcycle(g, z, r, op->omega, op->nu1, op->nu2); /* z = B r */
        double zr = 0.0, zdr = 0.0;
        for (int64_t v = 0; v < NV; ++v) {
            if (!is_interior(d, N + 1, v, vi)) continue;
            zr += z[v] * r[v];
            zdr += z[v] * (r[v] - rold[v]);
        }
        double beta = fresh ? 0.0 : zdr / zr_old;
        for (int64_t v = 0; v < NV; ++v)
            p[v] = z[v] + beta * p[v];
        orc_residual(d, N, g->S[0], p, zero, Ap); /* Ap = -(A p) on the interior */
        double pAp = 0.0;
        for (int64_t v = 0; v < NV; ++v)
            if (is_interior(d, N + 1, v, vi)) pAp -= p[v] * Ap[v];
        double alpha = zr / pAp;
        for (int64_t v = 0; v < NV; ++v) {
            rold[v] = r[v];
            if (!is_interior(d, N + 1, v, vi)) continue;
            u[v] += alpha * p[v];
            r[v] += alpha * Ap[v];
        }
        zr_old = zr;
        restart = 0;
    }
    free(z); free(p); free(Ap); free(rold); free(zero);
    rep->cycles = k;
    rep->status = status;
    rep->r0 = r0;
    rep->r_final = rk;
    rep->integrations = integ;
    for (int64_t c = 0; c < nc; ++c) {
        int b = 0;
        for (int m = 1; m < sfin[c]; m *= 2) ++b;
        if (b < 5) rep->cells_at_s[b]++;
    }
    orc_mg_destroy(g);
    free(K); free(S); free(r); free(sfin); free(done);
    return status;
}

/* ------------------------------------------------ whole-level compression */
/* Sec. 5.5 applied to a level of half stencils: S32 holds the upper-half
 * couplings [H][NV] (slot-major, slot j = stencil index centre+1+j) as FP32.
 * delta_v[j] = (float)((double)S32 - base_v) is the hierarchical surplus over
 * the centre-sample base; each vertex gets the cheapest tier that meets
 * tau_v = max(tau_abs, tau_rel * ref_v); a tile of 64 consecutive vertices
 * takes the largest tier of its vertices and every vertex in it is encoded
 * at that tier.  Outputs: tile_tier[ceil(NV/64)], e8[NV], words[NV][H].    */
void orc_compress(int d, int N, const float *S32, const float *eps_c, int min_tier, int max_tier,
                  double tau_abs, double tau_rel, uint8_t *tile_tier, uint8_t *e8, uint32_t *words)
{
    int ns = nst(d), H = ns / 2, c0 = ns / 2 + 1;
    int64_t NV = npow(N + 1, d), ntile = (NV + 63) / 64;
    float *delta = malloc(sizeof(float) * NV * H);
    uint8_t *vt = malloc(NV);
    for (int64_t v = 0; v < NV; ++v) {
        double ref = 0.0;
        for (int j = 0; j < H; ++j) {
            double b;
            orc_base_coupling(d, N, eps_c, v, c0 + j, &b, &ref);
            delta[v * H + j] = (float)((double)S32[(size_t)j * NV + v] - b);
        }
        double tau = tau_rel * ref;
        if (tau_abs > tau) tau = tau_abs;
        vt[v] = (uint8_t)orc_choose_tier(delta + v * H, H, tau, min_tier, max_tier);
    }
    for (int64_t t = 0; t < ntile; ++t) {
        uint8_t m = 0;
        for (int64_t v = t * 64; v < NV && v < t * 64 + 64; ++v)
            if (vt[v] > m) m = vt[v];
        tile_tier[t] = m;
        for (int64_t v = t * 64; v < NV && v < t * 64 + 64; ++v)
            e8[v] = (uint8_t)orc_encode_stencil(delta + v * H, H, m, words + v * H);
    }
    free(delta);
    free(vt);
}
