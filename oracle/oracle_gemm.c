/*
 * FP64 CPU oracle for C = alpha*A*B + beta*C  -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg may
 * load this file's library.  The product path (the HIP library under
 * paper_2301_03598_amd/) neither includes nor links anything from here, and
 * this file includes nothing from it.
 *
 * What it computes (paper section 2, the GEMM definition): for an m x n x k
 * problem, C[i][j] = alpha * sum_p A[i][p] * B[p][j] + beta * Cin[i][j], all
 * in IEEE double.  The inputs are decoded from the exact bytes the GPU
 * receives (FP64, FP32, FP16, BF16 or OCP FP8 e4m3fn); every such value is
 * exactly representable in double, and FP8 operands are dequantised as
 * scale * code, which is also exact in double (a 24-bit FP32 scale times a
 * 4-bit significand).
 *
 * How (section 3.1, Algorithm 1, the sequential cache-blocked GEMM): tile
 * loops over mm (outer) and nn, a zero-initialised output tile, then for each
 * kk block the three inner loops mmm, nnn, kkk in that order.  OpenMP runs
 * the independent (mm, nn) tiles in parallel; each tile's arithmetic is the
 * algorithm's loop nest unchanged.  alpha and beta are applied once per
 * output element after the k loop.
 *
 * Output rounding: oracle_round() rounds double values once, to nearest with
 * ties to even, into FP32, FP16 or BF16 bytes.  It is written from the
 * formats' definitions (significand width, exponent range, subnormals,
 * overflow to infinity) and is used to state the exactly rounded reference
 * for narrow outputs.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* dtype and order codes: the C-ABI's enumerations, restated independently */
enum { OR_F64 = 0, OR_F32 = 1, OR_F16 = 2, OR_BF16 = 3, OR_F8E4M3 = 4 };
enum { OR_ROW = 0, OR_COL = 1 };

enum { OR_OK = 0, OR_EINVAL = 1, OR_ENOMEM = 2 };

/* ---- decoders: bit patterns -> exact double values ------------------- */

/* IEEE binary16: 1 sign, 5 exponent (bias 15), 10 fraction bits. */
static double dec_f16(uint16_t h) {
    int s = h >> 15, e = (h >> 10) & 0x1f, f = h & 0x3ff;
    double v;
    if (e == 0)
        v = ldexp((double)f, -24);                 /* subnormal: f * 2^-24 */
    else if (e == 31)
        v = f ? NAN : INFINITY;
    else
        v = ldexp((double)(1024 + f), e - 25);     /* (1.f) * 2^(e-15) */
    return s ? -v : v;
}

/* bfloat16: 1 sign, 8 exponent (bias 127), 7 fraction bits. */
static double dec_bf16(uint16_t b) {
    int s = b >> 15, e = (b >> 7) & 0xff, f = b & 0x7f;
    double v;
    if (e == 0)
        v = ldexp((double)f, -133);                /* f * 2^(-126-7) */
    else if (e == 255)
        v = f ? NAN : INFINITY;
    else
        v = ldexp((double)(128 + f), e - 134);     /* (1.f) * 2^(e-127) */
    return s ? -v : v;
}

/* IEEE binary32 via its fields (no type punning through the host FPU). */
static double dec_f32(uint32_t w) {
    int s = w >> 31, e = (w >> 23) & 0xff;
    uint32_t f = w & 0x7fffff;
    double v;
    if (e == 0)
        v = ldexp((double)f, -149);
    else if (e == 255)
        v = f ? NAN : INFINITY;
    else
        v = ldexp((double)(0x800000u + f), e - 150);
    return s ? -v : v;
}

/* OCP FP8 E4M3 ("fn"): 1 sign, 4 exponent (bias 7), 3 fraction bits; no
 * infinities; S.1111.111 is NaN; max finite 448; min subnormal 2^-9. */
static double dec_f8e4m3(uint8_t q) {
    int s = q >> 7, e = (q >> 3) & 0xf, f = q & 0x7;
    double v;
    if (e == 15 && f == 7)
        v = NAN;
    else if (e == 0)
        v = ldexp((double)f, -9);                  /* f * 2^(-6-3) */
    else
        v = ldexp((double)(8 + f), e - 10);        /* (1.f) * 2^(e-7) */
    return s ? -v : v;
}

static double load_elem(const void *base, int dtype, int64_t idx) {
    switch (dtype) {
    case OR_F64: { double d; memcpy(&d, (const char *)base + 8 * idx, 8); return d; }
    case OR_F32: { uint32_t w; memcpy(&w, (const char *)base + 4 * idx, 4); return dec_f32(w); }
    case OR_F16: { uint16_t h; memcpy(&h, (const char *)base + 2 * idx, 2); return dec_f16(h); }
    case OR_BF16: { uint16_t b; memcpy(&b, (const char *)base + 2 * idx, 2); return dec_bf16(b); }
    case OR_F8E4M3: return dec_f8e4m3(((const uint8_t *)base)[idx]);
    }
    return NAN;
}

/* element (r, c) of a rows x cols matrix stored in `order` with leading dim ld */
static int64_t at(int order, int64_t ld, int64_t r, int64_t c) {
    return order == OR_ROW ? r * ld + c : c * ld + r;
}

/* Decode a whole operand into a dense row-major double array, times scale. */
int oracle_decode(const void *src, int dtype, int order, int64_t ld,
                  int64_t rows, int64_t cols, double scale, double *dst) {
    if (rows < 0 || cols < 0) return OR_EINVAL;
    for (int64_t r = 0; r < rows; ++r)
        for (int64_t c = 0; c < cols; ++c)
            dst[r * cols + c] = scale * load_elem(src, dtype, at(order, ld, r, c));
    return OR_OK;
}

/* ---- Algorithm 1 on dense row-major doubles ---------------------------- */

static void blocked_gemm(int64_t m, int64_t n, int64_t k, const double *A,
                         const double *B, double *acc_out, int64_t blk_m,
                         int64_t blk_n, int64_t blk_k) {
    int64_t tiles_m = (m + blk_m - 1) / blk_m, tiles_n = (n + blk_n - 1) / blk_n;
    int64_t tiles = tiles_m * tiles_n;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t t = 0; t < tiles; ++t) {
        int64_t mm = (t / tiles_n) * blk_m, nn = (t % tiles_n) * blk_n;
        int64_t me = mm + blk_m < m ? mm + blk_m : m;
        int64_t ne = nn + blk_n < n ? nn + blk_n : n;
        /* zero-initialise the output tile */
        for (int64_t mmm = mm; mmm < me; ++mmm)
            for (int64_t nnn = nn; nnn < ne; ++nnn)
                acc_out[mmm * n + nnn] = 0.0;
        /* the MAC iterations for this tile */
        for (int64_t kk = 0; kk < k; kk += blk_k) {
            int64_t ke = kk + blk_k < k ? kk + blk_k : k;
            for (int64_t mmm = mm; mmm < me; ++mmm)
                for (int64_t nnn = nn; nnn < ne; ++nnn) {
                    double c = acc_out[mmm * n + nnn];
                    for (int64_t kkk = kk; kkk < ke; ++kkk)
                        c = c + A[mmm * k + kkk] * B[kkk * n + nnn];
                    acc_out[mmm * n + nnn] = c;
                }
        }
    }
}

/*
 * oracle_gemm_f64: out (m x n, dense row-major double) =
 *     alpha * (decode(A)*a_scale) x (decode(B)*b_scale) + beta * decode(Cin)
 * Cin is read only when beta != 0 (BLAS convention) and may be NULL then.
 * blk_* <= 0 selects 64.  nthreads <= 0 leaves the OpenMP default.
 */
int oracle_gemm_f64(int64_t m, int64_t n, int64_t k, double alpha, double beta,
                    int ab_type, int c_type, int a_order, int b_order, int c_order,
                    int64_t lda, int64_t ldb, int64_t ldc, const void *A,
                    const void *B, const void *Cin, double a_scale, double b_scale,
                    double *out, int64_t blk_m, int64_t blk_n, int64_t blk_k,
                    int nthreads) {
    if (m < 0 || n < 0 || k < 0 || !out) return OR_EINVAL;
    if (blk_m <= 0) blk_m = 64;
    if (blk_n <= 0) blk_n = 64;
    if (blk_k <= 0) blk_k = 64;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
    if (m == 0 || n == 0) return OR_OK;
    double *Ad = NULL, *Bd = NULL;
    if (k > 0) {
        Ad = (double *)malloc(sizeof(double) * (size_t)(m * k));
        Bd = (double *)malloc(sizeof(double) * (size_t)(k * n));
        if (!Ad || !Bd) { free(Ad); free(Bd); return OR_ENOMEM; }
        oracle_decode(A, ab_type, a_order, lda, m, k, a_scale, Ad);
        oracle_decode(B, ab_type, b_order, ldb, k, n, b_scale, Bd);
        blocked_gemm(m, n, k, Ad, Bd, out, blk_m, blk_n, blk_k);
    } else {
        for (int64_t i = 0; i < m * n; ++i) out[i] = 0.0;
    }
    for (int64_t i = 0; i < m; ++i)
        for (int64_t j = 0; j < n; ++j) {
            double v = alpha * out[i * n + j];
            if (beta != 0.0)
                v = v + beta * load_elem(Cin, c_type, at(c_order, ldc, i, j));
            out[i * n + j] = v;
        }
    free(Ad);
    free(Bd);
    return OR_OK;
}

/*
 * One output element, for spot checks of results too large to recompute
 * whole: the k-sum in ascending p, then alpha and beta as above.
 */
double oracle_gemm_elem(int64_t i, int64_t j, int64_t k, double alpha, double beta,
                        int ab_type, int c_type, int a_order, int b_order,
                        int c_order, int64_t lda, int64_t ldb, int64_t ldc,
                        const void *A, const void *B, const void *Cin,
                        double a_scale, double b_scale) {
    double c = 0.0;
    for (int64_t p = 0; p < k; ++p)
        c = c + (a_scale * load_elem(A, ab_type, at(a_order, lda, i, p))) *
                    (b_scale * load_elem(B, ab_type, at(b_order, ldb, p, j)));
    double v = alpha * c;
    if (beta != 0.0) v = v + beta * load_elem(Cin, c_type, at(c_order, ldc, i, j));
    return v;
}

/* ---- rounding double -> narrow formats (round to nearest, ties even) --- */

/*
 * Round x to a binary format with `p` significand bits (including the
 * implicit one), minimum normal exponent emin and maximum finite value
 * maxv.  Returns the rounded value as a double (exact).  The step is the
 * spacing of representable numbers at x's binade, floored at the subnormal
 * spacing 2^(emin-p+1); x / step is then rounded to an integer with ties to
 * even (nearbyint in the default rounding mode).  Results beyond the largest
 * finite value round to infinity when |x| >= maxv + half a step at the top.
 */
static double round_format(double x, int p, int emin, double maxv) {
    if (isnan(x) || isinf(x) || x == 0.0) return x;
    int e;
    frexp(fabs(x), &e);         /* |x| = f * 2^e, f in [0.5, 1): binade exp e-1 */
    int be = e - 1;
    if (be < emin) be = emin;
    double step = ldexp(1.0, be - (p - 1));
    double r = nearbyint(x / step) * step;
    if (fabs(r) > maxv) return x > 0 ? INFINITY : -INFINITY;
    return r;
}

static uint16_t enc_bf16(double v) {   /* v exactly representable in bf16 */
    if (isnan(v)) return 0x7fc0;
    uint16_t s = signbit(v) ? 0x8000 : 0;
    double a = fabs(v);
    if (isinf(a)) return s | 0x7f80;
    if (a == 0.0) return s;
    int e;
    double f = frexp(a, &e);    /* a = f * 2^e, f in [0.5,1) */
    int be = e - 1;             /* unbiased exponent of the leading bit */
    if (be < -126) {            /* subnormal: a = frac * 2^-133 */
        return s | (uint16_t)(int64_t)ldexp(a, 133);
    }
    uint16_t frac = (uint16_t)((int64_t)ldexp(f, 8) - 128);
    return s | (uint16_t)((be + 127) << 7) | frac;
}

static uint16_t enc_f16(double v) {
    if (isnan(v)) return 0x7e00;
    uint16_t s = signbit(v) ? 0x8000 : 0;
    double a = fabs(v);
    if (isinf(a)) return s | 0x7c00;
    if (a == 0.0) return s;
    int e;
    double f = frexp(a, &e);
    int be = e - 1;
    if (be < -14) return s | (uint16_t)(int64_t)ldexp(a, 24);
    uint16_t frac = (uint16_t)((int64_t)ldexp(f, 11) - 1024);
    return s | (uint16_t)((be + 15) << 10) | frac;
}

static uint32_t enc_f32(double v) {
    if (isnan(v)) return 0x7fc00000u;
    uint32_t s = signbit(v) ? 0x80000000u : 0;
    double a = fabs(v);
    if (isinf(a)) return s | 0x7f800000u;
    if (a == 0.0) return s;
    int e;
    double f = frexp(a, &e);
    int be = e - 1;
    if (be < -126) return s | (uint32_t)(int64_t)ldexp(a, 149);
    uint32_t frac = (uint32_t)((int64_t)ldexp(f, 24) - 0x800000);
    return s | ((uint32_t)(be + 127) << 23) | frac;
}

/* Round `count` doubles once into c_type bytes (F64: plain copy). */
int oracle_round(const double *src, int64_t count, int c_type, void *dst) {
    for (int64_t i = 0; i < count; ++i) {
        double x = src[i];
        switch (c_type) {
        case OR_F64: memcpy((char *)dst + 8 * i, &x, 8); break;
        case OR_F32: {
            uint32_t w = enc_f32(round_format(x, 24, -126, 0x1.fffffep127));
            memcpy((char *)dst + 4 * i, &w, 4);
            break;
        }
        case OR_F16: {
            uint16_t h = enc_f16(round_format(x, 11, -14, 65504.0));
            memcpy((char *)dst + 2 * i, &h, 2);
            break;
        }
        case OR_BF16: {
            uint16_t b = enc_bf16(round_format(x, 8, -126, 0x1.fep127));
            memcpy((char *)dst + 2 * i, &b, 2);
            break;
        }
        default: return OR_EINVAL;
        }
    }
    return OR_OK;
}

/* Decode `count` elements of one dtype into doubles (test helper). */
int oracle_decode_vec(const void *src, int dtype, int64_t count, double *dst) {
    for (int64_t i = 0; i < count; ++i) dst[i] = load_elem(src, dtype, i);
    return OR_OK;
}
