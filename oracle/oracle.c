/*
 * oracle.c -- plain FP64 CPU oracle for the mixed-precision GEMM library.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code, header or table with the
 * GPU library: every rounding rule below is written from the number formats'
 * definitions, and the GEMM is the textbook definition.
 *
 * Contents
 *   - rounding of a real value onto the FP16, BF16 and FP8-E4M3 grids with
 *     round-to-nearest-even (paper Sec. V, "Limited range" / "Decreasing
 *     precision" items: 5 exponent bits, 10 fraction bits, max 65504,
 *     overflow to infinity, 1024 values per binade);
 *   - decoding of those formats back to FP64;
 *   - the FP64 GEMM  out = alpha*A*B + beta*C0  (paper Sec. IV, the BLAS
 *     GEMM that Tensor Cores express), optionally on a subset of rows.
 *
 * Precision: every product of two FP32 (or narrower) values is exact in
 * FP64; the only error is FP64 summation, at most K*2^-53*(|A||B|)_ij.
 * Summation runs over k = 0..K-1 in order for every output element.
 */
#include <math.h>
#include <stdint.h>
#include <string.h>

/* ------------------------------------------------------------------------
 * Generic round-to-nearest-even of a finite value a >= 0 onto the grid of a
 * binary floating-point format with p fraction bits and minimum normal
 * exponent emin.  Above 2^emin the spacing in [2^e, 2^(e+1)) is 2^(e-p);
 * below it the spacing is the subnormal quantum 2^(emin-p).  The quotient
 * a / quantum is exact (power-of-two scaling of a double), and nearbyint()
 * in the default rounding mode rounds half-way cases to even.
 * Overflow is NOT handled here; each format applies its own rule.
 * ---------------------------------------------------------------------- */
static double rne_to_grid(double a, int p, int emin)
{
    int e;
    if (a == 0.0) return 0.0;
    if (a < ldexp(1.0, emin)) {
        e = emin;
    } else {
        int ex;
        (void)frexp(a, &ex);     /* a = f * 2^ex, f in [0.5, 1) */
        e = ex - 1;              /* a in [2^e, 2^(e+1)) */
    }
    double quantum = ldexp(1.0, e - p);
    return nearbyint(a / quantum) * quantum;
}

/* Pack a rounded value r >= 0 (already on the grid, finite, in range) into
 * exponent/fraction fields of a format with p fraction bits, bias, emin. */
static uint32_t pack_bits(double r, int p, int bias, int emin)
{
    if (r == 0.0) return 0;
    if (r < ldexp(1.0, emin)) {                       /* subnormal */
        return (uint32_t)(r / ldexp(1.0, emin - p));  /* exact integer */
    }
    int ex;
    (void)frexp(r, &ex);
    int e = ex - 1;
    double frac = r / ldexp(1.0, e) - 1.0;            /* in [0, 1) */
    uint32_t mant = (uint32_t)(frac * ldexp(1.0, p)); /* exact integer */
    return ((uint32_t)(e + bias) << p) | mant;
}

/* ---------------------------- FP16 (binary16) --------------------------- */
/* 1 sign bit, 5 exponent bits (bias 15), 10 fraction bits. */
#define F16_P 10
#define F16_BIAS 15
#define F16_EMIN (-14)
#define F16_MAX 65504.0

uint16_t orc_f16_encode(double x)
{
    uint16_t sign = signbit(x) ? 0x8000u : 0u;
    if (isnan(x)) return (uint16_t)(sign | 0x7E00u);   /* quiet NaN */
    double a = fabs(x);
    if (isinf(a)) return (uint16_t)(sign | 0x7C00u);
    double r = rne_to_grid(a, F16_P, F16_EMIN);
    if (r > F16_MAX) return (uint16_t)(sign | 0x7C00u); /* overflow -> inf */
    return (uint16_t)(sign | pack_bits(r, F16_P, F16_BIAS, F16_EMIN));
}

double orc_f16_decode(uint16_t h)
{
    double s = (h & 0x8000u) ? -1.0 : 1.0;
    int field = (h >> 10) & 0x1F;
    int mant = h & 0x3FF;
    if (field == 0x1F) return mant ? NAN : s * INFINITY;
    if (field == 0) return s * ldexp((double)mant, F16_EMIN - F16_P);
    return s * ldexp(1.0 + mant / 1024.0, field - F16_BIAS);
}

/* ------------------------------- BF16 ----------------------------------- */
/* 1 sign bit, 8 exponent bits (bias 127), 7 fraction bits. */
#define BF16_P 7
#define BF16_BIAS 127
#define BF16_EMIN (-126)

uint16_t orc_bf16_encode(double x)
{
    uint16_t sign = signbit(x) ? 0x8000u : 0u;
    if (isnan(x)) return (uint16_t)(sign | 0x7FC0u);
    double a = fabs(x);
    if (isinf(a)) return (uint16_t)(sign | 0x7F80u);
    double r = rne_to_grid(a, BF16_P, BF16_EMIN);
    double bmax = ldexp(2.0 - ldexp(1.0, -BF16_P), 127);
    if (r > bmax) return (uint16_t)(sign | 0x7F80u);
    return (uint16_t)(sign | pack_bits(r, BF16_P, BF16_BIAS, BF16_EMIN));
}

double orc_bf16_decode(uint16_t h)
{
    double s = (h & 0x8000u) ? -1.0 : 1.0;
    int field = (h >> 7) & 0xFF;
    int mant = h & 0x7F;
    if (field == 0xFF) return mant ? NAN : s * INFINITY;
    if (field == 0) return s * ldexp((double)mant, BF16_EMIN - BF16_P);
    return s * ldexp(1.0 + mant / 128.0, field - BF16_BIAS);
}

/* --------------------------- FP8 E4M3 (OCP "fn") ------------------------ */
/* 1 sign bit, 4 exponent bits (bias 7), 3 fraction bits, no infinity; the
 * all-ones code S.1111.111 is NaN, so the largest finite value is
 * S.1111.110 = 448.  Encoding saturates: finite values beyond 448 (and
 * infinities) map to +-448. */
#define E4M3_P 3
#define E4M3_BIAS 7
#define E4M3_EMIN (-6)
#define E4M3_MAX 448.0

uint8_t orc_e4m3_encode_sat(double x)
{
    uint8_t sign = signbit(x) ? 0x80u : 0u;
    if (isnan(x)) return (uint8_t)(sign | 0x7Fu);
    double a = fabs(x);
    if (isinf(a) || a >= E4M3_MAX) return (uint8_t)(sign | 0x7Eu);
    double r = rne_to_grid(a, E4M3_P, E4M3_EMIN);
    if (r > E4M3_MAX) r = E4M3_MAX;
    return (uint8_t)(sign | pack_bits(r, E4M3_P, E4M3_BIAS, E4M3_EMIN));
}

double orc_e4m3_decode(uint8_t q)
{
    double s = (q & 0x80u) ? -1.0 : 1.0;
    int field = (q >> 3) & 0xF;
    int mant = q & 0x7;
    if (field == 0xF && mant == 0x7) return NAN;
    if (field == 0) return s * ldexp((double)mant, E4M3_EMIN - E4M3_P);
    return s * ldexp(1.0 + mant / 8.0, field - E4M3_BIAS);
}

/* ---------------------------- array helpers ----------------------------- */
void orc_f16_encode_array(const double* x, int64_t n, uint16_t* out)
{
    for (int64_t i = 0; i < n; ++i) out[i] = orc_f16_encode(x[i]);
}
void orc_f16_decode_array(const uint16_t* h, int64_t n, double* out)
{
    for (int64_t i = 0; i < n; ++i) out[i] = orc_f16_decode(h[i]);
}
void orc_bf16_encode_array(const double* x, int64_t n, uint16_t* out)
{
    for (int64_t i = 0; i < n; ++i) out[i] = orc_bf16_encode(x[i]);
}
void orc_bf16_decode_array(const uint16_t* h, int64_t n, double* out)
{
    for (int64_t i = 0; i < n; ++i) out[i] = orc_bf16_decode(h[i]);
}
void orc_e4m3_encode_array(const double* x, int64_t n, uint8_t* out)
{
    for (int64_t i = 0; i < n; ++i) out[i] = orc_e4m3_encode_sat(x[i]);
}
void orc_e4m3_decode_array(const uint8_t* q, int64_t n, double* out)
{
    for (int64_t i = 0; i < n; ++i) out[i] = orc_e4m3_decode(q[i]);
}

/* ------------------------------ FP64 GEMM ------------------------------- */
/*
 * out[r, :] = alpha * sum_k A[i, k] * B[k, :] + beta * C0[i, :]
 * for r = 0..nrows-1 and i = rows[r] (or i = r when rows is NULL).
 * Row-major storage with leading dimensions lda, ldb, ldc0, ldo.
 * BLAS convention: when beta == 0, C0 is not read (it may hold NaN).
 * For each output element the sum runs over k = 0, 1, ..., K-1 in order;
 * the k-outer / j-inner loop only changes which element is updated next.
 */
void orc_gemm_f64(int64_t M, int64_t N, int64_t K,
                  const double* A, int64_t lda,
                  const double* B, int64_t ldb,
                  double alpha, double beta,
                  const double* C0, int64_t ldc0,
                  double* out, int64_t ldo,
                  const int64_t* rows, int64_t nrows)
{
    (void)M;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t r = 0; r < nrows; ++r) {
        int64_t i = rows ? rows[r] : r;
        double* o = out + r * ldo;
        for (int64_t j = 0; j < N; ++j) o[j] = 0.0;
        for (int64_t k = 0; k < K; ++k) {
            double a = A[i * lda + k];
            const double* b = B + k * ldb;
            for (int64_t j = 0; j < N; ++j) o[j] += a * b[j];
        }
        for (int64_t j = 0; j < N; ++j) {
            double v = alpha * o[j];
            if (beta != 0.0) v += beta * C0[i * ldc0 + j];
            o[j] = v;
        }
    }
}

/* Number of OpenMP threads the GEMM above uses (1 without OpenMP). */
#ifdef _OPENMP
#include <omp.h>
int orc_num_threads(void) { return omp_get_max_threads(); }
#else
int orc_num_threads(void) { return 1; }
#endif
