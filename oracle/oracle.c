/*
 * CPU oracle for the OpenACC loop-nest matmul and the reduction(+) clause.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg call into this file.  It shares no code,
 * header, table or helper with the device library, and the device library
 * never calls it.
 *
 * What is computed, and where the paper defines it (IPMACC, arXiv 1412.1127):
 *
 *  - matmul: Listing 1a read without its directives (section 1.3,
 *    "Matrix-Matrix Multiplication Example"): for every (i, j),
 *    sum = 0; for l ascending: sum += a[i*LEN+l] * b[l*LEN+j]; c[i*LEN+j] = sum.
 *    float operands: `sum` is widened to double.  A product of two floats is
 *    exact in double, so the only rounding is the l-ascending accumulation.
 *    int operands (Listing 1b's element type): two's-complement wraparound,
 *    i.e. the sum mod 2**32; computed in uint64 (mod 2**64, which 2**32
 *    divides) and truncated.
 *  - reduction: the reduction clause of the parallelism-control directives
 *    (section 2.3, "Replacing the dummy OpenACC kernels region calls", and the
 *    SRAD paragraph of section 4.2): result = init + x[0] + x[1] + ... in
 *    index order; double for float input, int64 then mod 2**32 for int32.
 *  - bf16 three-term split of a float, hi = RN(x), mid = RN(x - hi),
 *    lo = RN(x - hi - mid) with RN = round-to-nearest-even to bfloat16: the
 *    precision path that runs the float matmul on bf16 matrix cores.
 *  - balanced base-256 digits (int8 limbs) of an int32: the exact integer
 *    path that runs the int matmul on int8 matrix cores.
 *
 * Loop order.  oracle_matmul_f32 / _i32 run the i-l-j order with OpenMP over
 * i.  Every c[i][j] still receives its terms in l-ascending order, so the
 * result is bitwise that of the literal i-j-l order, which is kept as
 * oracle_matmul_*_ijl and checked against it in the tests.
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -shared -fPIC (no fast-math).
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

void oracle_set_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }
int oracle_max_threads(void) { return omp_get_max_threads(); }

/* ---------------------------------------------------------------- matmul -- */

void oracle_matmul_f32_ijl(int64_t len, const float *a, const float *b, double *c)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < len; ++i)
        for (int64_t j = 0; j < len; ++j) {
            double sum = 0.0;
            for (int64_t l = 0; l < len; ++l)
                sum += (double)a[i * len + l] * (double)b[l * len + j];
            c[i * len + j] = sum;
        }
}

void oracle_matmul_f32(int64_t len, const float *a, const float *b, double *c)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < len; ++i) {
        double *crow = c + i * len;
        for (int64_t j = 0; j < len; ++j) crow[j] = 0.0;
        for (int64_t l = 0; l < len; ++l) {
            const double ail = (double)a[i * len + l];
            const float *brow = b + l * len;
            for (int64_t j = 0; j < len; ++j) crow[j] += ail * (double)brow[j];
        }
    }
}

void oracle_matmul_i32_ijl(int64_t len, const int32_t *a, const int32_t *b, int32_t *c)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < len; ++i)
        for (int64_t j = 0; j < len; ++j) {
            uint64_t sum = 0;
            for (int64_t l = 0; l < len; ++l)
                sum += (uint64_t)(int64_t)a[i * len + l] * (uint64_t)(int64_t)b[l * len + j];
            c[i * len + j] = (int32_t)(uint32_t)sum;
        }
}

void oracle_matmul_i32(int64_t len, const int32_t *a, const int32_t *b, int32_t *c)
{
#pragma omp parallel
    {
        uint64_t *acc = (uint64_t *)malloc((size_t)(len > 0 ? len : 1) * sizeof(uint64_t));
#pragma omp for schedule(static)
        for (int64_t i = 0; i < len; ++i) {
            for (int64_t j = 0; j < len; ++j) acc[j] = 0;
            for (int64_t l = 0; l < len; ++l) {
                const uint64_t ail = (uint64_t)(int64_t)a[i * len + l];
                const int32_t *brow = b + l * len;
                for (int64_t j = 0; j < len; ++j) acc[j] += ail * (uint64_t)(int64_t)brow[j];
            }
            for (int64_t j = 0; j < len; ++j) c[i * len + j] = (int32_t)(uint32_t)acc[j];
        }
        free(acc);
    }
}

/* Rows [row0, row0 + nrows) of C only, same arithmetic as the full product
 * (c holds nrows * len entries): a bounded slice of a large problem. */
void oracle_matmul_f32_rows(int64_t len, int64_t row0, int64_t nrows, const float *a, const float *b, double *c)
{
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < nrows; ++r) {
        const int64_t i = row0 + r;
        double *crow = c + r * len;
        for (int64_t j = 0; j < len; ++j) crow[j] = 0.0;
        for (int64_t l = 0; l < len; ++l) {
            const double ail = (double)a[i * len + l];
            const float *brow = b + l * len;
            for (int64_t j = 0; j < len; ++j) crow[j] += ail * (double)brow[j];
        }
    }
}

void oracle_matmul_i32_rows(int64_t len, int64_t row0, int64_t nrows, const int32_t *a, const int32_t *b,
                            int32_t *c)
{
#pragma omp parallel
    {
        uint64_t *acc = (uint64_t *)malloc((size_t)(len > 0 ? len : 1) * sizeof(uint64_t));
#pragma omp for schedule(static)
        for (int64_t r = 0; r < nrows; ++r) {
            const int64_t i = row0 + r;
            for (int64_t j = 0; j < len; ++j) acc[j] = 0;
            for (int64_t l = 0; l < len; ++l) {
                const uint64_t ail = (uint64_t)(int64_t)a[i * len + l];
                const int32_t *brow = b + l * len;
                for (int64_t j = 0; j < len; ++j) acc[j] += ail * (uint64_t)(int64_t)brow[j];
            }
            for (int64_t j = 0; j < len; ++j) c[r * len + j] = (int32_t)(uint32_t)acc[j];
        }
        free(acc);
    }
}

/* The same loop nest on rectangular operands with leading dimensions:
 * C (m x n) = A (m x k) B (k x n), row-major, element (i, j) of X at
 * x[i*ldx + j]; c[i*ldc + j] = sum over l ascending of a[i*lda+l]*b[l*ldb+j].
 * Listing 1a is the case m = n = k = LEN, lda = ldb = ldc = LEN. */
void oracle_gemm_f32(int64_t m, int64_t n, int64_t k, const float *a, int64_t lda, const float *b, int64_t ldb,
                     double *c, int64_t ldc)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < m; ++i) {
        double *crow = c + i * ldc;
        for (int64_t j = 0; j < n; ++j) crow[j] = 0.0;
        for (int64_t l = 0; l < k; ++l) {
            const double ail = (double)a[i * lda + l];
            const float *brow = b + l * ldb;
            for (int64_t j = 0; j < n; ++j) crow[j] += ail * (double)brow[j];
        }
    }
}

void oracle_gemm_i32(int64_t m, int64_t n, int64_t k, const int32_t *a, int64_t lda, const int32_t *b, int64_t ldb,
                     int32_t *c, int64_t ldc)
{
#pragma omp parallel
    {
        uint64_t *acc = (uint64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(uint64_t));
#pragma omp for schedule(static)
        for (int64_t i = 0; i < m; ++i) {
            for (int64_t j = 0; j < n; ++j) acc[j] = 0;
            for (int64_t l = 0; l < k; ++l) {
                const uint64_t ail = (uint64_t)(int64_t)a[i * lda + l];
                const int32_t *brow = b + l * ldb;
                for (int64_t j = 0; j < n; ++j) acc[j] += ail * (uint64_t)(int64_t)brow[j];
            }
            for (int64_t j = 0; j < n; ++j) c[i * ldc + j] = (int32_t)(uint32_t)acc[j];
        }
        free(acc);
    }
}

/* Selected entries only, each by the literal l-ascending loop: for sizes
 * where the full product would take too long on the host. */
void oracle_matmul_f32_at(int64_t len, const float *a, const float *b, int64_t m,
                          const int64_t *ii, const int64_t *jj, double *out)
{
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < m; ++s) {
        const int64_t i = ii[s], j = jj[s];
        double sum = 0.0;
        for (int64_t l = 0; l < len; ++l)
            sum += (double)a[i * len + l] * (double)b[l * len + j];
        out[s] = sum;
    }
}

void oracle_matmul_i32_at(int64_t len, const int32_t *a, const int32_t *b, int64_t m,
                          const int64_t *ii, const int64_t *jj, int32_t *out)
{
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < m; ++s) {
        const int64_t i = ii[s], j = jj[s];
        uint64_t sum = 0;
        for (int64_t l = 0; l < len; ++l)
            sum += (uint64_t)(int64_t)a[i * len + l] * (uint64_t)(int64_t)b[l * len + j];
        out[s] = (int32_t)(uint32_t)sum;
    }
}

/* ------------------------------------------------------------- reduction -- */

double oracle_sum_f32(int64_t n, const float *x, double init)
{
    double s = init;
    for (int64_t k = 0; k < n; ++k) s += (double)x[k];
    return s;
}

int32_t oracle_sum_i32(int64_t n, const int32_t *x, int32_t init)
{
    int64_t s = init;
    for (int64_t k = 0; k < n; ++k) s += x[k];
    return (int32_t)(uint32_t)(uint64_t)s;
}

/* --------------------------------------- reduction operators and types -- */
/* The reduction clause with the operators +, max, min and logical or
 * (section 2.3's reduction lowering; the BFS paragraph of section 4.2 names
 * a boolean "more nodes" flag, the SRAD paragraph a loop with two sum
 * variables).  One variable: out = init (op) f(x[0]) (op) f(x[1]) ... in
 * index order, where f(x) = x, or f(x) = x*x evaluated in the element type
 * (as the loop body `v += t * t` does in C).
 *   dtype 0 float32: + accumulates in double; max/min exact (fmax/fmin: a
 *                    NaN operand is ignored); out: double.
 *   dtype 1 int32:   + and * modulo 2^32; max/min signed; out: int32.
 *   dtype 2 float64: + accumulates in long double; out: double.
 *   dtype 3 int64:   + and * modulo 2^64; out: int64.
 *   op 3 (logical or): out = 1 if init or any x[k] compares unequal to zero,
 *                    else 0 (f must be the identity).
 * init points to one value of the element type. */
void oracle_reduce(int dtype, int op, int square, const void *x, int64_t n, const void *init, void *out)
{
    if (op == 3) {
        int any = 0;
        for (int64_t k = -1; k < n && !any; ++k) {
            const void *p = k < 0 ? init : x;
            const int64_t i = k < 0 ? 0 : k;
            switch (dtype) {
            case 0: any = ((const float *)p)[i] != 0.0f; break;
            case 1: any = ((const int32_t *)p)[i] != 0; break;
            case 2: any = ((const double *)p)[i] != 0.0; break;
            default: any = ((const int64_t *)p)[i] != 0; break;
            }
        }
        switch (dtype) {
        case 0: *(double *)out = any; break;
        case 1: *(int32_t *)out = any; break;
        case 2: *(double *)out = any; break;
        default: *(int64_t *)out = any; break;
        }
        return;
    }
    if (dtype == 0) {
        const float *v = (const float *)x;
        double acc = *(const float *)init;
        for (int64_t k = 0; k < n; ++k) {
            const float t = square ? v[k] * v[k] : v[k];
            acc = op == 0 ? acc + (double)t : op == 1 ? fmax(acc, (double)t) : fmin(acc, (double)t);
        }
        *(double *)out = acc;
    } else if (dtype == 2) {
        const double *v = (const double *)x;
        long double acc = *(const double *)init;
        for (int64_t k = 0; k < n; ++k) {
            const double t = square ? v[k] * v[k] : v[k];
            acc = op == 0 ? acc + (long double)t : op == 1 ? fmaxl(acc, (long double)t) : fminl(acc, (long double)t);
        }
        *(double *)out = (double)acc;
    } else if (dtype == 1) {
        const int32_t *v = (const int32_t *)x;
        uint32_t acc = (uint32_t) * (const int32_t *)init;
        for (int64_t k = 0; k < n; ++k) {
            const uint32_t t = square ? (uint32_t)v[k] * (uint32_t)v[k] : (uint32_t)v[k];
            if (op == 0)
                acc += t;
            else if (op == 1)
                acc = (int32_t)t > (int32_t)acc ? t : acc;
            else
                acc = (int32_t)t < (int32_t)acc ? t : acc;
        }
        *(int32_t *)out = (int32_t)acc;
    } else {
        const int64_t *v = (const int64_t *)x;
        uint64_t acc = (uint64_t) * (const int64_t *)init;
        for (int64_t k = 0; k < n; ++k) {
            const uint64_t t = square ? (uint64_t)v[k] * (uint64_t)v[k] : (uint64_t)v[k];
            if (op == 0)
                acc += t;
            else if (op == 1)
                acc = (int64_t)t > (int64_t)acc ? t : acc;
            else
                acc = (int64_t)t < (int64_t)acc ? t : acc;
        }
        *(int64_t *)out = (int64_t)acc;
    }
}

/* ------------------------------------------------------ bf16 3-term split -- */

static float bits_to_float(uint32_t u)
{
    float f;
    memcpy(&f, &u, sizeof f);
    return f;
}

static uint32_t float_to_bits(float f)
{
    uint32_t u;
    memcpy(&u, &f, sizeof u);
    return u;
}

/* Round a finite float to the nearest bfloat16, ties to the even pattern.
 * The two candidates are the float with the low 16 bits cleared (toward zero)
 * and the next bf16 pattern away from zero; distances are exact in double. */
uint16_t oracle_round_bf16(float x)
{
    const uint32_t u = float_to_bits(x);
    const uint32_t down = u & 0xFFFF0000u;
    const uint32_t up = down + 0x00010000u;
    const double dx = (double)x;
    const double dd = fabs(dx - (double)bits_to_float(down));
    const double du = fabs((double)bits_to_float(up) - dx);
    if (dd < du) return (uint16_t)(down >> 16);
    if (du < dd) return (uint16_t)(up >> 16);
    return (uint16_t)((((down >> 16) & 1u) == 0u) ? (down >> 16) : (up >> 16));
}

double oracle_bf16_value(uint16_t h) { return (double)bits_to_float((uint32_t)h << 16); }

void oracle_split_bf16x3(int64_t n, const float *x, uint16_t *hi, uint16_t *mid, uint16_t *lo)
{
    for (int64_t k = 0; k < n; ++k) {
        const double v = (double)x[k];
        const uint16_t h = oracle_round_bf16(x[k]);
        const double r1 = v - oracle_bf16_value(h);          /* exact */
        const uint16_t m = oracle_round_bf16((float)r1);     /* r1 is a float value */
        const double r2 = r1 - oracle_bf16_value(m);         /* exact */
        const uint16_t o = oracle_round_bf16((float)r2);
        hi[k] = h;
        mid[k] = m;
        lo[k] = o;
    }
}

/* --------------------------------------------------- int8 limb digits -- */

int64_t oracle_maxabs_i32(int64_t n, const int32_t *x)
{
    int64_t m = 0;
    for (int64_t k = 0; k < n; ++k) {
        const int64_t v = x[k] < 0 ? -(int64_t)x[k] : (int64_t)x[k];
        if (v > m) m = v;
    }
    return m;
}

/* Balanced base-256 digits: d_k in [-128, 127] with x == sum_k d_k * 256**k,
 * exactly for the first nl-1 digits' worth of range and mod 2**32 overall.
 * d[k*n + e] holds digit k of element e. */
void oracle_limbs_i8(int64_t n, const int32_t *x, int nl, int8_t *d)
{
    for (int64_t e = 0; e < n; ++e) {
        int64_t r = x[e];
        for (int k = 0; k < nl; ++k) {
            int64_t t = r + 128;
            int64_t q = t >= 0 ? t / 256 : -((-t + 255) / 256); /* floor(t / 256) */
            int64_t digit = t - q * 256 - 128;                   /* in [-128, 127] */
            d[(int64_t)k * n + e] = (int8_t)digit;
            r = (r - digit) / 256;                                /* exact */
        }
    }
}
