/* CPU oracle: declarations.  TEST INFRASTRUCTURE ONLY; see oracle.c. */
#ifndef ACCX_ORACLE_H
#define ACCX_ORACLE_H
#include <stdint.h>

void oracle_set_threads(int n);
int oracle_max_threads(void);

void oracle_matmul_f32_ijl(int64_t len, const float *a, const float *b, double *c);
void oracle_matmul_f32(int64_t len, const float *a, const float *b, double *c);
void oracle_matmul_i32_ijl(int64_t len, const int32_t *a, const int32_t *b, int32_t *c);
void oracle_matmul_i32(int64_t len, const int32_t *a, const int32_t *b, int32_t *c);
void oracle_matmul_f32_rows(int64_t len, int64_t row0, int64_t nrows, const float *a, const float *b, double *c);
void oracle_matmul_i32_rows(int64_t len, int64_t row0, int64_t nrows, const int32_t *a, const int32_t *b,
                            int32_t *c);
void oracle_gemm_f32(int64_t m, int64_t n, int64_t k, const float *a, int64_t lda, const float *b, int64_t ldb,
                     double *c, int64_t ldc);
void oracle_gemm_i32(int64_t m, int64_t n, int64_t k, const int32_t *a, int64_t lda, const int32_t *b, int64_t ldb,
                     int32_t *c, int64_t ldc);
void oracle_matmul_f32_at(int64_t len, const float *a, const float *b, int64_t m,
                          const int64_t *ii, const int64_t *jj, double *out);
void oracle_matmul_i32_at(int64_t len, const int32_t *a, const int32_t *b, int64_t m,
                          const int64_t *ii, const int64_t *jj, int32_t *out);

double oracle_sum_f32(int64_t n, const float *x, double init);
void oracle_reduce(int dtype, int op, int square, const void *x, int64_t n, const void *init, void *out);
int32_t oracle_sum_i32(int64_t n, const int32_t *x, int32_t init);

uint16_t oracle_round_bf16(float x);
double oracle_bf16_value(uint16_t h);
void oracle_split_bf16x3(int64_t n, const float *x, uint16_t *hi, uint16_t *mid, uint16_t *lo);

int64_t oracle_maxabs_i32(int64_t n, const int32_t *x);
void oracle_limbs_i8(int64_t n, const int32_t *x, int nl, int8_t *d);
#endif
