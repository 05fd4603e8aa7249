// The loop nest of Listing 1a (section 1.3) as a translator emits it: one
// lightweight thread per output element (i, j), the l loop run sequentially
// inside the thread, no data shared between threads ("output
// parallelization", the Matrix Multiplication paragraph of section 4.2).
//
// Two thread mappings:
//  - gang/vector (default): j on the 64 lanes of a wavefront, i on the
//    workgroup's y dimension and the grid.  Loads of b and stores of c are
//    coalesced along j; a[i][l] is the same address for the whole wavefront.
//  - Listing 1b's mapping: i = threadIdx.x + blockIdx.x*16,
//    j = threadIdx.y + blockIdx.y*16, 16x16 blocks.  Neighbouring lanes then
//    walk different rows of a (stride LEN) and store c with stride LEN.
// Both guard i < m, j < n, so any size is accepted (the listing's grid of
// LEN/16 blocks assumes 16 | LEN and has no guard).  The nest runs on
// rectangular operands with leading dimensions as well: C (m x n) =
// A (m x k) B (k x n); k = 0 gives C = 0.
//
// float: `sum` is float and each step is one fused multiply-add (the listing
// declares `float sum`; the contraction is the compiler's default).
// int: unsigned 32-bit multiply-add, i.e. wraparound modulo 2^32.
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace accx {
namespace {

template <typename T> struct Mac;
template <> struct Mac<float> {
    using Acc = float;
    __device__ static inline float step(float s, float x, float y) { return __builtin_fmaf(x, y, s); }
};
template <> struct Mac<int32_t> {
    using Acc = uint32_t;
    __device__ static inline uint32_t step(uint32_t s, int32_t x, int32_t y)
    {
        return s + (uint32_t)x * (uint32_t)y;
    }
};

constexpr int GV_X = 64;  // j lanes per wavefront
constexpr int GV_Y = 4;   // rows i per workgroup (one wavefront each)

// c[i*ldc + j] = sum over l of a[i*lda + l] * b[l*ldb + j], 0 <= i < m,
// 0 <= j < n (Listing 1a: m = n = k = lda = ldb = ldc = LEN).
template <typename T>
__global__ __launch_bounds__(GV_X *GV_Y) void matmul_plain_gv(const T *__restrict__ a, const T *__restrict__ b,
                                                              T *__restrict__ c, GemmShape sh)
{
    const int64_t j = (int64_t)blockIdx.x * GV_X + threadIdx.x;
    const int64_t i = (int64_t)blockIdx.y * GV_Y + threadIdx.y;
    if (i >= sh.m || j >= sh.n) return;
    const T *arow = a + i * sh.lda;
    const T *bcol = b + j;
    typename Mac<T>::Acc sum = 0;
    for (int64_t l = 0; l < sh.k; ++l) sum = Mac<T>::step(sum, arow[l], bcol[l * sh.ldb]);
    c[i * sh.ldc + j] = (T)sum;
}

template <typename T>
__global__ __launch_bounds__(256) void matmul_plain_listing1b(const T *__restrict__ a, const T *__restrict__ b,
                                                              T *__restrict__ c, GemmShape sh)
{
    const int64_t i = (int64_t)threadIdx.x + (int64_t)blockIdx.x * 16;
    const int64_t j = (int64_t)threadIdx.y + (int64_t)blockIdx.y * 16;
    if (i >= sh.m || j >= sh.n) return;
    typename Mac<T>::Acc sum = 0;
    for (int64_t l = 0; l < sh.k; ++l) sum = Mac<T>::step(sum, a[i * sh.lda + l], b[l * sh.ldb + j]);
    c[i * sh.ldc + j] = (T)sum;
}

// Grid y stays below 2^15 workgroups: the runtime caps m and n at 2^17, so
// (m + 3) / 4 and (n + 15) / 16 are at most 2^15.
template <typename T>
hipError_t launch(const T *a, const T *b, T *c, const GemmShape &sh, bool listing1b, hipStream_t s)
{
    if (sh.m <= 0 || sh.n <= 0) return hipSuccess;
    if (listing1b) {
        const dim3 grid((unsigned)((sh.m + 15) / 16), (unsigned)((sh.n + 15) / 16));
        tmark("matmul_plain_listing1b", s, true);
        hipLaunchKernelGGL(matmul_plain_listing1b<T>, grid, dim3(16, 16), 0, s, a, b, c, sh);
        tmark("matmul_plain_listing1b", s, false);
    } else {
        const dim3 grid((unsigned)((sh.n + GV_X - 1) / GV_X), (unsigned)((sh.m + GV_Y - 1) / GV_Y));
        tmark("matmul_plain", s, true);
        hipLaunchKernelGGL(matmul_plain_gv<T>, grid, dim3(GV_X, GV_Y), 0, s, a, b, c, sh);
        tmark("matmul_plain", s, false);
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_matmul_plain_f32(const float *a, const float *b, float *c, const GemmShape &sh, bool listing1b,
                                   hipStream_t s)
{
    return launch<float>(a, b, c, sh, listing1b, s);
}

hipError_t launch_matmul_plain_i32(const int32_t *a, const int32_t *b, int32_t *c, const GemmShape &sh,
                                   bool listing1b, hipStream_t s)
{
    return launch<int32_t>(a, b, c, sh, listing1b, s);
}

}  // namespace accx
