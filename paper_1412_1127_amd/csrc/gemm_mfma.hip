// The loop nest of Listing 1a (section 1.3) on the matrix cores of gfx950,
// tiled through LDS.  This is the MI355X form of what the Matrix
// Multiplication paragraph of section 4.2 credits for the CUDA version's
// speed: a workgroup fetches input tiles with a few wide, coalesced accesses
// into the software-managed on-chip memory and shares them among its threads,
// instead of each thread streaming a row of a and a column of b by itself.
//
// Two element paths share one tiled kernel:
//  - float32 on bf16 matrix cores ("bf16x3"): each operand x is split into
//    three bf16 terms x = hi + mid + lo (hi = RN(x), mid = RN(x - hi),
//    lo = RN(x - hi - mid), RN = round to nearest even); C accumulates in
//    float32 the products of term pairs (p, q): all six with p+q <= 2
//    (FULL6), those five without mid*mid (FIVE), or the three with p+q <= 1
//    (CHEAP3).
//  - int32 on int8 matrix cores: each operand is written in balanced
//    base-256 digits d_k in [-128, 127], x = sum d_k 256^k (mod 2^32); C is
//    the sum over digit pairs (k, m) with k+m <= 3 of (A_k B_m) << 8(k+m),
//    modulo 2^32.  Products with the same shift share an int32 accumulator.
//
// Packed operand layout (written by the pack kernels below, read by the
// GEMM).  An operand of R rows of K elements (A: rows of A; B: columns of B,
// i.e. rows of B^T) with P planes is cut into units of 32 rows x 64 bytes of
// each plane.  Unit (rb, kb) starts at byte (rb*nkb + kb) * P * 2048; inside
// it, plane p, 16-byte chunk c (0..3) of row r (0..31) is at
// p*2048 + c*512 + r*16.  Rows >= R and elements >= K are zero.  The layout
// makes every global->LDS copy a contiguous 1 KB block (one direct-to-LDS
// dwordx4 load per wavefront) and every matrix-core operand fetch a
// conflict-free ds_read_b128 of 1 KB (lane l: row l%32, chunk l/32).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "kernels.h"
#include "mfma_tile.h"

namespace accx {
namespace {

using namespace dev;

// One thread per (unit, row, chunk): 8 consecutive K elements of one row.
template <bool TRANS>
__global__ __launch_bounds__(256) void pack_bf16x3(const float *__restrict__ X, int64_t R, int64_t K, int64_t ld,
                                                   char *__restrict__ out, int64_t nrb, int64_t nkb)
{
    pack_bf16x3_range<TRANS>(X, R, K, ld, out, nrb, nkb, (int64_t)blockIdx.x * 256 + threadIdx.x,
                             (int64_t)gridDim.x * 256);
}


// Digit 0 of four consecutive elements, packed into one word: the balanced
// base-256 digit ((x + 128) mod 256) - 128 is the low byte of x read as int8.
__device__ inline int low_bytes4(int32_t a, int32_t b, int32_t c, int32_t d)
{
    return (int)(((uint32_t)a & 255u) | (((uint32_t)b & 255u) << 8) | (((uint32_t)c & 255u) << 16) |
                 ((uint32_t)d << 24));
}

// Record a workgroup's max |x| (256 threads, each holding its own max) in
// the operand's word *maxabs (stamp << 32 | max, see recorded_max).  Only
// maxima above 127 are recorded: the digit count depends on max |x| only
// through thresholds from 127 up, so the word ends as this call's stamp and
// the operand's max |x| when that exceeds 127, and is left as it was
// otherwise.  A compare-and-swap loop replaces a word that carries another
// stamp or a smaller maximum; none on one-digit data, and few once the
// largest maxima are in (a single contended address serialises every atomic
// on it).
__device__ inline void block_max_record(uint32_t mx, uint64_t *maxabs, uint32_t stamp)
{
    __shared__ uint32_t wmax[4];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const uint32_t t = __shfl_xor(mx, o, 64);
        mx = t > mx ? t : mx;
    }
    if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t m = wmax[0];
#pragma unroll
        for (int w = 1; w < 4; ++w) m = wmax[w] > m ? wmax[w] : m;
        if (m > 127u) {
            uint64_t w = __hip_atomic_load(maxabs, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const uint64_t want = ((uint64_t)stamp << 32) | m;
            while (recorded_max(w, stamp) < m &&
                   !__hip_atomic_compare_exchange_strong(maxabs, &w, want, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                         __HIP_MEMORY_SCOPE_AGENT)) {
            }
        }
    }
}

// int32 -> the first `nplanes` balanced base-256 digit planes (int8) of a
// packed operand whose units hold `pstride` planes, 16 K elements per
// thread.  Element addressing as for the bf16x3 pack (leading dimension ld).
// Work item id in [id0, total) by `step`; returns the thread's max |x|.
template <bool TRANS>
__device__ inline uint32_t pack_i8_items(const int32_t *__restrict__ X, int64_t R, int64_t K, int64_t ld,
                                         char *__restrict__ out, int64_t nrb, int64_t nkb, int nplanes, int pstride,
                                         int64_t id0, int64_t step)
{
    const int64_t total = nrb * nkb * 128;
    uint32_t mx = 0;
    for (int64_t id = id0; id < total; id += step) {
        const int64_t unit = id >> 7;
        const int w = (int)(id & 127);
        int r, c;
        if (TRANS) {
            r = w & 31;
            c = w >> 5;
        } else {
            r = w >> 2;
            c = w & 3;
        }
        const int64_t rb = unit / nkb, kb = unit - rb * nkb;
        const int64_t row = rb * 32 + r;
        const int64_t k0 = kb * 64 + c * 16;
        int32_t v[16];
        if (!TRANS && row < R && k0 + 16 <= K && ((ld & 3) == 0) && (((uintptr_t)X & 15u) == 0)) {
            const i32x4 *p = reinterpret_cast<const i32x4 *>(X + row * ld + k0);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const i32x4 w4 = p[q];
                v[4 * q] = w4.x, v[4 * q + 1] = w4.y, v[4 * q + 2] = w4.z, v[4 * q + 3] = w4.w;
            }
        } else {
#pragma unroll
            for (int t = 0; t < 16; ++t) {
                const bool in = row < R && k0 + t < K;
                v[t] = in ? (TRANS ? X[(k0 + t) * ld + row] : X[row * ld + k0 + t]) : 0;
            }
        }
#pragma unroll
        for (int t = 0; t < 16; ++t) {
            const uint32_t a = v[t] < 0 ? (uint32_t)0 - (uint32_t)v[t] : (uint32_t)v[t];
            mx = a > mx ? a : mx;
        }
        char *u = out + unit * ((int64_t)pstride * PLANE_BYTES) + c * 512 + r * 16;
        if (nplanes == 1) {  // one digit: the low bytes, no carries to follow
            *reinterpret_cast<i32x4 *>(u) = i32x4{low_bytes4(v[0], v[1], v[2], v[3]), low_bytes4(v[4], v[5], v[6], v[7]),
                                                  low_bytes4(v[8], v[9], v[10], v[11]),
                                                  low_bytes4(v[12], v[13], v[14], v[15])};
            continue;
        }
        int64_t rem[16];
#pragma unroll
        for (int t = 0; t < 16; ++t) rem[t] = v[t];
        for (int p = 0; p < nplanes; ++p) {
            i32x4 word = {0, 0, 0, 0};
#pragma unroll
            for (int t = 0; t < 16; ++t) {
                const int d = (int)(((uint32_t)rem[t] + 128u) & 255u) - 128;  // in [-128, 127]
                rem[t] = (rem[t] - d) >> 8;                                     // exact division by 256
                word[t >> 2] |= (int)((uint32_t)(uint8_t)(int8_t)d << (8 * (t & 3)));
            }
            *reinterpret_cast<i32x4 *>(u + (int64_t)p * PLANE_BYTES) = word;
        }
    }
    return mx;
}

// One digit (the low byte of each element) of int32 rows into the packed
// layout, with coalesced loads: a wavefront takes 4 rows x 64 elements of one
// unit (lane l: row l / 16, elements 4 (l % 16) .. +3 -- one 16-byte load;
// 16 lanes read a row's 256 bytes), packs the low bytes of its four elements
// into one word and stores it at its place in the unit (four lanes fill one
// 16-byte chunk).  Work items are (32-row block, 4-row group, K unit), K
// fastest, so that consecutive wavefronts walk along the same rows; each
// wavefront keeps NI items' loads in flight.  w0 / wstep: this wavefront's
// first item and the number of wavefronts.  Returns the lane's max |x|.
__device__ inline uint32_t pack_i8_rows_one(const int32_t *__restrict__ X, int64_t R, int64_t K, int64_t ld,
                                            char *__restrict__ out, int64_t nrb, int64_t nkb, int pstride, int64_t w0,
                                            int64_t wstep)
{
    constexpr int NI = 4;
    const int lane = threadIdx.x & 63;
    const int lr = lane >> 4, lk = (lane & 15) * 4;
    const int64_t items = nrb * 8 * nkb;
    const bool vec = ((ld & 3) == 0) && ((((uintptr_t)X) & 15u) == 0);
    uint32_t mx = 0;
    for (int64_t i0 = w0; i0 < items; i0 += (int64_t)NI * wstep) {
        i32x4 v[NI];
#pragma unroll
        for (int u = 0; u < NI; ++u) {
            const int64_t it = i0 + u * wstep;
            v[u] = i32x4{0, 0, 0, 0};
            if (it < items) {
                const int64_t kb = it % nkb, rq = it / nkb;  // rq = 32-row block * 8 + row group
                const int64_t row = rq * 4 + lr, k = kb * 64 + lk;
                if (row < R) {
                    if (vec && k + 4 <= K) {
                        v[u] = __builtin_nontemporal_load(reinterpret_cast<const i32x4 *>(X + row * ld + k));
                    } else {
#pragma unroll
                        for (int e = 0; e < 4; ++e)
                            if (k + e < K) v[u][e] = X[row * ld + k + e];
                    }
                }
            }
        }
#pragma unroll
        for (int u = 0; u < NI; ++u) {
            const int64_t it = i0 + u * wstep;
            if (it >= items) break;
            const int64_t kb = it % nkb, rq = it / nkb;
            const int64_t rb = rq >> 3;
            const int r = (int)(rq & 7) * 4 + lr;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const uint32_t a = v[u][e] < 0 ? (uint32_t)0 - (uint32_t)v[u][e] : (uint32_t)v[u][e];
                mx = a > mx ? a : mx;
            }
            char *o = out + (rb * nkb + kb) * ((int64_t)pstride * PLANE_BYTES) + (lk >> 4) * 512 + r * 16 +
                      (lk & 15);
            *reinterpret_cast<int *>(o) = low_bytes4(v[u][0], v[u][1], v[u][2], v[u][3]);
        }
    }
    return mx;
}

template <bool TRANS>
__global__ __launch_bounds__(256) void pack_i8(const int32_t *__restrict__ X, int64_t R, int64_t K, int64_t ld,
                                               char *__restrict__ out, int64_t nrb, int64_t nkb, int nplanes)
{
    (void)pack_i8_items<TRANS>(X, R, K, ld, out, nrb, nkb, nplanes, nplanes, (int64_t)blockIdx.x * 256 + threadIdx.x,
                               (int64_t)gridDim.x * 256);
}


// ---- transposed operands (B^T): packing through an LDS transpose ----------
//
// Operand row r is column r of the K x R row-major array X, so one 32-row
// unit touches only 128 bytes of each row of X.  A workgroup therefore
// stages a tile of TP_ROWS rows x 256 columns of X in LDS, each row read as
// one coalesced 1 KB segment, and then builds 16-byte chunks of eight 32-row
// units from LDS columns (consecutive lanes read consecutive columns: no
// bank conflicts).  16 rows (16 KB of LDS) rather than 32: the pair kernels
// give every workgroup, those packing A too, the transpose's LDS, and at
// 32 KB it held them to five per CU.
constexpr int TP_COLS = 256;         // columns of X per tile (eight units)
constexpr int TP_ROWS = 16;          // rows of X per tile
constexpr int BF_SPLIT = 32 / TP_ROWS;  // tiles per 32-element bf16x3 K unit
constexpr int I8_SPLIT = 64 / TP_ROWS;  // tiles per 64-element int8 K unit

__device__ inline void stage_rows(const uint32_t *__restrict__ X, int64_t R, int64_t K, int64_t ld, int64_t k0,
                                  int64_t c0, uint32_t (*t)[TP_COLS])
{
    // TP_ROWS rows x 64 four-column groups, TP_ROWS / 4 per thread
    const bool vec = ((ld & 3) == 0) && ((((uintptr_t)X) & 15u) == 0);
#pragma unroll
    for (int j = 0; j < TP_ROWS * 64 / 256; ++j) {
        const int q = j * 256 + threadIdx.x;
        const int row = q >> 6, c4 = (q & 63) * 4;
        const int64_t k = k0 + row, col = c0 + c4;
        uint32_t w[4] = {0u, 0u, 0u, 0u};
        if (k < K) {
            if (vec && col + 4 <= R) {
                const u32x4_t v = __builtin_nontemporal_load(reinterpret_cast<const u32x4_t *>(X + k * ld + col));
                w[0] = v.x, w[1] = v.y, w[2] = v.z, w[3] = v.w;
            } else {
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    if (col + e < R) w[e] = X[k * ld + col + e];
            }
        }
        *reinterpret_cast<u32x4_t *>(&t[row][c4]) = u32x4_t{w[0], w[1], w[2], w[3]};
    }
}

// bf16x3 planes of B^T for column tile bx of X and part by % BF_SPLIT of
// the 32-element K unit by / BF_SPLIT.
__device__ inline void pack_bf16x3_cols(const float *__restrict__ X, int64_t R, int64_t K, int64_t ld,
                                        char *__restrict__ out, int64_t nrb, int64_t nkb, int64_t bx, int64_t by,
                                        uint32_t (*t)[TP_COLS])
{
    constexpr int CPT = TP_ROWS / 8;  // 8-element chunks per row per tile
    const int64_t kb = by / BF_SPLIT, rb0 = bx * (TP_COLS / 32);
    const int part = (int)(by % BF_SPLIT);
    stage_rows(reinterpret_cast<const uint32_t *>(X), R, K, ld, kb * 32 + part * TP_ROWS, rb0 * 32, t);
    __syncthreads();
    // 8 units x 32 rows x CPT chunks of 8 elements
#pragma unroll
    for (int j = 0; j < 8 * 32 * CPT / 256; ++j) {
        const int q = j * 256 + threadIdx.x;
        const int r = q & 31, c = (q >> 5) % CPT, u = q / (32 * CPT);
        if (rb0 + u >= nrb) continue;
        u16x8 h, m, l;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            uint16_t a, b, d;
            split3(__uint_as_float(t[c * 8 + e][u * 32 + r]), a, b, d);
            h[e] = a;
            m[e] = b;
            l[e] = d;
        }
        char *o = out + ((rb0 + u) * nkb + kb) * (3 * PLANE_BYTES) + (part * CPT + c) * 512 + r * 16;
        *reinterpret_cast<u16x8 *>(o) = h;
        *reinterpret_cast<u16x8 *>(o + PLANE_BYTES) = m;
        *reinterpret_cast<u16x8 *>(o + 2 * PLANE_BYTES) = l;
    }
}

// Grid: gbx column tiles of X per K tile, BF_SPLIT K tiles per K unit.
__global__ __launch_bounds__(256) void pack_bf16x3_t(const float *__restrict__ X, int64_t R, int64_t K, int64_t ld,
                                                     char *__restrict__ out, int64_t nrb, int64_t nkb, int gbx)
{
    __shared__ __attribute__((aligned(16))) uint32_t t[TP_ROWS][TP_COLS];
    pack_bf16x3_cols(X, R, K, ld, out, nrb, nkb, blockIdx.x % gbx, blockIdx.x / gbx, t);
}

// A and B^T of one product in one launch (one kernel start instead of two):
// workgroups [0, ga) pack the rows of A, the others column tiles of B
// (gbx per K tile).
__global__ __launch_bounds__(256) void pack_bf16x3_pair(const float *__restrict__ A, int64_t M, int64_t lda,
                                                        char *__restrict__ pa, const float *__restrict__ B, int64_t N,
                                                        int64_t ldb, char *__restrict__ pb, int64_t K, int ga, int gbx)
{
    __shared__ __attribute__((aligned(16))) uint32_t t[TP_ROWS][TP_COLS];
    const int64_t nkb = (K + 31) / 32;
    if ((int)blockIdx.x < ga) {
        pack_bf16x3_range<false>(A, M, K, lda, pa, (M + 31) / 32, nkb, (int64_t)blockIdx.x * 256 + threadIdx.x,
                                 (int64_t)ga * 256);
    } else {
        const int64_t b = blockIdx.x - ga;
        pack_bf16x3_cols(B, N, K, ldb, pb, (N + 31) / 32, nkb, b % gbx, b / gbx, t);
    }
}

// ---- float32 operands for the float32 matrix cores: one plane of 4-byte
// elements in the same unit layout (32 rows x 16 elements per unit, chunk c
// of row r = elements 4c..4c+3 at c*512 + r*16).  A plain copy into the
// layout; B^T goes through the LDS transpose (a 16-element K unit is one
// staged tile of TP_ROWS = 16 rows of X).
static_assert(TP_ROWS == 16, "one float32 K unit per staged tile");

// Rows of A: one thread per (unit, row, chunk), work items id0, id0 + step, ...
__device__ inline void pack_f32_range(const float *__restrict__ X, int64_t R, int64_t K, int64_t ld,
                                      char *__restrict__ out, int64_t nrb, int64_t nkb, int64_t id0, int64_t step)
{
    const int64_t total = nrb * nkb * 128;
    for (int64_t id = id0; id < total; id += step) {
        const int64_t unit = id >> 7;
        const int w = (int)(id & 127);
        const int r = w >> 2, c = w & 3;
        const int64_t rb = unit / nkb, kb = unit - rb * nkb;
        const int64_t row = rb * 32 + r, k0 = kb * 16 + c * 4;
        f32x4 v = {0.0f, 0.0f, 0.0f, 0.0f};
        if (row < R && k0 + 4 <= K && ((ld & 3) == 0) && (((uintptr_t)X & 15u) == 0)) {
            v = *reinterpret_cast<const f32x4 *>(X + row * ld + k0);
        } else if (row < R) {
#pragma unroll
            for (int t = 0; t < 4; ++t) v[t] = k0 + t < K ? X[row * ld + k0 + t] : 0.0f;
        }
        *reinterpret_cast<f32x4 *>(out + unit * PLANE_BYTES + c * 512 + r * 16) = v;
    }
}

// B^T for column tile bx of X and K unit kb.
__device__ inline void pack_f32_cols(const float *__restrict__ X, int64_t R, int64_t K, int64_t ld,
                                     char *__restrict__ out, int64_t nrb, int64_t nkb, int64_t bx, int64_t kb,
                                     uint32_t (*t)[TP_COLS])
{
    const int64_t rb0 = bx * (TP_COLS / 32);
    stage_rows(reinterpret_cast<const uint32_t *>(X), R, K, ld, kb * 16, rb0 * 32, t);
    __syncthreads();
    // 8 units x 32 rows x 4 chunks of 4 elements
#pragma unroll
    for (int j = 0; j < 8 * 32 * 4 / 256; ++j) {
        const int q = j * 256 + threadIdx.x;
        const int r = q & 31, c = (q >> 5) & 3, u = q >> 7;
        if (rb0 + u >= nrb) continue;
        const f32x4 v = {__uint_as_float(t[4 * c][u * 32 + r]), __uint_as_float(t[4 * c + 1][u * 32 + r]),
                         __uint_as_float(t[4 * c + 2][u * 32 + r]), __uint_as_float(t[4 * c + 3][u * 32 + r])};
        *reinterpret_cast<f32x4 *>(out + ((rb0 + u) * nkb + kb) * PLANE_BYTES + c * 512 + r * 16) = v;
    }
}

__global__ __launch_bounds__(256) void pack_f32_a(const float *__restrict__ X, int64_t R, int64_t K, int64_t ld,
                                                  char *__restrict__ out, int64_t nrb, int64_t nkb)
{
    pack_f32_range(X, R, K, ld, out, nrb, nkb, (int64_t)blockIdx.x * 256 + threadIdx.x, (int64_t)gridDim.x * 256);
}

// Grid: gbx column tiles of X per K unit.
__global__ __launch_bounds__(256) void pack_f32_t(const float *__restrict__ X, int64_t R, int64_t K, int64_t ld,
                                                  char *__restrict__ out, int64_t nrb, int64_t nkb, int gbx)
{
    __shared__ __attribute__((aligned(16))) uint32_t t[TP_ROWS][TP_COLS];
    pack_f32_cols(X, R, K, ld, out, nrb, nkb, blockIdx.x % gbx, blockIdx.x / gbx, t);
}

// A and B^T in one launch: workgroups [0, ga) pack A, the others B.
__global__ __launch_bounds__(256) void pack_f32_pair(const float *__restrict__ A, int64_t M, int64_t lda,
                                                     char *__restrict__ pa, const float *__restrict__ B, int64_t N,
                                                     int64_t ldb, char *__restrict__ pb, int64_t K, int ga, int gbx)
{
    __shared__ __attribute__((aligned(16))) uint32_t t[TP_ROWS][TP_COLS];
    const int64_t nkb = (K + 15) / 16;
    if ((int)blockIdx.x < ga) {
        pack_f32_range(A, M, K, lda, pa, (M + 31) / 32, nkb, (int64_t)blockIdx.x * 256 + threadIdx.x,
                       (int64_t)ga * 256);
    } else {
        const int64_t b = blockIdx.x - ga;
        pack_f32_cols(B, N, K, ldb, pb, (N + 31) / 32, nkb, b % gbx, b / gbx, t);
    }
}

// The first `nplanes` int8 digit planes (of `pstride` per unit) of B^T for
// column tile bx of X and part by % I8_SPLIT of the 64-element K unit
// by / I8_SPLIT; returns the thread's max |x|.
// ONE: nplanes is 1 (the multi-digit code is left out of the kernel).
template <bool ONE>
__device__ inline uint32_t pack_i8_cols(const int32_t *__restrict__ X, int64_t R, int64_t K, int64_t ld,
                                        char *__restrict__ out, int64_t nrb, int64_t nkb, int nplanes, int pstride,
                                        int64_t bx, int64_t by, uint32_t (*t)[TP_COLS])
{
    constexpr int CPT = TP_ROWS / 16;  // 16-element chunks per row per tile
    const int64_t kb = by / I8_SPLIT, rb0 = bx * (TP_COLS / 32);
    const int part = (int)(by % I8_SPLIT);
    stage_rows(reinterpret_cast<const uint32_t *>(X), R, K, ld, kb * 64 + part * TP_ROWS, rb0 * 32, t);
    __syncthreads();
    uint32_t mx = 0;
    // 8 units x 32 rows x CPT chunks of 16 elements
#pragma unroll
    for (int j = 0; j < 8 * 32 * CPT / 256; ++j) {
        const int q = j * 256 + threadIdx.x;
        const int r = q & 31, c = (q >> 5) % CPT, u = q / (32 * CPT);
        if (rb0 + u >= nrb) continue;
        int32_t x[16];
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            x[e] = (int32_t)t[c * 16 + e][u * 32 + r];
            const uint32_t a = x[e] < 0 ? (uint32_t)0 - (uint32_t)x[e] : (uint32_t)x[e];
            mx = a > mx ? a : mx;
        }
        char *o = out + ((rb0 + u) * nkb + kb) * ((int64_t)pstride * PLANE_BYTES) + (part * CPT + c) * 512 + r * 16;
        if (ONE || nplanes == 1) {  // one digit: the low bytes
            *reinterpret_cast<i32x4 *>(o) = i32x4{low_bytes4(x[0], x[1], x[2], x[3]), low_bytes4(x[4], x[5], x[6], x[7]),
                                                  low_bytes4(x[8], x[9], x[10], x[11]),
                                                  low_bytes4(x[12], x[13], x[14], x[15])};
            continue;
        }
        int64_t rem[16];
#pragma unroll
        for (int e = 0; e < 16; ++e) rem[e] = x[e];
        for (int p = 0; p < nplanes; ++p) {
            i32x4 word = {0, 0, 0, 0};
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                const int d = (int)(((uint32_t)rem[e] + 128u) & 255u) - 128;  // in [-128, 127]
                rem[e] = (rem[e] - d) >> 8;                                     // exact division by 256
                word[e >> 2] |= (int)((uint32_t)(uint8_t)(int8_t)d << (8 * (e & 3)));
            }
            *reinterpret_cast<i32x4 *>(o + (int64_t)p * PLANE_BYTES) = word;
        }
    }
    return mx;
}

// Grid: gbx column tiles of X per K tile, I8_SPLIT K tiles per K unit.
__global__ __launch_bounds__(256) void pack_i8_t(const int32_t *__restrict__ X, int64_t R, int64_t K, int64_t ld,
                                                 char *__restrict__ out, int64_t nrb, int64_t nkb, int nplanes, int gbx)
{
    __shared__ __attribute__((aligned(16))) uint32_t t[TP_ROWS][TP_COLS];
    (void)pack_i8_cols<false>(X, R, K, ld, out, nrb, nkb, nplanes, nplanes, blockIdx.x % gbx, blockIdx.x / gbx, t);
}

// A and B^T of one product in one launch: workgroups [0, ga) pack the rows of
// A (max |x| into maxabs[0]), the others the gb column tiles of B (gbx per K
// tile, taken grid-stride; maxabs[1]).  Units hold `pstride` planes, of
// which `nplanes` are written.  maxabs (optional): the two max|x| words of
// this call (stamp `stamp`), as block_max_record leaves them.
// decide (optional): the two max|x| words of a finished one-digit pass; the
// launch is then the multi-digit pass: it runs only if more than one digit
// is needed and writes that many planes (nplanes is ignored).
// ONE: one digit (nplanes = 1, no decide): coalesced row packing for A and no
// multi-digit code in the kernel (fewer registers, more wavefronts per CU).
template <bool ONE>
__global__ __launch_bounds__(256) void pack_i8_pair(const int32_t *__restrict__ A, int64_t M, int64_t lda,
                                                    char *__restrict__ pa, const int32_t *__restrict__ B, int64_t N,
                                                    int64_t ldb, char *__restrict__ pb, int64_t K, int nplanes,
                                                    int pstride, int ga, int gbx, int64_t gb,
                                                    uint64_t *__restrict__ maxabs, const uint64_t *__restrict__ decide,
                                                    uint32_t stamp)
{
    int np = nplanes;
    if (decide) {
        np = limbs_needed(decide, stamp);
        if (np == 1) return;  // uniform: the whole grid exits
    }
    __shared__ __attribute__((aligned(16))) uint32_t t[TP_ROWS][TP_COLS];
    const int64_t nkb = (K + 63) / 64;
    uint32_t mx = 0;
    if ((int)blockIdx.x < ga) {
        if constexpr (ONE)
            mx = pack_i8_rows_one(A, M, K, lda, pa, (M + 31) / 32, nkb, pstride,
                                  (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6), (int64_t)ga * 4);
        else
            mx = pack_i8_items<false>(A, M, K, lda, pa, (M + 31) / 32, nkb, np, pstride,
                                      (int64_t)blockIdx.x * 256 + threadIdx.x, (int64_t)ga * 256);
    } else {
        // the staging buffer is reused: a barrier before each refill
        for (int64_t b = blockIdx.x - ga; b < gb; b += gridDim.x - ga) {
            const uint32_t m =
                pack_i8_cols<ONE>(B, N, K, ldb, pb, (N + 31) / 32, nkb, np, pstride, b % gbx, b / gbx, t);
            mx = m > mx ? m : mx;
            __syncthreads();
        }
    }
    if (maxabs) block_max_record(mx, maxabs + ((int)blockIdx.x < ga ? 0 : 1), stamp);
}


// One workgroup's tile (or split-K part of a tile) of gemm_packed.
template <bool INT8, int P, int BM, int BN, int KBK, int WGM, int WGN, int NS, int NPROD, uint64_t PL, int NACC,
          int LAM, bool F32MM, bool RED = false>
__device__ __attribute__((always_inline)) inline void gemm_packed_body(const GemmArgs &g, char *lds)
{
    int tm, tn;
    const int T = g.tiles_m * g.tiles_n;
    const int t = (int)(blockIdx.x % (unsigned)T);  // split K: part blockIdx.x / T of tile t
    tile_of(t, g.tiles_m, g.tiles_n, tm, tn);
    // probe records are per tile of the probed pass, which may be larger
    if (g.probe && !g.probe[(tm >> g.probe_shm) * g.probe_tiles_n + (tn >> g.probe_shn)].corrected)
        return;                                                          // whole workgroup: uniform
    if (g.decide && !limb_gate(g.decide, g.gen, g.expect)) return;      // the whole grid: uniform
    if (g.ksplit > 1) {
        GemmArgs h = g;
        h.split = (int)(blockIdx.x / (unsigned)T);
        h.tile = t;
        const int64_t kb0 = (int64_t)h.split * g.kb_count;
        h.kb_count = kb0 + g.kb_count <= g.nkb ? g.kb_count : g.nkb - kb0;
        const int64_t off = kb0 * (int64_t)P * PLANE_BYTES;
        h.A = g.A + off;
        h.B = g.B + off;
        gemm_tile<INT8, P, BM, BN, KBK, WGM, WGN, NS, NPROD, PL, NACC, LAM, F32MM>(h, tm, tn, lds);
    } else {
        gemm_tile<INT8, P, BM, BN, KBK, WGM, WGN, NS, NPROD, PL, NACC, LAM, F32MM, RED>(g, tm, tn, lds);
    }
}

template <bool INT8, int P, int BM, int BN, int KBK, int WGM, int WGN, int NS, int NPROD, uint64_t PL, int NACC,
          int LAM, bool F32MM, bool RED = false>
__global__ __launch_bounds__(WGM *WGN * 64) void gemm_packed(GemmArgs g)
{
    __shared__ __attribute__((aligned(1024)))
    char lds[gemm_lds_bytes<BM, BN, KBK, NS, NPROD, PL>() + (RED ? red_lds_bytes<WGM * WGN * 64, NS>() : 0)];
    gemm_packed_body<INT8, P, BM, BN, KBK, WGM, WGN, NS, NPROD, PL, NACC, LAM, F32MM, RED>(g, lds);
}

// int32 with several int8 digits per operand (packed units of P planes), on
// 128 x 128 tiles of 8 wavefronts (64 x 32 each, one int32 accumulator set
// per shift group), two LDS stages.  A persistent grid takes the tiles
// grid-stride, so that the launch costs little when it exits at once.  The
// digit count comes from the device (g.decide: the max|x| words of the
// one-digit pass; the kernel exits when one digit is enough) or from the
// caller (g.expect).  Digit pairs (k, m) below the count with k + m <= 3:
// 4 products for two digits, 8 for three, 10 for four.
constexpr int I8M_BM = 128, I8M_BN = 128, I8M_KBK = 64, I8M_WGM = 2, I8M_WGN = 4, I8M_NS = 2;
template <int P> constexpr int i8_multi_lds_bytes()
{
    return gemm_lds_bytes<I8M_BM, I8M_BN, I8M_KBK, I8M_NS, P >= 4 ? 10 : P == 3 ? 8 : 4,
                          P >= 4 ? PL_L4 : P == 3 ? PL_L3 : PL_L2>();
}

// The tiles of the multi-digit product with nd digits, grid-stride.
template <int P>
__device__ __attribute__((always_inline)) inline void gemm_i8_multi_body(const GemmArgs &g, int nd, char *lds)
{
    constexpr int BM = I8M_BM, BN = I8M_BN, KBK = I8M_KBK, WGM = I8M_WGM, WGN = I8M_WGN, NS = I8M_NS;
    const int T = g.tiles_m * g.tiles_n;
    for (int t = blockIdx.x; t < T; t += gridDim.x) {
        int tm, tn;
        tile_of(t, g.tiles_m, g.tiles_n, tm, tn);
        if (nd == 2) {
            gemm_tile<true, P, BM, BN, KBK, WGM, WGN, NS, 4, PL_L2, 3>(g, tm, tn, lds);
        } else if constexpr (P >= 3) {
            if (P == 3 || nd == 3) {
                gemm_tile<true, P, BM, BN, KBK, WGM, WGN, NS, 8, PL_L3, 4>(g, tm, tn, lds);
            } else if constexpr (P >= 4) {
                gemm_tile<true, P, BM, BN, KBK, WGM, WGN, NS, 10, PL_L4, 4>(g, tm, tn, lds);
            }
        }
        __syncthreads();  // every wavefront is done with the LDS stages before the next tile's loads
    }
}

template <int P>
__global__ __launch_bounds__(512) void gemm_i8_multi(GemmArgs g)
{
    __shared__ __attribute__((aligned(1024))) char lds[i8_multi_lds_bytes<P>()];
    const int nd = g.decide ? limbs_needed(g.decide, g.gen) : g.expect;
    if (nd < 2) return;  // uniform: the whole grid exits
    gemm_i8_multi_body<P>(g, nd, lds);
}

// The automatic int32 path on the one-digit 256 x 256 tile: one launch that
// runs either that tile (g, one workgroup per tile or split-K part) or, when
// the one-digit pass's maxima call for more digits, the multi-digit product
// (gm: four-plane operands, 128 x 128 tiles taken grid-stride by the same
// workgroups).  Saves the launch of the multi-digit kernel that would exit at
// once on one-digit data.
// grid1: the workgroups of the one-digit tile (tiles x split parts); the
// grid may be larger, for the multi-digit product's sake.
__global__ __launch_bounds__(512) void gemm_i8_auto256(GemmArgs g, GemmArgs gm, int grid1)
{
    constexpr int LDS1 = gemm_lds_bytes<256, 256, 64, 3, 1, PL_L1>();
    constexpr int LDSM = i8_multi_lds_bytes<4>();
    __shared__ __attribute__((aligned(1024))) char lds[LDS1 > LDSM ? LDS1 : LDSM];
    const int nd = limbs_needed(g.decide, g.gen);
    if (nd > 1)
        gemm_i8_multi_body<4>(gm, nd, lds);
    else if ((int)blockIdx.x < grid1)
        gemm_packed_body<true, 1, 256, 256, 64, 2, 4, 3, 1, PL_L1, 1, 1, false>(g, lds);
}

// ------------------------------------------------------- float64 probe --


// One workgroup per output tile of the cheap pass: probe_tile (mfma_tile.h)
// with 512 threads, records written for the correction launch.
constexpr int PROBE_THREADS = 512;

// fin (optional): a co-scheduled reduction's per-workgroup partials, which
// workgroup 0 adds (index order, fixed tree) into *fin.result = fin.init +
// sum once its tile is probed -- the reduction's last step rides in this
// launch instead of a launch of its own.
__global__ __launch_bounds__(PROBE_THREADS) void probe_f64(const char *__restrict__ pa, const char *__restrict__ pb,
                                                           const float *__restrict__ C, GemmShape sh, int bm, int bn,
                                                           int tiles_n, int64_t nkb, double tau2,
                                                           ProbeRecord *__restrict__ rec, RedFinal fin)
{
    __shared__ __attribute__((aligned(16))) ProbeLds L;
    const int64_t tile = blockIdx.x;
    probe_tile<PROBE_THREADS>(pa, pb, C, sh.m, sh.n, sh.k, sh.ldc, bm, bn, tile, (int)(tile / tiles_n),
                              (int)(tile % tiles_n), nkb, tau2, rec + tile, L);
    if (fin.result && blockIdx.x == 0) {
        __shared__ float w8[PROBE_THREADS / 64];
        float t = 0.0f;
        for (int k = threadIdx.x; k < fin.parts; k += PROBE_THREADS) t += __uint_as_float(fin.part[k]);
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o, 64);
        if ((threadIdx.x & 63) == 0) w8[threadIdx.x >> 6] = t;
        __syncthreads();
        if (threadIdx.x == 0) {
            float sum = 0.0f;
#pragma unroll
            for (int w = 0; w < PROBE_THREADS / 64; ++w) sum += w8[w];
            *fin.result = fin.init + sum;
        }
    }
}

// Tile configurations (BM x BN, wavefront grid, K-step bytes, ring depth):
//  T256     256 x 256, 8 waves (2x4), 32 B (bf16x3) / 64 B (int8), 3 stages:
//           one workgroup per CU, 144 / 96 KB LDS (bf16x3 with two planes:
//           96 KB); first-product look-ahead (bf16x3), full look-ahead
//           (one-digit int8).
//  T256x128 256 x 128, 4 waves (2x2), 32 B / 64 B, 2 stages: 72 / 48 KB LDS,
//           two workgroups per CU that do not share barriers.
//  T128     128 x 128, 4 waves (2x2), 32 B, 3 stages: 72 KB (bf16x3);
//           first-product look-ahead for bf16x3.
//  T64       64 x 64,  4 waves (2x2), 64 B, 2 stages.
// (Several int8 digits per operand: gemm_i8_multi's own 128 x 128 tile.)
//  T256W4   256 x 256, 4 waves (2x2, 128 x 128 each), 32 B / 64 B, 3
//           stages: a third less LDS read traffic per matrix instruction
//           than T256, one wavefront per SIMD, accumulators in AGPRs; for
//           bf16x3 a look-ahead loop (fragments of the next step read during
//           this step's matrix instructions).
template <bool INT8, int P, int BM, int BN, int KBK, int WGM, int WGN, int NS, int NPROD, uint64_t PL, int NACC,
          int LAM = 0, bool F32MM = false>
hipError_t launch_tile(GemmArgs g, hipStream_t s)
{
    g.tiles_m = (int)((g.M + BM - 1) / BM);
    g.tiles_n = (int)((g.N + BN - 1) / BN);
    if (NACC != 1 || g.accumulate || g.probe) g.ksplit = 1;  // split K: one accumulator set, C = result
    if (g.ksplit > 1) {
        g.kb_count = (g.nkb + g.ksplit - 1) / g.ksplit;
        if ((g.nkb + g.kb_count - 1) / g.kb_count != g.ksplit) return hipErrorInvalidValue;  // host policy bug
        hipError_t e = launch_zero_u32(g.tickets, g.tiles_m * g.tiles_n, s);
        if (e != hipSuccess) return e;
    }
    const dim3 grid((unsigned)(g.tiles_m * g.tiles_n * (g.ksplit > 1 ? g.ksplit : 1)));
    hipLaunchKernelGGL((gemm_packed<INT8, P, BM, BN, KBK, WGM, WGN, NS, NPROD, PL, NACC, LAM, F32MM>), grid,
                       dim3(WGM * WGN * 64), 0, s, g);
    return hipGetLastError();
}

// Tiled GEMM of one plane set: bf16x3 (P = 3) or one int8 digit (P = 1);
// several int8 digits run gemm_i8_multi.
template <bool INT8, int P, int NPROD, uint64_t PL, int NACC>
hipError_t run_gemm(int tile, const GemmArgs &g, hipStream_t s)
{
    static_assert(!INT8 || P == 1, "several int8 digits: gemm_i8_multi");
    constexpr int KS = P == 3 ? 32 : 64;  // K-step bytes of the big tiles
    switch (tile) {
    case GEMM_TILE_256:
        // Look-ahead: full for the one-digit int8 tile (two fragment sets of
        // 48 registers fit beside its 128 accumulator registers), first-product
        // only for bf16x3, whose three planes leave no room for a second full
        // set at two wavefronts per SIMD.  (A fourth stage, which fits for a
        // two-plane pass, measured 4 % slower: the loads are not the limit.)
        return launch_tile<INT8, P, 256, 256, KS, 2, 4, 3, NPROD, PL, NACC, INT8 ? 1 : 2>(g, s);
    case GEMM_TILE_256W4:
        // look-ahead for bf16x3 only: the int8 tile (two K sub-steps per
        // stage) would need more registers than a wavefront has
        return launch_tile<INT8, P, 256, 256, KS, 2, 2, 3, NPROD, PL, NACC, INT8 ? 0 : 1>(g, s);
    case GEMM_TILE_256x128:
        return launch_tile<INT8, P, 256, 128, KS, 2, 2, 2, NPROD, PL, NACC>(g, s);
    case GEMM_TILE_128:
        return launch_tile<INT8, P, 128, 128, 32, 2, 2, 3, NPROD, PL, NACC, INT8 ? 0 : 2>(g, s);
    default: break;
    }
    return launch_tile<INT8, P, 64, 64, 64, 2, 2, 2, NPROD, PL, NACC>(g, s);
}

// Multi-digit int8 GEMM: one 128 KB workgroup per CU, at most one per tile.
template <int P>
hipError_t launch_i8_multi(GemmArgs g, hipStream_t s)
{
    g.tiles_m = (int)((g.M + 127) / 128);
    g.tiles_n = (int)((g.N + 127) / 128);
    g.ksplit = 1;
    const int64_t tiles = (int64_t)g.tiles_m * g.tiles_n;
    const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>(tiles, device_cu_count()));
    hipLaunchKernelGGL(gemm_i8_multi<P>, dim3(grid), dim3(512), 0, s, g);
    return hipGetLastError();
}

// float32 matrix cores: one plane of 4-byte elements, 64-byte K steps (16
// elements: two fragment pairs, eight matrix instructions per 32 x 32 block),
// plain loop.  The float32 instructions are sixteen times slower per byte of
// operand than the bf16 ones, so the loads hide behind them without
// look-ahead.
hipError_t run_gemm_f32mm(int tile, const GemmArgs &g, hipStream_t s)
{
    constexpr uint64_t PL1 = prod(0, 0, 0, 0);
    switch (tile) {
    case GEMM_TILE_256:
    case GEMM_TILE_256W4:
        return launch_tile<false, 1, 256, 256, 64, 2, 4, 3, 1, PL1, 1, 0, true>(g, s);
    case GEMM_TILE_256x128:
        return launch_tile<false, 1, 256, 128, 64, 2, 2, 3, 1, PL1, 1, 0, true>(g, s);
    case GEMM_TILE_128:
        return launch_tile<false, 1, 128, 128, 64, 2, 2, 3, 1, PL1, 1, 0, true>(g, s);
    default: break;
    }
    return launch_tile<false, 1, 64, 64, 64, 2, 2, 2, 1, PL1, 1, 0, true>(g, s);
}

int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Pseudo-random operands for timing runs (not part of any result): a
// 32-bit integer hash of the element index, mapped to float32 in [-1, 1) or
// to int32 in [-16, 16].

__global__ void fill_hash(uint32_t *p, int64_t n, int as_int)
{
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const uint32_t h = hash32((uint32_t)i * 2654435761u + 12345u);
        if (as_int)
            p[i] = (uint32_t)((int32_t)(h % 33u) - 16);
        else
            p[i] = __float_as_uint((float)(h >> 8) * (1.0f / 8388608.0f) - 1.0f);
    }
}

__global__ void zero_u32(uint32_t *p, int n)
{
    for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0u;
}

unsigned pack_grid(int64_t units)
{
    int64_t blocks = cdiv(units * 128, 256);
    const int64_t cap = (int64_t)device_cu_count() * 16;
    if (blocks > cap) blocks = cap;
    return (unsigned)(blocks < 1 ? 1 : blocks);
}

}  // namespace

hipError_t launch_zero_u32(uint32_t *p, int n, hipStream_t s)
{
    hipLaunchKernelGGL(zero_u32, dim3(1), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

hipError_t launch_fill_hash(void *p, int64_t n, bool as_int, hipStream_t s)
{
    hipLaunchKernelGGL(fill_hash, dim3((unsigned)std::min<int64_t>(4096, cdiv(n, 256))), dim3(256), 0, s,
                       static_cast<uint32_t *>(p), n, as_int ? 1 : 0);
    return hipGetLastError();
}

// The largest square tile that still gives every CU a workgroup; the
// smallest tile when none does.
int default_tile(int64_t m, int64_t n)
{
    const int64_t cus = device_cu_count();
    if (cdiv(m, 256) * cdiv(n, 256) >= cus) return GEMM_TILE_256;
    if (cdiv(m, 128) * cdiv(n, 128) >= cus) return GEMM_TILE_128;
    return GEMM_TILE_64;
}

size_t packed_bytes(int64_t rows, int64_t k_elems, int elem_bytes, int planes)
{
    const int64_t nrb = cdiv(rows, 32);
    const int64_t nkb = cdiv(k_elems * elem_bytes, 64);
    return (size_t)(nrb * nkb * planes * PLANE_BYTES);
}

hipError_t launch_pack_bf16x3(const float *x, int64_t rows, int64_t k, int64_t ld, bool trans, void *out,
                              hipStream_t s)
{
    const int64_t nrb = cdiv(rows, 32), nkb = cdiv(k, 32);
    if (nrb * nkb == 0) return hipSuccess;
    const unsigned grid = pack_grid(nrb * nkb);
    tmark("pack_bf16x3", s, true);
    if (trans)
        hipLaunchKernelGGL(pack_bf16x3_t, dim3((unsigned)(cdiv(rows, TP_COLS) * BF_SPLIT * nkb)), dim3(256), 0, s, x,
                           rows, k, ld, static_cast<char *>(out), nrb, nkb, (int)cdiv(rows, TP_COLS));
    else
        hipLaunchKernelGGL(pack_bf16x3<false>, dim3(grid), dim3(256), 0, s, x, rows, k, ld, static_cast<char *>(out),
                           nrb, nkb);
    tmark("pack_bf16x3", s, false);
    return hipGetLastError();
}

hipError_t launch_pack_i8(const int32_t *x, int64_t rows, int64_t k, int64_t ld, bool trans, int planes, void *out,
                          hipStream_t s)
{
    const int64_t nrb = cdiv(rows, 32), nkb = cdiv(k, 64);
    if (nrb * nkb == 0) return hipSuccess;
    const unsigned grid = pack_grid(nrb * nkb);
    tmark("pack_i8", s, true);
    if (trans)
        hipLaunchKernelGGL(pack_i8_t, dim3((unsigned)(cdiv(rows, TP_COLS) * I8_SPLIT * nkb)), dim3(256), 0, s, x, rows,
                           k, ld, static_cast<char *>(out), nrb, nkb, planes, (int)cdiv(rows, TP_COLS));
    else
        hipLaunchKernelGGL(pack_i8<false>, dim3(grid), dim3(256), 0, s, x, rows, k, ld, static_cast<char *>(out), nrb,
                           nkb, planes);
    tmark("pack_i8", s, false);
    return hipGetLastError();
}

hipError_t launch_pack_bf16x3_pair(const float *a, int64_t m, int64_t lda, const float *b, int64_t n, int64_t ldb,
                                   int64_t k, void *pa, void *pb, hipStream_t s)
{
    const int64_t nkb = cdiv(k, 32), ua = cdiv(m, 32) * nkb;
    const int64_t ga = ua > 0 ? pack_grid(ua) : 0, gbx = cdiv(n, TP_COLS), gb = gbx * BF_SPLIT * nkb;
    if (ga + gb == 0) return hipSuccess;
    tmark("pack_bf16x3", s, true);
    hipLaunchKernelGGL(pack_bf16x3_pair, dim3((unsigned)(ga + gb)), dim3(256), 0, s, a, m, lda,
                       static_cast<char *>(pa), b, n, ldb, static_cast<char *>(pb), k, (int)ga, (int)std::max<int64_t>(gbx, 1));
    tmark("pack_bf16x3", s, false);
    return hipGetLastError();
}

hipError_t launch_pack_i8_pair(const int32_t *a, int64_t m, int64_t lda, const int32_t *b, int64_t n, int64_t ldb,
                               int64_t k, int planes, void *pa, void *pb, uint64_t *maxabs, hipStream_t s,
                               const uint64_t *decide, uint32_t stamp)
{
    const int64_t nkb = cdiv(k, 64), ua = cdiv(m, 32) * nkb;
    int64_t ga = ua > 0 ? pack_grid(ua) : 0;
    const int64_t gbx = cdiv(n, TP_COLS), gb = gbx * I8_SPLIT * nkb;
    int64_t gbl = gb;  // workgroups for B's column tiles
    if (decide) {
        // the multi-digit pass usually exits at once: a grid of a few
        // workgroups per CU, each looping, keeps that exit cheap
        const int64_t cap = (int64_t)device_cu_count() * 2;
        ga = std::min<int64_t>(ga, cap);
        gbl = std::min<int64_t>(gbl, cap);
    }
    const bool one = !decide && planes == 1;
    if (one && ua > 0) ga = std::min<int64_t>(cdiv(ua * 8, 4 * 4), (int64_t)device_cu_count() * 8);  // 4 items per wavefront
    if (ga + gbl == 0) return hipSuccess;
    tmark("pack_i8", s, true);
    if (one)
        hipLaunchKernelGGL(pack_i8_pair<true>, dim3((unsigned)(ga + gbl)), dim3(256), 0, s, a, m, lda,
                           static_cast<char *>(pa), b, n, ldb, static_cast<char *>(pb), k, 1, 1, (int)ga,
                           (int)std::max<int64_t>(gbx, 1), gb, maxabs, decide, stamp);
    else
        hipLaunchKernelGGL(pack_i8_pair<false>, dim3((unsigned)(ga + gbl)), dim3(256), 0, s, a, m, lda,
                           static_cast<char *>(pa), b, n, ldb, static_cast<char *>(pb), k, planes, decide ? 4 : planes,
                           (int)ga, (int)std::max<int64_t>(gbx, 1), gb, maxabs, decide, stamp);
    tmark("pack_i8", s, false);
    return hipGetLastError();
}

hipError_t launch_pack_f32(const float *x, int64_t rows, int64_t k, int64_t ld, bool trans, void *out, hipStream_t s)
{
    const int64_t nrb = cdiv(rows, 32), nkb = cdiv(k, 16);
    if (nrb * nkb == 0) return hipSuccess;
    tmark("pack_f32", s, true);
    if (trans)
        hipLaunchKernelGGL(pack_f32_t, dim3((unsigned)(cdiv(rows, TP_COLS) * nkb)), dim3(256), 0, s, x, rows, k, ld,
                           static_cast<char *>(out), nrb, nkb, (int)cdiv(rows, TP_COLS));
    else
        hipLaunchKernelGGL(pack_f32_a, dim3(pack_grid(nrb * nkb)), dim3(256), 0, s, x, rows, k, ld,
                           static_cast<char *>(out), nrb, nkb);
    tmark("pack_f32", s, false);
    return hipGetLastError();
}

hipError_t launch_pack_f32_pair(const float *a, int64_t m, int64_t lda, const float *b, int64_t n, int64_t ldb,
                                int64_t k, void *pa, void *pb, hipStream_t s)
{
    const int64_t nkb = cdiv(k, 16), ua = cdiv(m, 32) * nkb;
    const int64_t ga = ua > 0 ? pack_grid(ua) : 0, gbx = cdiv(n, TP_COLS), gb = gbx * nkb;
    if (ga + gb == 0) return hipSuccess;
    tmark("pack_f32", s, true);
    hipLaunchKernelGGL(pack_f32_pair, dim3((unsigned)(ga + gb)), dim3(256), 0, s, a, m, lda, static_cast<char *>(pa),
                       b, n, ldb, static_cast<char *>(pb), k, (int)ga, (int)std::max<int64_t>(gbx, 1));
    tmark("pack_f32", s, false);
    return hipGetLastError();
}

void tile_dims(int tile, int64_t m, int64_t n, int &bm, int &bn)
{
    const int t = tile ? tile : default_tile(m, n);
    bm = (t == GEMM_TILE_256 || t == GEMM_TILE_256W4 || t == GEMM_TILE_256x128) ? 256 : t == GEMM_TILE_128 ? 128 : 64;
    bn = (t == GEMM_TILE_256 || t == GEMM_TILE_256W4) ? 256 : t == GEMM_TILE_256x128 ? 128 : bm;
}

hipError_t launch_probe_f64(const void *pa, const void *pb, const float *c, const GemmShape &sh, int tile, double tau,
                            ProbeRecord *rec, hipStream_t s, const RedFinal &fin)
{
    int bm, bn;
    tile_dims(tile, sh.m, sh.n, bm, bn);
    const int tiles_m = (int)cdiv(sh.m, bm), tiles_n = (int)cdiv(sh.n, bn);
    if (tiles_m * tiles_n == 0) return hipSuccess;
    tmark("probe_f64", s, true);
    hipLaunchKernelGGL(probe_f64, dim3((unsigned)(tiles_m * tiles_n)), dim3(PROBE_THREADS), 0, s, static_cast<const char *>(pa),
                       static_cast<const char *>(pb), c, sh, bm, bn, tiles_n, cdiv(sh.k * 2, 64), tau * tau, rec, fin);
    tmark("probe_f64", s, false);
    return hipGetLastError();
}

int split_k_parts(int tile, int64_t m, int64_t n, int64_t nkb)
{
    int bm, bn;
    tile_dims(tile, m, n, bm, bn);
    const int64_t T = cdiv(m, bm) * cdiv(n, bn);
    const int64_t cus = device_cu_count();
    if (T <= 0 || 2 * T > cus) return 1;
    // parts to fill the workgroup slots: two per CU for the 128 x 128 tile
    // (four wavefronts; two workgroups fit a CU's registers and LDS, and
    // their barriers do not wait for each other: the three-product pass of
    // 512 x 4096 x 4096 runs 65 us in 4 parts against 79 us in 2), one for
    // the others
    const int64_t per_cu = tile == GEMM_TILE_128 ? 2 : 1;
    int64_t parts = std::min<int64_t>(dev::KSPLIT_MAX, per_cu * cus / T);
    parts = std::min<int64_t>(parts, nkb / 8);  // at least eight 64-byte K units per part
    if (parts < 2) return 1;
    return (int)cdiv(nkb, cdiv(nkb, parts));  // every part non-empty
}

size_t split_k_bytes(int tile, int64_t m, int64_t n, int parts)
{
    if (parts <= 1) return 0;
    int bm, bn;
    tile_dims(tile, m, n, bm, bn);
    const int64_t T = cdiv(m, bm) * cdiv(n, bn);
    return (size_t)(256 + 4 * T + 255) / 256 * 256 + (size_t)parts * T * bm * bn * 4;
}

int probe_tiles(int tile, int64_t m, int64_t n)
{
    int bm, bn;
    tile_dims(tile, m, n, bm, bn);
    return (int)(cdiv(m, bm) * cdiv(n, bn));
}

void set_split(GemmArgs &g, const SplitK &sk, int64_t tiles_bytes_offset)
{
    g.ksplit = sk.parts > 1 ? std::min(sk.parts, KSPLIT_MAX) : 1;  // the host plans at most KSPLIT_MAX
    if (g.ksplit > 1) {
        g.tickets = static_cast<uint32_t *>(sk.work);
        g.partials = static_cast<char *>(sk.work) + tiles_bytes_offset;
    }
}

int log2i(int v)
{
    int l = 0;
    while ((1 << l) < v) ++l;
    return l;
}

hipError_t launch_gemm_bf16x3(const void *pa, const void *pb, float *c, const GemmShape &sh, int products,
                              bool accumulate, int tile, hipStream_t s, const ProbeRecord *probe, const SplitK &sk,
                              int probe_tile)
{
    if (sh.m <= 0 || sh.n <= 0) return hipSuccess;
    GemmArgs g{};
    g.A = static_cast<const char *>(pa);
    g.B = static_cast<const char *>(pb);
    g.C = c;
    g.M = sh.m;
    g.N = sh.n;
    g.ldc = sh.ldc;
    g.nkb = cdiv(sh.k * 2, 64);
    g.nrb_a = cdiv(sh.m, 32);
    g.nrb_b = cdiv(sh.n, 32);
    g.accumulate = accumulate ? 1 : 0;
    g.probe = probe;
    const int t = tile ? tile : default_tile(sh.m, sh.n);
    if (probe) {
        // the records' tiles (probe_tile) contain whole tiles of this launch
        int bm, bn, pbm, pbn;
        tile_dims(t, sh.m, sh.n, bm, bn);
        tile_dims(probe_tile ? probe_tile : t, sh.m, sh.n, pbm, pbn);
        if (pbm % bm || pbn % bn) return hipErrorInvalidValue;
        g.probe_shm = log2i(pbm / bm);
        g.probe_shn = log2i(pbn / bn);
        g.probe_tiles_n = (int)cdiv(sh.n, pbn);
    }
    if (sk.parts > 1) {
        int bm, bn;
        tile_dims(t, sh.m, sh.n, bm, bn);
        set_split(g, sk, (256 + 4 * cdiv(sh.m, bm) * cdiv(sh.n, bn) + 255) / 256 * 256);
    }
    hipError_t e;
    const char *tname = accumulate ? "gemm_bf16x3_corr" : "gemm_bf16x3";
    tmark(tname, s, true);
    if (products == 6)
        e = run_gemm<false, 3, 6, PL_FULL6, 1>(t, g, s);
    else if (products == 5)
        e = run_gemm<false, 3, 5, PL_FIVE, 1>(t, g, s);
    else if (products == 3)
        e = run_gemm<false, 3, 3, PL_CHEAP3, 1>(t, g, s);
    else if (products == -3)
        e = run_gemm<false, 3, 3, PL_CORR3, 1>(t, g, s);
    else
        e = hipErrorInvalidValue;
    tmark(tname, s, false);
    return e;
}

hipError_t launch_gemm_bf16x3_red(const void *pa, const void *pb, float *c, const GemmShape &sh, const float *x,
                                  int64_t n, uint32_t *part, hipStream_t s)
{
    if (sh.m <= 0 || sh.n <= 0) return hipErrorInvalidValue;  // no workgroup to carry the sum
    if (((uintptr_t)x & 15u) != 0) return hipErrorInvalidValue;
    GemmArgs g{};
    g.A = static_cast<const char *>(pa);
    g.B = static_cast<const char *>(pb);
    g.C = c;
    g.M = sh.m;
    g.N = sh.n;
    g.ldc = sh.ldc;
    g.nkb = cdiv(sh.k * 2, 64);
    g.nrb_a = cdiv(sh.m, 32);
    g.nrb_b = cdiv(sh.n, 32);
    g.tiles_m = (int)cdiv(sh.m, 256);
    g.tiles_n = (int)cdiv(sh.n, 256);
    g.ksplit = 1;
    const int64_t grid = (int64_t)g.tiles_m * g.tiles_n;
    g.red_x = x;
    g.red_nvec = n / 4;
    g.red_ntail = (int)(n % 4);
    g.red_per = cdiv(g.red_nvec, grid);
    g.red_part = part;
    tmark("gemm_bf16x3", s, true);
    hipLaunchKernelGGL((gemm_packed<false, 3, 256, 256, 32, 2, 4, 3, 3, PL_CHEAP3, 1, 2, false, true>), dim3((unsigned)grid),
                       dim3(512), 0, s, g);
    tmark("gemm_bf16x3", s, false);
    return hipGetLastError();
}

int red_fused_parts(int64_t m, int64_t n) { return (int)(cdiv(m, 256) * cdiv(n, 256)); }

int64_t red_fused_capacity(int64_t m, int64_t n, int64_t k)
{
    // K-steps of the 256 x 256 three-product pass (16 elements each) x 512
    // threads x RED_RV vectors of 4 floats, per workgroup
    const int64_t nsteps = cdiv(k * 2, 64) * 2;
    return (int64_t)red_fused_parts(m, n) * nsteps * 512 * RED_RV * 4;
}

hipError_t launch_gemm_f32mm(const void *pa, const void *pb, float *c, const GemmShape &sh, int tile, hipStream_t s,
                              const SplitK &sk)
{
    if (sh.m <= 0 || sh.n <= 0) return hipSuccess;
    GemmArgs g{};
    g.A = static_cast<const char *>(pa);
    g.B = static_cast<const char *>(pb);
    g.C = c;
    g.M = sh.m;
    g.N = sh.n;
    g.ldc = sh.ldc;
    g.nkb = cdiv(sh.k * 4, 64);
    g.nrb_a = cdiv(sh.m, 32);
    g.nrb_b = cdiv(sh.n, 32);
    const int t = tile ? tile : default_tile(sh.m, sh.n);
    if (sk.parts > 1) {
        int bm, bn;
        tile_dims(t, sh.m, sh.n, bm, bn);
        set_split(g, sk, (256 + 4 * cdiv(sh.m, bm) * cdiv(sh.n, bn) + 255) / 256 * 256);
    }
    tmark("gemm_f32mm", s, true);
    const hipError_t e = run_gemm_f32mm(t, g, s);
    tmark("gemm_f32mm", s, false);
    return e;
}

hipError_t launch_gemm_i8(const void *pa, const void *pb, int32_t *c, const GemmShape &sh, int limbs, int tile,
                          hipStream_t s, const uint64_t *decide, uint32_t stamp, const SplitK &sk)
{
    if (sh.m <= 0 || sh.n <= 0) return hipSuccess;
    GemmArgs g{};
    g.A = static_cast<const char *>(pa);
    g.B = static_cast<const char *>(pb);
    g.C = c;
    g.M = sh.m;
    g.N = sh.n;
    g.ldc = sh.ldc;
    g.nkb = cdiv(sh.k, 64);
    g.nrb_a = cdiv(sh.m, 32);
    g.nrb_b = cdiv(sh.n, 32);
    g.decide = decide;
    g.gen = stamp;
    g.expect = limbs;
    const int t = tile ? tile : default_tile(sh.m, sh.n);
    if (sk.parts > 1 && limbs == 1) {
        int bm, bn;
        tile_dims(t, sh.m, sh.n, bm, bn);
        set_split(g, sk, (256 + 4 * cdiv(sh.m, bm) * cdiv(sh.n, bn) + 255) / 256 * 256);
    }
    hipError_t e;
    tmark("gemm_i8", s, true);
    switch (limbs) {
    case 1: e = run_gemm<true, 1, 1, PL_L1, 1>(t, g, s); break;
    case 2: e = launch_i8_multi<2>(g, s); break;
    case 3: e = launch_i8_multi<3>(g, s); break;
    case 4: e = launch_i8_multi<4>(g, s); break;
    default: e = hipErrorInvalidValue;
    }
    tmark("gemm_i8", s, false);
    return e;
}

hipError_t launch_gemm_i8_auto(const void *pa1, const void *pb1, const void *pa4, const void *pb4, int32_t *c,
                               const GemmShape &sh, int tile, hipStream_t s, const uint64_t *maxabs, uint32_t stamp,
                               const SplitK &sk)
{
    if (sh.m <= 0 || sh.n <= 0) return hipSuccess;
    const int t = tile ? tile : default_tile(sh.m, sh.n);
    if (t != GEMM_TILE_256) {  // the other one-digit tiles: two launches
        hipError_t e = launch_gemm_i8(pa1, pb1, c, sh, 1, t, s, maxabs, stamp, sk);
        if (e == hipSuccess) e = launch_gemm_i8(pa4, pb4, c, sh, 4, 0, s, maxabs, stamp);
        return e;
    }
    GemmArgs g{};
    g.A = static_cast<const char *>(pa1);
    g.B = static_cast<const char *>(pb1);
    g.C = c;
    g.M = sh.m;
    g.N = sh.n;
    g.ldc = sh.ldc;
    g.nkb = cdiv(sh.k, 64);
    g.nrb_a = cdiv(sh.m, 32);
    g.nrb_b = cdiv(sh.n, 32);
    g.decide = maxabs;
    g.gen = stamp;
    g.expect = 1;
    g.tiles_m = (int)cdiv(sh.m, 256);
    g.tiles_n = (int)cdiv(sh.n, 256);
    if (sk.parts > 1) set_split(g, sk, (256 + 4 * (int64_t)g.tiles_m * g.tiles_n + 255) / 256 * 256);
    if (g.ksplit > 1) {
        g.kb_count = (g.nkb + g.ksplit - 1) / g.ksplit;
        if ((g.nkb + g.kb_count - 1) / g.kb_count != g.ksplit) return hipErrorInvalidValue;  // host policy bug
        hipError_t e = launch_zero_u32(g.tickets, g.tiles_m * g.tiles_n, s);
        if (e != hipSuccess) return e;
    }
    GemmArgs gm = g;
    gm.A = static_cast<const char *>(pa4);
    gm.B = static_cast<const char *>(pb4);
    gm.expect = 4;
    gm.ksplit = 1;
    gm.tiles_m = (int)cdiv(sh.m, I8M_BM);
    gm.tiles_n = (int)cdiv(sh.n, I8M_BN);
    const int64_t grid1 = (int64_t)g.tiles_m * g.tiles_n * (g.ksplit > 1 ? g.ksplit : 1);
    const int64_t gridm = std::min<int64_t>((int64_t)gm.tiles_m * gm.tiles_n, device_cu_count());
    tmark("gemm_i8", s, true);
    hipLaunchKernelGGL(gemm_i8_auto256, dim3((unsigned)std::max(grid1, gridm)), dim3(512), 0, s, g, gm, (int)grid1);
    tmark("gemm_i8", s, false);
    return hipGetLastError();
}

}  // namespace accx
