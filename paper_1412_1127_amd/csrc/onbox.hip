// Measurement kernels: what this GPU reaches with nothing but the resource
// a hot-path kernel is bound by, so that a kernel's fraction of roofline can
// be stated against the measured ceiling as well as against the datasheet
// (the Methodology section times kernels with the vendor profiler and
// reports harmonic means of repeated runs; these give the ceilings such
// timings are compared with).
//  - onbox_mfma: matrix instructions only.  Each wavefront keeps NCH
//    independent 32 x 32 accumulators and issues one matrix instruction per
//    accumulator per round, from operands already in registers; no memory
//    traffic inside the loop.  Two wavefronts per SIMD, as the tiled GEMM
//    runs.
//  - onbox_read: a read-only stream of a buffer, 16-byte non-temporal loads,
//    eight in flight per thread, three workgroups of 256 threads per CU, each
//    folding what it read into one word (so that no load can be dropped).
// Results go to one device word (onbox_sink); nothing is allocated.
#include <hip/hip_runtime.h>

#include "kernels.h"
#include "mfma_tile.h"

namespace accx {

// Where the measurement kernels leave their (practically never written)
// result: external linkage, so that the compiler must keep the work.
__device__ uint32_t onbox_sink;

namespace {

using namespace dev;

constexpr int NCH = 8;             // independent accumulators per wavefront
constexpr int MFMA_THREADS = 512;  // eight wavefronts: two per SIMD

template <bool I8>
__global__ __launch_bounds__(MFMA_THREADS) void onbox_mfma(int64_t rounds, uint32_t seed)
{
    using M = Mma<I8>;
    typename M::Frag a, b;
    const uint32_t s = seed ^ (threadIdx.x * 2654435761u);
    if constexpr (I8) {
        a = i32x4{(int)s, (int)(s >> 3), (int)(s >> 5), (int)(s >> 7)};
        b = i32x4{(int)(s >> 1), (int)(s >> 2), (int)(s >> 4), (int)(s >> 6)};
    } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            a[e] = (__bf16)(float)((s >> e) & 7u);
            b[e] = (__bf16)(float)((s >> (e + 8)) & 7u);
        }
    }
    typename M::Acc c[NCH];
#pragma unroll
    for (int j = 0; j < NCH; ++j) c[j] = (typename M::Acc)0;
    for (int64_t r = 0; r < rounds; ++r) {
#pragma unroll
        for (int j = 0; j < NCH; ++j) c[j] = M::run(a, b, c[j]);
    }
    uint32_t fold = 0;
#pragma unroll
    for (int j = 0; j < NCH; ++j)
#pragma unroll
        for (int e = 0; e < 16; ++e) fold ^= word_of(c[j][e]);
    if (fold == seed) onbox_sink = fold;  // practically never: keeps the work
}

constexpr int RD_THREADS = 256;
constexpr int RD_UNROLL = 8;

__global__ __launch_bounds__(RD_THREADS) void onbox_read(const u32x4_t *__restrict__ x, int64_t nvec)
{
    uint32_t fold = 0;
    const int64_t stride = (int64_t)gridDim.x * RD_THREADS;
    int64_t i = (int64_t)blockIdx.x * RD_THREADS + threadIdx.x;
    for (; i + (RD_UNROLL - 1) * stride < nvec; i += RD_UNROLL * stride) {
        u32x4_t v[RD_UNROLL];
#pragma unroll
        for (int u = 0; u < RD_UNROLL; ++u) v[u] = __builtin_nontemporal_load(x + i + u * stride);
#pragma unroll
        for (int u = 0; u < RD_UNROLL; ++u) fold += (v[u].x ^ v[u].y) + (v[u].z ^ v[u].w);
    }
    for (; i < nvec; i += stride) {
        const u32x4_t v = __builtin_nontemporal_load(x + i);
        fold += (v.x ^ v.y) + (v.z ^ v.w);
    }
    if (fold == 0x9e3779b9u) onbox_sink = fold;  // practically never: keeps the loads
}

}  // namespace

hipError_t launch_onbox_mfma(int kind, int64_t rounds, double *ops, hipStream_t s)
{
    const unsigned grid = (unsigned)device_cu_count();
    const double per_inst = kind == 0 ? 32.0 * 32 * 16 * 2 : 32.0 * 32 * 32 * 2;
    *ops = (double)grid * (MFMA_THREADS / 64) * (double)rounds * NCH * per_inst;
    if (kind == 0)
        hipLaunchKernelGGL(onbox_mfma<false>, dim3(grid), dim3(MFMA_THREADS), 0, s, rounds, 0x1234567u);
    else
        hipLaunchKernelGGL(onbox_mfma<true>, dim3(grid), dim3(MFMA_THREADS), 0, s, rounds, 0x1234567u);
    return hipGetLastError();
}

hipError_t launch_onbox_read(const void *x, int64_t bytes, hipStream_t s)
{
    const int64_t nvec = bytes / 16;
    const unsigned grid = (unsigned)device_cu_count() * 3;
    hipLaunchKernelGGL(onbox_read, dim3(grid), dim3(RD_THREADS), 0, s, static_cast<const u32x4_t *>(x), nvec);
    return hipGetLastError();
}

}  // namespace accx
